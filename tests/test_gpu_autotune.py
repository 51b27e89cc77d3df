"""Autotuning of the single-solve kernel: the recorded choice changes speed
only (every configuration gives the oracle's result), overrides still win,
and clearing returns to the automatic choice."""
import json
import os
import sys

import numpy as np
import pytest

from paper_1511_06441_amd import inputs as gen

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture
def solver(torch):
    from paper_1511_06441_amd import csp
    s = csp.Solver(0)
    yield s
    s.close()


def _solve(solver, torch, di, N):
    lab = torch.zeros(N, dtype=torch.int32, device="cuda")
    res, cnt = solver.solve(di, labels=lab)
    return res, cnt, lab.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("case", [(2, 64, 1, 5, 5, 200), (2, 300, 2, 9, 9, 2000), (3, 33, 3, 10, 10, 300),
                                  (3, 48, 4, 10, 10, 400), (4, 9, 5, 8, 8, 80)],
                         ids=lambda c: f"d{c[0]}n{c[1]}")
def test_autotuned_solve_equals_oracle(solver, torch, case):
    from oracle import oracle as O
    from paper_1511_06441_amd import csp
    d, n, seed, K1, K2, M = case
    inst = gen.opposite_faces(d, n, seed, K1, K2, M)
    ref = O.solve_instance(inst)
    di = csp.to_device(inst)
    blocks, path, ms = solver.autotune(di)
    _say("case", inst.name, "blocks", blocks, "path", path, "ms %.3f" % ms)
    assert blocks >= 1 and path in (0, 1, 2, 3) and ms > 0
    res, cnt, lab = _solve(solver, torch, di, inst.N)
    assert res.tuple() == ref.tuple() and cnt.asdict() == ref.counters
    assert np.array_equal(lab, ref.labels)


def test_autotune_cube128_and_overrides(solver, torch):
    from paper_1511_06441_amd import csp
    rec = json.load(open(os.path.join(GOLDEN, "cube128_s11_M700.json")))
    inst = gen.cube128(11, 700)
    di = csp.to_device(inst)
    blocks, path, ms = solver.autotune(di)
    _say("cube128 autotune: blocks", blocks, "path", path, "ms %.3f" % ms)
    res, cnt, _ = _solve(solver, torch, di, inst.N)
    assert res.tuple() == (rec["T"], rec["X"], rec["x"], rec["Y"], rec["F2"])
    assert cnt.asdict() == rec["counters"]
    # an explicit override wins over the recorded choice and gives the same answer
    csp.csp_set_blocks(solver.ctx, 64)
    csp.csp_set_path(solver.ctx, 1)
    try:
        r2, c2, _ = _solve(solver, torch, di, inst.N)
        assert csp.csp_last_path(solver.ctx) == 1
    finally:
        csp.csp_set_blocks(solver.ctx, 0)
        csp.csp_set_path(solver.ctx, 0)
    assert r2.tuple() == res.tuple() and c2.asdict() == cnt.asdict()
    # the choice applies to other M on the same lattice too
    inst4 = gen.cube128(11, 400)
    rec4 = json.load(open(os.path.join(GOLDEN, "cube128_s11_M400.json")))
    r4, c4, _ = _solve(solver, torch, csp.to_device(inst4), inst4.N)
    assert r4.tuple() == (rec4["T"], rec4["X"], rec4["x"], rec4["Y"], rec4["F2"])
    assert c4.asdict() == rec4["counters"]
    csp.csp_autotune_clear(solver.ctx)
    r5, c5, _ = _solve(solver, torch, di, inst.N)
    assert r5.tuple() == res.tuple() and c5.asdict() == cnt.asdict()


def test_autotune_rejects_bad_input(solver, torch):
    from paper_1511_06441_amd import csp
    inst = gen.square64(1)
    di = csp.to_device(inst)
    with pytest.raises(csp.CspError) as e:
        csp.csp_autotune(solver.ctx, 2, 64, di.f1, di.f2, di.A, di.B, 0)
    assert e.value.code == csp.CSP_EINVAL
    bad = gen.square64(1)
    bad.B = bad.A.copy()
    with pytest.raises(csp.CspError) as e:
        solver.autotune(csp.to_device(bad))
    assert e.value.code == csp.CSP_EINVAL
    # nothing was recorded by the failed calls: the solve still runs as before
    res, cnt, _ = _solve(solver, torch, di, inst.N)
    assert res.T == 142


@pytest.mark.parametrize("target", [8192, 65536])
def test_batch_target_keeps_results(solver, torch, target):
    """Gang sizes from an explicit target give the oracle's results."""
    from oracle import oracle as O
    from paper_1511_06441_amd import csp
    insts = [gen.mixed_instance(43, j, lo2=(32, 400), lo3=(12, 48)) for j in range(24)]
    dev = [csp.to_device(i) for i in insts]
    csp.csp_set_batch_target(solver.ctx, target)
    try:
        res, cnt = csp.csp_solve_batch(solver.ctx, dev)
    finally:
        csp.csp_set_batch_target(solver.ctx, 0)
    _say("batch target", target, "kernel ms %.3f" % csp.csp_last_kernel_ms(solver.ctx))
    for inst, r, c in zip(insts, res, cnt):
        ref = O.solve_instance(inst, want_labels=False)
        assert r.tuple() == ref.tuple() and c.asdict() == ref.counters, inst.name


def test_autotune_batch(solver, torch):
    from paper_1511_06441_amd import csp
    insts = [gen.mixed_instance(44, j, lo2=(32, 400), lo3=(12, 48)) for j in range(32)]
    dev = [csp.to_device(i) for i in insts]
    base, bcnt = csp.csp_solve_batch(solver.ctx, dev)
    tgt, ms = csp.csp_autotune_batch(solver.ctx, dev)
    _say("batch autotune: vertices per workgroup", tgt, "ms %.3f" % ms)
    assert tgt in (0, 65536, 32768, 16384, 8192) and ms > 0
    res, cnt = csp.csp_solve_batch(solver.ctx, dev)
    assert [r.tuple() for r in res] == [r.tuple() for r in base]
    assert [c.asdict() for c in cnt] == [c.asdict() for c in bcnt]
    csp.csp_autotune_clear(solver.ctx)
    with pytest.raises(csp.CspError):
        csp.csp_set_batch_target(solver.ctx, -1)
