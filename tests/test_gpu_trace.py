"""Per-cycle trace (t, delivered, |I_t|, sent): identical to the oracle's
trace row by row, and consistent with the counters at full size."""
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


@pytest.fixture(scope="module")
def solver(torch):
    from paper_1511_06441_amd import csp
    s = csp.Solver(0)
    yield s
    s.close()


def _gpu_trace(solver, torch, inst, cap, blocks=0, path=0, dense=-1):
    from paper_1511_06441_amd import csp
    di = csp.to_device(inst)
    tr = torch.full((cap, 4), -7, dtype=torch.int64, device="cuda")
    csp.csp_set_trace(solver.ctx, tr)
    csp.csp_set_blocks(solver.ctx, blocks)
    csp.csp_set_path(solver.ctx, path)
    csp.csp_set_dense_threshold(solver.ctx, dense)
    try:
        res, cnt = solver.solve(di)
        rows = csp.csp_last_trace_rows(solver.ctx)
    finally:
        csp.csp_set_trace(solver.ctx, None)
        csp.csp_set_blocks(solver.ctx, 0)
        csp.csp_set_path(solver.ctx, 0)
        csp.csp_set_dense_threshold(solver.ctx, -1)
    torch.cuda.synchronize()
    return res, cnt, rows, tr.cpu().numpy()


CASES = [lambda: gen.square64(1), lambda: gen.square64(2),
         lambda: gen.opposite_faces(3, 20, 5, 8, 8, 140),
         lambda: gen.opposite_faces(2, 150, 6, 20, 20, 900),
         lambda: gen.opposite_faces(2, 40, 7, 5, 5, 30),          # no path: M below every path weight
         lambda: gen.cube_boundary_to_center(24, 8, K=30, M=2000)]


@pytest.mark.parametrize("k", range(len(CASES)))
@pytest.mark.parametrize("blocks,path", [(0, 0), (8, 1), (16, 3)])
def test_trace_equals_oracle(solver, torch, k, blocks, path):
    from oracle import oracle as O
    inst = CASES[k]()
    _say("case", inst.name, "blocks", blocks, "path", path)
    ref = O.solve_instance(inst, want_labels=False, trace_cap=1 << 16)
    res, cnt, rows, tr = _gpu_trace(solver, torch, inst, 1 << 16, blocks, path)
    assert res.tuple() == ref.tuple() and cnt.asdict() == ref.counters
    assert rows == len(ref.trace) == cnt.C
    assert np.array_equal(tr[:rows], ref.trace), inst.name
    assert (tr[rows:] == -7).all()


def test_trace_capacity_counts_beyond(solver, torch):
    from oracle import oracle as O
    inst = gen.square64(3)
    ref = O.solve_instance(inst, want_labels=False, trace_cap=1 << 16)
    cap = 10
    res, cnt, rows, tr = _gpu_trace(solver, torch, inst, cap)
    assert rows == len(ref.trace) > cap
    assert np.array_equal(tr[:cap], ref.trace[:cap])


def test_trace_global_label_kernel_refused(solver, torch):
    from paper_1511_06441_amd import csp
    with pytest.raises(csp.CspError):
        _gpu_trace(solver, torch, gen.square64(1), 64, path=2)


@pytest.mark.parametrize("name", ["cube256_s21", "cube128_s11_M700", "paper125_s61"])
def test_trace_at_scale_matches_counters(solver, torch, name):
    """Active set and deliveries per cycle at full size: the rows add up to
    the oracle's stored counters."""
    with open(os.path.join(GOLDEN, name + ".json")) as fh:
        rec = json.load(fh)
    if name.startswith("cube256"):
        inst = gen.cube256(rec["meta"]["seed"], rec["M"])
    elif name.startswith("cube128"):
        inst = gen.cube128(rec["meta"]["seed"], rec["M"])
    else:
        inst = gen.cube_boundary_to_center(rec["n"], rec["meta"]["seed"], K=rec["meta"]["K1"], M=rec["M"])
    _say("case", name)
    res, cnt, rows, tr = _gpu_trace(solver, torch, inst, 1 << 15)
    c = rec["counters"]
    tr = tr[:rows]
    nA = int(inst.A.sum())
    assert res.tuple() == (rec["T"], rec["X"], rec["x"], rec["Y"], rec["F2"])
    assert rows == c["C"]
    assert int(tr[:, 1].sum()) == c["R"]
    assert int(tr[:, 2].sum()) == c["U"] - nA
    assert int(tr[:, 2].max()) == c["I"]
    assert tr[-1, 0] == rec["T"] and tr[-1, 3] == 0
    assert (np.diff(tr[:, 0]) > 0).all()
    # flows in transit after each sending round (the first round, from A at
    # t = 0, has no row): their peak is P
    sent0 = c["E"] - int(tr[:, 3].sum())
    transit = sent0 + np.cumsum(tr[:, 3] - tr[:, 1])
    assert (transit >= 0).all()
    assert max(sent0, int(transit.max())) == c["P"]


# the environments of section 7 (passage times 1 and 2, M above every path
# weight): Lemma 1's, Theorem 2's construction and Theorem 1's random one
SECTION7 = [lambda: gen.lemma1_environment(100), lambda: gen.fractal_environment(8),
            lambda: gen.fractal_environment(7, levels=3), lambda: gen.binary_environment(150, 0.3, 5),
            lambda: gen.binary_environment(150, 0.7, 6)]


@pytest.mark.parametrize("k", range(len(SECTION7)))
@pytest.mark.parametrize("dense", [0, 0xFFFFFFFF])
@pytest.mark.parametrize("blocks", [0, 16])
def test_section7_environments_trace(solver, torch, k, dense, blocks):
    """Active set and deliveries per cycle on the adversarial environments,
    row by row against the oracle, in both forms of the improved set."""
    from oracle import oracle as O
    inst = SECTION7[k]()
    _say("case", inst.name, "dense", dense, "blocks", blocks)
    ref = O.solve_instance(inst, trace_cap=1 << 16)
    res, cnt, rows, tr = _gpu_trace(solver, torch, inst, 1 << 16, blocks=blocks, dense=dense)
    assert res.tuple() == ref.tuple() and cnt.asdict() == ref.counters
    assert rows == len(ref.trace)
    assert np.array_equal(tr[:rows], ref.trace), inst.name
