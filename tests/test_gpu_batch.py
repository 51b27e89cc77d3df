"""Batched solves (one persistent launch per dimension): every problem's T,
X, x, Y, F2, labels and counters equal the oracle's, and equal the same
problem solved alone."""
import sys

import numpy as np
import pytest

from paper_1511_06441_amd import inputs as gen

pytestmark = pytest.mark.gpu


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


def _batch(solver, torch, insts):
    from paper_1511_06441_amd import csp
    dev = [csp.to_device(i) for i in insts]
    labs = [torch.zeros(i.N, dtype=torch.int32, device="cuda") for i in insts]
    res, cnt = csp.csp_solve_batch(solver.ctx, dev, labels=labs)
    torch.cuda.synchronize()
    _say("  batch kernel ms %.3f" % csp.csp_last_kernel_ms(solver.ctx))
    return res, cnt, [l.cpu().numpy().view(np.uint32) for l in labs]


def _check_vs_oracle(inst, res, cnt, lab):
    from oracle import oracle as O
    ref = O.solve_instance(inst)
    assert res.tuple() == ref.tuple(), (inst.name, res.tuple(), ref.tuple())
    assert cnt.asdict() == ref.counters, (inst.name, cnt.asdict(), ref.counters)
    assert np.array_equal(lab, ref.labels), inst.name


def test_mixed_small_batch_vs_oracle(solver, torch):
    insts = [gen.mixed_instance(41, j, lo2=(8, 48), lo3=(4, 16)) for j in range(48)]
    _say("mixed small batch of", len(insts))
    res, cnt, labs = _batch(solver, torch, insts)
    for inst, r, c, l in zip(insts, res, cnt, labs):
        _check_vs_oracle(inst, r, c, l)


def test_gangs_vs_oracle(solver, torch):
    """Problems too large for one workgroup's LDS run on gangs of workgroups."""
    insts = [gen.opposite_faces(2, 420, 3, 9, 9, 3000),      # 176,400 vertices
             gen.opposite_faces(3, 52, 4, 12, 12, 600),      # 140,608 vertices
             gen.opposite_faces(2, 300, 5, 4, 4, 1200),
             gen.square64(1), gen.square64(2),
             gen.opposite_faces(3, 20, 6, 7, 7, 160)]
    for i, inst in enumerate(insts):
        inst.name = f"gang{i}"
    _say("gang batch")
    res, cnt, labs = _batch(solver, torch, insts)
    for inst, r, c, l in zip(insts, res, cnt, labs):
        _check_vs_oracle(inst, r, c, l)


def test_all_dimensions_and_extreme_M(solver, torch):
    """d = 1..4 in one batch (one persistent launch per dimension), with M = 1,
    M on both sides of the 16-bit label limit, the largest M, a corner-to-
    corner problem, and a 4-d problem that needs a gang."""
    insts = [gen.opposite_faces(1, 200, 1, 9, 9, 500), gen.opposite_faces(1, 7, 2, 3, 3, 1),
             gen.opposite_faces(4, 6, 3, 5, 5, 40), gen.opposite_faces(4, 9, 4, 8, 8, 0x0FFFFFFF),
             gen.opposite_faces(2, 40, 5, 5, 5, 65535), gen.opposite_faces(2, 40, 6, 5, 5, 65536),
             gen.opposite_faces(3, 20, 7, 9, 9, 70001), gen.opposite_faces(4, 24, 8, 7, 7, 400),
             gen.opposite_faces(1, 2, 9, 4, 4, 10)]
    corner = gen.opposite_faces(3, 17, 10, 6, 6, 200)
    corner.A = np.zeros(corner.N, np.uint8)
    corner.A[0] = 1
    corner.B = np.zeros(corner.N, np.uint8)
    corner.B[corner.N - 1] = 1
    insts.append(corner)
    for i, inst in enumerate(insts):
        inst.name = f"dims{i}_d{inst.d}_n{inst.n}_M{inst.M}"
    _say("all-dimension batch of", len(insts))
    res, cnt, labs = _batch(solver, torch, insts)
    for inst, r, c, l in zip(insts, res, cnt, labs):
        _check_vs_oracle(inst, r, c, l)
    assert res[1].T == -1                                   # M = 1: no water leaves A


def test_repeated_batch_with_remembered_sizes(solver, torch):
    """The second run of a batch starts with the pool sizes the first one
    grew to; results and counters are the same and equal the oracle's."""
    from oracle import oracle as O
    from paper_1511_06441_amd import csp
    insts = [gen.mixed_instance(45, j, lo2=(16, 120), lo3=(8, 30)) for j in range(40)]
    dev = [csp.to_device(i) for i in insts]
    csp.csp_autotune_clear(solver.ctx)
    r1, c1 = csp.csp_solve_batch(solver.ctx, dev)
    ms1 = csp.csp_last_kernel_ms(solver.ctx)
    r2, c2 = csp.csp_solve_batch(solver.ctx, dev)
    ms2 = csp.csp_last_kernel_ms(solver.ctx)
    _say("first run %.2f ms, second %.2f ms" % (ms1, ms2))
    for inst, a, b, ca, cb in zip(insts, r1, r2, c1, c2):
        ref = O.solve_instance(inst, want_labels=False)
        assert a.tuple() == b.tuple() == ref.tuple(), inst.name
        assert ca.asdict() == cb.asdict() == ref.counters, inst.name
    csp.csp_autotune_clear(solver.ctx)


def test_batch_equals_alone(solver, torch):
    from paper_1511_06441_amd import csp
    insts = [gen.mixed_instance(41, j, lo2=(16, 200), lo3=(8, 40)) for j in range(24)]
    res, cnt, labs = _batch(solver, torch, insts)
    for inst, r, c, l in zip(insts, res, cnt, labs):
        di = csp.to_device(inst)
        lab = torch.zeros(inst.N, dtype=torch.int32, device="cuda")
        r1, c1 = solver.solve(di, labels=lab)
        torch.cuda.synchronize()
        assert r.tuple() == r1.tuple() and c.asdict() == c1.asdict(), inst.name
        assert np.array_equal(l, lab.cpu().numpy().view(np.uint32)), inst.name


def test_batch_overflow_retry(solver, torch):
    """A tiny starting wheel forces per-problem retries; results are unchanged."""
    from paper_1511_06441_amd import csp
    insts = [gen.mixed_instance(7, j, lo2=(8, 64), lo3=(4, 20)) for j in range(16)]
    csp.csp_set_pool_hint(solver.ctx, 1)
    try:
        res, cnt, labs = _batch(solver, torch, insts)
    finally:
        csp.csp_set_pool_hint(solver.ctx, 0)
    for inst, r, c, l in zip(insts, res, cnt, labs):
        _check_vs_oracle(inst, r, c, l)


def test_config4_sample_vs_plain(solver, torch):
    """The first 64 problems of the 1,024-problem mixed batch (master seed 41):
    batched results equal plain single-problem solves."""
    from paper_1511_06441_amd import csp
    insts = [gen.mixed_instance(41, j) for j in range(64)]
    _say("config-4 sample, vertices", sum(i.N for i in insts))
    res, cnt, labs = _batch(solver, torch, insts)
    for inst, r, c in zip(insts, res, cnt):
        di = csp.to_device(inst)
        r1, c1 = solver.solve(di)
        assert r.tuple() == r1.tuple() and c.asdict() == c1.asdict(), inst.name
        assert r.T < 0 or 0 < r.F2 < inst.M


def test_candidate_phase_overflow_always_retried(solver, torch):
    """A gang of 27 ranges on this 60^3 lattice (8,192 vertices per
    workgroup) overflows a wheel bucket while it accepts candidates.  The
    overflow must send the problem round again every time: when thread 0
    cleared the flag word non-atomically, the flag was sometimes lost and
    flows were dropped without a retry (about one run in three)."""
    from oracle import oracle as O
    from paper_1511_06441_amd import csp
    inst = gen.mixed_instance(41, 639)
    ref = O.solve_instance(inst, want_labels=False)
    dev = [csp.to_device(inst)]
    csp.csp_set_batch_target(solver.ctx, 8192)
    try:
        for k in range(60):
            # forget the sizes the overflow taught, so every run starts small
            csp.csp_autotune_clear(solver.ctx)
            csp.csp_set_batch_target(solver.ctx, 8192)
            res, cnt = csp.csp_solve_batch(solver.ctx, dev)
            assert res[0].tuple() == ref.tuple(), k
            assert cnt[0].asdict() == ref.counters, (k, cnt[0].asdict(), ref.counters)
    finally:
        csp.csp_set_batch_target(solver.ctx, 0)


def _golden(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", name + ".json")) as fh:
        return json.load(fh)


def test_config4_full_batch_vs_stored_oracle(solver, torch):
    """All 1,024 problems of the mixed batch (master seed 41, 306,237,961
    vertices) in one csp_solve_batch call against the oracle's stored
    outputs: T, X, x, Y, F2, every counter and the SHA-256 of every
    problem's labels.  The edges are drawn on the GPU with the same seeded
    generator (checked against the host draw by the CPU tests)."""
    import hashlib
    from paper_1511_06441_amd import csp
    rec = _golden("batch1024_s41")["problems"]
    assert len(rec) == 1024
    dev, labs = [], []
    for j, g in enumerate(rec):
        s, d, n, K, M = gen.mixed_params(41, j)
        assert (d, n, K, M, s) == (g["d"], g["n"], g["K"], g["M"], g["seed"])
        f1, f2 = gen.lattice_edges_torch(d, n, s, K, K, device="cuda")
        dev.append(csp.DeviceInstance(d, n, f1, f2, gen.face_mask_torch(d, n, 0, 0, "cuda"),
                                      gen.face_mask_torch(d, n, 0, n - 1, "cuda"), M))
        labs.append(torch.zeros(n ** d, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    _say("config-4 batch of 1,024 problems")
    res, cnt = csp.csp_solve_batch(solver.ctx, dev, labels=labs)
    torch.cuda.synchronize()
    _say("  batch kernel ms %.3f" % csp.csp_last_kernel_ms(solver.ctx))
    bad = []
    for j, g in enumerate(rec):
        lab = labs[j].cpu().numpy().view(np.uint32)
        ok = (res[j].tuple() == (g["T"], g["X"], g["x"], g["Y"], g["F2"]) and cnt[j].asdict() == g["counters"]
              and hashlib.sha256(lab.astype("<u4").tobytes()).hexdigest() == g["labels_sha256"])
        if not ok:
            bad.append(j)
    assert not bad, ("problems differing from the oracle", bad[:20])
