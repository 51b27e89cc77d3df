"""HIP path vs the CPU oracle: T, X, x, Y, F2, every final label and every
counter must match exactly (all arithmetic is integer).

Small and ragged lattices run the oracle in-process; the 128^3 and 256^3
workloads compare against stored oracle outputs (tests/golden/*.json,
written by tests/golden/make_golden.py, which calls only the oracle).
"""
import glob
import hashlib
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
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def solver(torch):
    from paper_1511_06441_amd import csp
    s = csp.Solver(0)
    yield s
    s.close()


PATHS = [1, 2, 3]       # range-owned, global labels, range-owned with pencils for d = 3


def gpu_solve(solver, torch, inst, blocks=0, path=0, dense=-1, **kw):
    from paper_1511_06441_amd import csp
    di = csp.to_device(inst)
    lab = torch.zeros(inst.N, dtype=torch.int32, device="cuda")
    csp.csp_set_blocks(solver.ctx, blocks)
    csp.csp_set_path(solver.ctx, path)
    csp.csp_set_dense_threshold(solver.ctx, dense)
    try:
        res, cnt = solver.solve(di, labels=lab, **kw)
        used = csp.csp_last_path(solver.ctx)
    finally:
        csp.csp_set_blocks(solver.ctx, 0)
        csp.csp_set_path(solver.ctx, 0)
        csp.csp_set_dense_threshold(solver.ctx, -1)
    torch.cuda.synchronize()
    _say("  path", used, "kernel_ms %.3f" % csp.csp_last_kernel_ms(solver.ctx))
    assert path == 0 or used == (1 if path == 3 else path)
    return res, cnt, lab.cpu().numpy().view(np.uint32)


def _oracle(inst):
    from oracle import oracle as O
    return O.solve_instance(inst)


def _compare(inst, res, cnt, lab, ref):
    assert res.tuple() == ref.tuple(), (inst.name, res.tuple(), ref.tuple())
    assert cnt.asdict() == ref.counters, (inst.name, cnt.asdict(), ref.counters)
    bad = np.nonzero(lab != ref.labels)[0]
    assert bad.size == 0, (inst.name, bad[:10], lab[bad[:10]], ref.labels[bad[:10]])


def _corner(d, n, seed, K, M):
    inst = gen.opposite_faces(d, n, seed, K, K, M)
    inst.A = np.zeros(inst.N, np.uint8)
    inst.A[0] = 1
    inst.B = np.zeros(inst.N, np.uint8)
    inst.B[inst.N - 1] = 1
    inst.name = f"corner_d{d}_n{n}_s{seed}"
    return inst


SMALL = [
    # (d, n, seed, K1, K2, M, f1_const, f2_const)
    (1, 2, 1, 5, 5, 10, None, None),
    (1, 3, 2, 5, 5, 4, None, None),
    (1, 50, 3, 9, 9, 200, None, None),
    (2, 2, 4, 3, 3, 7, None, None),
    (2, 3, 5, 4, 4, 9, None, None),
    (2, 5, 6, 5, 5, 20, None, None),
    (2, 17, 7, 5, 5, 60, None, None),
    (2, 17, 8, 5, 5, 5, None, None),          # infeasible
    (2, 31, 9, 255, 255, 3000, None, None),   # long timers, wide wheel
    (2, 40, 10, 1, 3, 100, 1, None),          # unit times
    (2, 23, 11, 1, 1, 50, 1, 1),              # all ones: ties everywhere
    (3, 2, 12, 5, 5, 20, None, None),
    (3, 3, 13, 7, 7, 30, None, None),
    (3, 7, 14, 10, 10, 60, None, None),
    (3, 20, 15, 10, 10, 150, None, None),
    (3, 33, 16, 10, 10, 300, None, None),
    (4, 3, 17, 4, 4, 20, None, None),
    (4, 5, 18, 6, 6, 40, None, None),
    (4, 9, 19, 8, 8, 80, None, None),
]


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("case", SMALL, ids=[f"d{c[0]}n{c[1]}s{c[2]}M{c[5]}" for c in SMALL])
def test_small_vs_oracle(solver, torch, case, path):
    d, n, seed, K1, K2, M, c1, c2 = case
    inst = gen.opposite_faces(d, n, seed, K1, K2, M, f1_const=c1, f2_const=c2)
    inst.name = f"d{d}n{n}s{seed}M{M}"
    _say("case", inst.name, "path", path)
    ref = _oracle(inst)
    res, cnt, lab = gpu_solve(solver, torch, inst, path=path)
    _compare(inst, res, cnt, lab, ref)


# dense form of I_t: 0 sweeps the bitmap every cycle, 2^32-1 never does,
# 64 switches between the two forms from cycle to cycle
DENSE = [0, 64, 0xFFFFFFFF]


@pytest.mark.parametrize("dense", DENSE)
@pytest.mark.parametrize("path", [1, 3])
@pytest.mark.parametrize("case", SMALL, ids=[f"d{c[0]}n{c[1]}s{c[2]}M{c[5]}" for c in SMALL])
def test_dense_sweep_vs_oracle(solver, torch, case, path, dense):
    d, n, seed, K1, K2, M, c1, c2 = case
    inst = gen.opposite_faces(d, n, seed, K1, K2, M, f1_const=c1, f2_const=c2)
    inst.name = f"d{d}n{n}s{seed}M{M}"
    _say("case", inst.name, "path", path, "dense", dense)
    ref = _oracle(inst)
    res, cnt, lab = gpu_solve(solver, torch, inst, path=path, dense=dense, blocks=8)
    _compare(inst, res, cnt, lab, ref)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("blocks", [1, 2, 3, 8, 64, 256])
@pytest.mark.parametrize("which", ["square", "cube", "corner"])
def test_block_counts_vs_oracle(solver, torch, blocks, which, path):
    """Multi-block grids (grid barrier, cross-block queues) on small inputs."""
    if which == "square":
        inst = gen.square64(2)
    elif which == "cube":
        inst = gen.opposite_faces(3, 24, 5, 10, 10, 200)
        inst.name = "cube24"
    else:
        inst = _corner(3, 12, 3, 6, 150)
    _say("case", inst.name, "blocks", blocks, "path", path)
    ref = _oracle(inst)
    res, cnt, lab = gpu_solve(solver, torch, inst, blocks=blocks, path=path)
    _compare(inst, res, cnt, lab, ref)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_square64_vs_oracle(solver, torch, seed, path):
    inst = gen.square64(seed)
    _say("case", inst.name, "path", path)
    ref = _oracle(inst)
    res, cnt, lab = gpu_solve(solver, torch, inst, path=path)
    _compare(inst, res, cnt, lab, ref)


def test_corner_and_boundary_shapes(solver, torch):
    for inst in (_corner(2, 30, 1, 5, 80), _corner(3, 10, 2, 5, 60),
                 gen.cube_boundary_to_center(20, 4, K=100, M=3000)):
        _say("case", inst.name)
        ref = _oracle(inst)
        res, cnt, lab = gpu_solve(solver, torch, inst)
        _compare(inst, res, cnt, lab, ref)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("case", [(2, 17, 31, 1), (2, 17, 32, 65535), (2, 17, 33, 65536), (3, 7, 34, 70001),
                                  (2, 17, 35, 0x0FFFFFFF), (3, 9, 36, 0x0FFFFFFF), (4, 4, 37, 0x0FFFFFFF)],
                         ids=lambda c: f"d{c[0]}n{c[1]}M{c[3]}")
def test_extreme_M(solver, torch, case, path):
    """M = 1 (no flow can leave A), M on both sides of the 16-bit label
    boundary, and the largest M the library takes."""
    d, n, seed, M = case
    inst = gen.opposite_faces(d, n, seed, 9, 9, M)
    _say("case", inst.name, "M", M, "path", path)
    ref = _oracle(inst)
    res, cnt, lab = gpu_solve(solver, torch, inst, path=path)
    _compare(inst, res, cnt, lab, ref)
    if M == 1:
        assert res.T == -1


def test_empty_A(solver, torch):
    inst = gen.square64(1)
    inst.A = np.zeros(inst.N, np.uint8)
    res, cnt, lab = gpu_solve(solver, torch, inst)
    assert res.tuple() == (-1, -1, -1, -1, -1) and lab.max() == 0


# ---------------------------------------------------------------------------
# full-size workloads against stored oracle outputs
# ---------------------------------------------------------------------------

def _golden_cases():
    out = []
    for pat in ("cube*.json", "paper*.json"):
        for f in sorted(glob.glob(os.path.join(GOLDEN, pat))):
            out.append(os.path.basename(f)[:-5])
    return out


def _build(rec):
    nm = rec["name"]
    if nm.startswith("cube128"):
        return gen.cube128(rec["meta"]["seed"], rec["M"])
    if nm.startswith("cube256stress"):
        return gen.cube256_stress(rec["meta"]["seed"], rec["M"])
    if nm.startswith("cube256"):
        return gen.cube256(rec["meta"]["seed"], rec["M"])
    if nm.startswith("paper"):
        return gen.cube_boundary_to_center(rec["n"], rec["meta"]["seed"], K=rec["meta"]["K1"], M=rec["M"])
    raise KeyError(nm)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("name", _golden_cases())
def test_full_size_vs_stored_oracle(solver, torch, name, path):
    with open(os.path.join(GOLDEN, name + ".json")) as fh:
        rec = json.load(fh)
    inst = _build(rec)
    _say("case", name, "path", path)
    res, cnt, lab = gpu_solve(solver, torch, inst, path=path)
    assert res.tuple() == (rec["T"], rec["X"], rec["x"], rec["Y"], rec["F2"])
    assert cnt.asdict() == rec["counters"]
    assert hashlib.sha256(lab.astype("<u4").tobytes()).hexdigest() == rec["labels_sha256"]


@pytest.mark.parametrize("dense", [0, 1024])
@pytest.mark.parametrize("name", _golden_cases())
def test_full_size_dense_vs_stored_oracle(solver, torch, name, dense):
    """The full-size workloads with the improved set swept into vertex order
    every cycle (0) or when a range's set exceeds 1,024 vertices."""
    with open(os.path.join(GOLDEN, name + ".json")) as fh:
        rec = json.load(fh)
    inst = _build(rec)
    _say("case", name, "dense", dense)
    res, cnt, lab = gpu_solve(solver, torch, inst, dense=dense)
    assert res.tuple() == (rec["T"], rec["X"], rec["x"], rec["Y"], rec["F2"])
    assert cnt.asdict() == rec["counters"]
    assert hashlib.sha256(lab.astype("<u4").tobytes()).hexdigest() == rec["labels_sha256"]


@pytest.mark.parametrize("path", PATHS)
def test_stress_closed_form(solver, torch, path):
    """f1 == 1 on the 256^3 cube: only straight axis-0 lines arrive by 255."""
    from tests import pins
    inst = gen.cube256_stress(22)
    _say("case", inst.name, "path", path)
    res, cnt, lab = gpu_solve(solver, torch, inst, path=path)
    assert res.tuple() == pins.straight_line_answer(3, 256, inst.f2)


# ---------------------------------------------------------------------------
# determinism, retries, errors, host-pointer entry, path recovery
# ---------------------------------------------------------------------------

def test_repeat_runs_identical(solver, torch):
    inst = gen.cube128(12, 700)
    r1, c1, l1 = gpu_solve(solver, torch, inst)
    r2, c2, l2 = gpu_solve(solver, torch, inst)
    assert r1.tuple() == r2.tuple() and c1.asdict() == c2.asdict() and np.array_equal(l1, l2)


@pytest.mark.parametrize("path", PATHS)
def test_pool_overflow_retry_gives_same_result(solver, torch, path):
    from paper_1511_06441_amd import csp
    inst = gen.square64(3)
    ref = _oracle(inst)
    csp.csp_set_pool_hint(solver.ctx, 1)
    try:
        res, cnt, lab = gpu_solve(solver, torch, inst, blocks=4, path=path)
    finally:
        csp.csp_set_pool_hint(solver.ctx, 0)
    _compare(inst, res, cnt, lab, ref)


@pytest.mark.parametrize("path", [1, 3])
def test_pool_overflow_retry_3d(solver, torch, path):
    """A tiny wheel and candidate buffers on a 3-d lattice (contiguous and
    pencil ranges) force retries; results equal the oracle's."""
    from paper_1511_06441_amd import csp
    inst = gen.opposite_faces(3, 24, 9, 6, 6, 150)
    ref = _oracle(inst)
    csp.csp_set_pool_hint(solver.ctx, 1)
    try:
        res, cnt, lab = gpu_solve(solver, torch, inst, blocks=16, path=path)
    finally:
        csp.csp_set_pool_hint(solver.ctx, 0)
    _compare(inst, res, cnt, lab, ref)


def test_cycle_cap_cancels(solver, torch):
    from paper_1511_06441_amd import csp
    inst = gen.square64(1)
    with pytest.raises(csp.CspError) as e:
        gpu_solve(solver, torch, inst, max_cycles=5)
    assert e.value.code == csp.CSP_ECANCELED
    res, cnt, lab = gpu_solve(solver, torch, inst)          # context still usable
    assert res.T == 142


def test_invalid_inputs_rejected(solver, torch):
    from paper_1511_06441_amd import csp
    base = gen.opposite_faces(2, 8, 1, 5, 5, 30)

    def expect_einval(inst, d=None, n=None, M=None):
        di = csp.to_device(inst)
        with pytest.raises(csp.CspError) as e:
            csp.csp_solve_dev(solver.ctx, d or inst.d, n or inst.n, di.f1, di.f2, di.A, di.B,
                              inst.M if M is None else M)
        assert e.value.code == csp.CSP_EINVAL

    bad = gen.opposite_faces(2, 8, 1, 5, 5, 30)
    bad.B = bad.A.copy()
    expect_einval(bad)                                       # A and B overlap
    bad = gen.opposite_faces(2, 8, 1, 5, 5, 30)
    bad.f2[3] = 0
    expect_einval(bad)                                       # zero weight on a real edge
    expect_einval(base, M=0)
    expect_einval(base, M=csp.CSP_MAX_M + 1)
    expect_einval(base, d=5)
    expect_einval(base, n=1)
    # a zero on a padding entry is fine
    ok = gen.opposite_faces(2, 8, 1, 5, 5, 30)
    assert ok.f1[7] == 0
    gpu_solve(solver, torch, ok)


def test_host_pointer_entry(solver, torch):
    from paper_1511_06441_amd import csp
    inst = gen.square64(2)
    ref = _oracle(inst)
    lab = np.zeros(inst.N, np.uint32)
    res, cnt = csp.csp_solve(solver.ctx, inst.d, inst.n, inst.f1, inst.f2, inst.A, inst.B, inst.M, lab)
    _compare(inst, res, cnt, lab, ref)


@pytest.mark.parametrize("case", [(2, 12, 1, 5, 5, 50), (3, 6, 3, 10, 10, 60), (2, 64, 2, 5, 5, 200),
                                  (3, 16, 4, 10, 10, 150)])
def test_reconstruct_vs_oracle(solver, torch, case):
    from oracle import oracle as O
    from paper_1511_06441_amd import csp
    d, n, seed, K1, K2, M = case
    inst = gen.opposite_faces(d, n, seed, K1, K2, M)
    path_ref, res_ref, _ = O.reconstruct(d, n, inst.f1, inst.f2, inst.A, inst.B, M)
    di = csp.to_device(inst)
    scratch = torch.zeros(inst.N, dtype=torch.uint8, device="cuda")
    path, res = solver.reconstruct(di, scratch)
    assert res.tuple() == res_ref.tuple()
    assert path.tolist() == path_ref.tolist()
    assert int(scratch.sum().item()) == 0


@pytest.mark.parametrize("case", [(2, 12, 1, 5, 5, 50), (3, 9, 5, 10, 10, 90), (4, 5, 6, 6, 6, 40),
                                  (2, 17, 8, 5, 5, 5)])
def test_reconstruct_host_buffers_vs_oracle(solver, torch, case):
    """csp_reconstruct on host arrays gives the oracle's path and result;
    a path buffer that is too short is refused with the needed length."""
    from oracle import oracle as O
    from paper_1511_06441_amd import csp
    d, n, seed, K1, K2, M = case
    inst = gen.opposite_faces(d, n, seed, K1, K2, M)
    path_ref, res_ref, _ = O.reconstruct(d, n, inst.f1, inst.f2, inst.A, inst.B, M)
    path, res = csp.csp_reconstruct(solver.ctx, d, n, inst.f1, inst.f2, inst.A, inst.B, M, inst.N + 1)
    assert res.tuple() == res_ref.tuple()
    assert path.tolist() == [int(v) for v in path_ref]
    if len(path_ref) > 1:
        with pytest.raises(csp.CspError) as e:
            csp.csp_reconstruct(solver.ctx, d, n, inst.f1, inst.f2, inst.A, inst.B, M, 1)
        assert e.value.code == csp.CSP_EINVAL


# ---------------------------------------------------------------------------
# path recovery from the improvement log (one solve, then a walk back)
# ---------------------------------------------------------------------------

LOG_CASES = [(2, 12, 1, 5, 5, 50), (3, 6, 3, 10, 10, 60), (2, 64, 2, 5, 5, 200), (3, 16, 4, 10, 10, 150),
             (2, 150, 6, 20, 20, 900), (3, 40, 8, 3, 3, 200), (2, 40, 9, 1, 1, 100)]


@pytest.mark.parametrize("case", LOG_CASES)
@pytest.mark.parametrize("blocks,path", [(0, 0), (16, 1), (16, 3)])
def test_reconstruct_log_vs_oracle(solver, torch, case, blocks, path):
    """The logged walk gives the oracle's repeated-solve path, result and counters."""
    from oracle import oracle as O
    from paper_1511_06441_amd import csp
    d, n, seed, K1, K2, M = case
    inst = gen.opposite_faces(d, n, seed, K1, K2, M)
    _say("case", inst.name, "blocks", blocks, "path", path)
    path_ref, res_ref, _ = O.reconstruct(d, n, inst.f1, inst.f2, inst.A, inst.B, M)
    ref = _oracle(inst)
    di = csp.to_device(inst)
    csp.csp_set_blocks(solver.ctx, blocks)
    csp.csp_set_path(solver.ctx, path)
    try:
        got, res, cnt = solver.reconstruct_log(di)
    finally:
        csp.csp_set_blocks(solver.ctx, 0)
        csp.csp_set_path(solver.ctx, 0)
    assert res.tuple() == res_ref.tuple() == ref.tuple()
    assert cnt.asdict() == ref.counters
    assert got.tolist() == path_ref.tolist()


@pytest.mark.parametrize("case", [LOG_CASES[1], LOG_CASES[3], LOG_CASES[5]])
@pytest.mark.parametrize("path", [1, 3])
def test_reconstruct_log_dense_form_vs_oracle(solver, torch, case, path):
    """The logged walk with I_t built in dense form every cycle (the bitmap
    sweep orders the improved vertices, and so the log, differently) gives the
    oracle's repeated-solve path, result and counters."""
    from oracle import oracle as O
    from paper_1511_06441_amd import csp
    d, n, seed, K1, K2, M = case
    inst = gen.opposite_faces(d, n, seed, K1, K2, M)
    _say("case", inst.name, "blocks 16, path", path, "dense 0")
    path_ref, res_ref, _ = O.reconstruct(d, n, inst.f1, inst.f2, inst.A, inst.B, M)
    ref = _oracle(inst)
    di = csp.to_device(inst)
    csp.csp_set_blocks(solver.ctx, 16)
    csp.csp_set_path(solver.ctx, path)
    csp.csp_set_dense_threshold(solver.ctx, 0)
    try:
        got, res, cnt = solver.reconstruct_log(di)
    finally:
        csp.csp_set_blocks(solver.ctx, 0)
        csp.csp_set_path(solver.ctx, 0)
        csp.csp_set_dense_threshold(solver.ctx, -1)
    assert res.tuple() == res_ref.tuple() == ref.tuple()
    assert cnt.asdict() == ref.counters
    assert got.tolist() == path_ref.tolist()


@pytest.mark.parametrize("which", ["cube128", "paper75"])
def test_reconstruct_log_equals_repeated_solves_full_size(solver, torch, which):
    from paper_1511_06441_amd import csp
    inst = gen.cube128(11, 700) if which == "cube128" else gen.cube_boundary_to_center(75, 61, K=100, M=10000)
    _say("case", inst.name)
    di = csp.to_device(inst)
    got, res, cnt = solver.reconstruct_log(di)
    scratch = torch.zeros(inst.N, dtype=torch.uint8, device="cuda")
    path, res2 = solver.reconstruct(di, scratch)
    assert res.tuple() == res2.tuple()
    assert got.tolist() == path.tolist()
    _say("  path vertices", len(got))


def test_reconstruct_log_retries_small_log(solver, torch):
    """A one-flow wheel also shrinks the starting log: retries give the same path."""
    from oracle import oracle as O
    from paper_1511_06441_amd import csp
    inst = gen.opposite_faces(3, 24, 9, 6, 6, 150)
    path_ref, res_ref, _ = O.reconstruct(3, 24, inst.f1, inst.f2, inst.A, inst.B, 150)
    csp.csp_set_pool_hint(solver.ctx, 1)
    try:
        got, res, cnt = solver.reconstruct_log(csp.to_device(inst))
    finally:
        csp.csp_set_pool_hint(solver.ctx, 0)
    assert res.tuple() == res_ref.tuple() and got.tolist() == path_ref.tolist()
