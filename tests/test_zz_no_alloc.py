"""csp_solve_dev_noalloc, the solve for callers that cannot allocate device
memory: on two calls in a row, the second on a smaller lattice, its result,
counters and labels equal csp_solve_dev's on the same inputs; a lattice whose
state cannot fit the static scratch is refused with CSP_EINVAL."""
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


def _both(solver, torch, inst):
    from paper_1511_06441_amd import csp
    di = csp.to_device(inst, "cuda:0")
    lab_ref = torch.zeros(inst.N, dtype=torch.int32, device="cuda:0")
    lab = torch.full((inst.N,), -1, dtype=torch.int32, device="cuda:0")
    _say("noalloc vs solve_dev:", inst.name)
    ref, cref = csp.csp_solve_dev(solver.ctx, di.d, di.n, di.f1, di.f2, di.A, di.B, di.M, labels=lab_ref)
    got, cgot = csp.csp_solve_dev_noalloc(solver.ctx, di.d, di.n, di.f1, di.f2, di.A, di.B, di.M, labels=lab)
    torch.cuda.synchronize()
    assert got.tuple() == ref.tuple(), (inst.name, got.tuple(), ref.tuple())
    assert cgot.asdict() == cref.asdict(), inst.name
    assert torch.equal(lab, lab_ref), inst.name
    return got


def test_noalloc_equals_solve_dev_twice_second_smaller(solver, torch):
    a = _both(solver, torch, gen.cube128(11, 400))
    b = _both(solver, torch, gen.square64(2))
    assert a.T > 0 and b.T > 0


def test_noalloc_refuses_a_lattice_beyond_the_scratch(solver, torch):
    from paper_1511_06441_amd import csp
    n, d = 256, 3
    f1, f2 = gen.lattice_edges_torch(d, n, 21, 100, 100, device="cuda")
    A = gen.face_mask_torch(d, n, 0, 0, "cuda")
    B = gen.face_mask_torch(d, n, 0, n - 1, "cuda")
    torch.cuda.synchronize()
    _say("noalloc refuses 256^3")
    with pytest.raises(csp.CspError) as e:
        csp.csp_solve_dev_noalloc(solver.ctx, d, n, f1, f2, A, B, 10000)
    assert e.value.code == csp.CSP_EINVAL and "CSP_SCRATCH_BYTES" in str(e.value)
