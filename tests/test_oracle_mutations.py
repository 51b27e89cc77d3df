"""The pins have teeth: plant plausible mistakes in a copy of the oracle's C
source (on the CPU, in a temporary directory) and check that the pin suite's
comparisons catch every one of them."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_1511_06441_amd import inputs as gen
from tests import pins

MUTATIONS = {
    "send test not strict": ("if (q > L[P]) {", "if (q >= L[P]) {"),
    "tie to larger source": ("f->src < tsrc[f->dst]", "f->src > tsrc[f->dst]"),
    "arrival one unit late": ("bk[(t + a1[j]) % NB]", "bk[(t + a1[j] + 1) % NB]"),
    "weight not subtracted": ("int64_t q = L[Q] - (int64_t)a2[j];", "int64_t q = L[Q] - (int64_t)a2[j] + 1;"),
    "X ties to larger index": ("(X < 0 || L[Q] > L[X])", "(X < 0 || L[Q] >= L[X])"),
    "F2 off by one": ("F2 = M - L[X];", "F2 = M - L[X] + 1;"),
    "commit not strict": ("if (tq[Q] > L[Q]) {", "if (tq[Q] >= L[Q]) {"),
    "A starts at M-1": ("L[v] = A[v] ? M : 0;", "L[v] = A[v] ? M - 1 : 0;"),
    "upper edge reads the weight as its time": ("a1[pos] = f1[k * N + v];", "a1[pos] = f2[k * N + v];"),
    "lower edge reads the wrong axis": ("a2[pos] = f2[k * N + u];", "a2[pos] = f2[((k + 1) % d) * N + u];"),
    "deliveries miscounted": ("R += b->n;", "R += b->n - (b->n > 1);"),
    "edge id of wrong end": ("eid[pos] = k * N + v;", "eid[pos] = k * N + v + stride[k];"),
    "continue after reaching B": ("if (X >= 0) break;", "if (X >= 0 && 0) break;"),
}


def _build_mutant(tmp_path, name, old, new):
    src = open(O.SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / f"m_{abs(hash(name))}.c"
    path.write_text(src.replace(old, new))
    so = str(path)[:-2] + ".so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-w", "-o", so, str(path)])
    L = ctypes.CDLL(so)
    p, i64 = ctypes.c_void_p, ctypes.c_int64
    L.orc_solve_lattice.argtypes = [ctypes.c_int, i64, p, p, p, p, i64, p, p, p, p, i64, p, i64]
    return L


def _run(L, inst):
    lab = np.zeros(inst.N, np.uint32)
    res = np.zeros(5, np.int64)
    cnt = np.zeros(7, np.int64)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    rc = L.orc_solve_lattice(inst.d, inst.n, ptr(inst.f1), ptr(inst.f2), ptr(inst.A), ptr(inst.B),
                             inst.M, ptr(lab), ptr(res), ptr(cnt), None, 0, None, 0)
    if rc != 0:
        return None                      # rejecting valid input is a caught mistake
    return tuple(res.tolist()), lab.astype(np.int64), dict(zip(O.COUNTER_NAMES, cnt.tolist()))


def _corner_to_corner(d, n, M):
    """All f equal to 1, A and B opposite corners: the last vertex before X is
    reached along several equally good paths, so only the tie rule picks Y."""
    inst = gen.opposite_faces(d, n, 1, 1, 1, M, f1_const=1, f2_const=1)
    inst.A = np.zeros(inst.N, np.uint8)
    inst.A[0] = 1
    inst.B = np.zeros(inst.N, np.uint8)
    inst.B[inst.N - 1] = 1
    return inst


# the opposite-faces case with every f equal to 1 reaches all of B at once
# with equal labels, so only the tie rule picks X
CASES = [lambda: gen.opposite_faces(2, 12, 1, 5, 5, 50),
         lambda: gen.opposite_faces(3, 6, 3, 10, 10, 60),
         lambda: gen.opposite_faces(2, 9, 6, 5, 5, 8),
         lambda: gen.opposite_faces(2, 8, 3, 9, 3, 12),
         lambda: gen.opposite_faces(2, 6, 1, 1, 1, 20, f1_const=1, f2_const=1),
         lambda: _corner_to_corner(3, 4, 30)]


@pytest.fixture(scope="module")
def references():
    out = []
    for make in CASES:
        inst = make()
        ref = pins.dp_solve(inst.N, pins.lattice_edge_list(inst.d, inst.n, inst.f1, inst.f2),
                            inst.A, inst.B, inst.M)
        out.append((inst, ref))
    return out


def test_unmutated_oracle_matches(references):
    for inst, ref in references:
        r = O.solve_instance(inst)
        assert r.tuple() == (ref["T"], ref["X"], ref["x"], ref["Y"], ref["F2"])
        assert np.array_equal(r.labels.astype(np.int64), ref["labels"])
        assert r.counters == ref["counters"]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutant_is_caught(tmp_path, references, name):
    old, new = MUTATIONS[name]
    L = _build_mutant(tmp_path, name, old, new)
    caught = False
    for inst, ref in references:
        out = _run(L, inst)
        if out is None:
            caught = True
            break
        res, lab, cnt = out
        if (res != (ref["T"], ref["X"], ref["x"], ref["Y"], ref["F2"])
                or not np.array_equal(lab, ref["labels"]) or cnt != ref["counters"]):
            caught = True
            break
    assert caught, f"mutation '{name}' was not caught by the recurrence pin"
