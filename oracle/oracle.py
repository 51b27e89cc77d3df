"""ctypes front end of the CPU oracle (csp_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  Nothing here
depends on the HIP library.

Results are {T, X, x, Y, F2} with -1 everywhere when no path exists
(section 1 of the paper defines the problem; section 5 "Termination" the
outputs).  Counters are {C, U, D, E, R, P, I}: cycles, label improvements
(A counted at time 0), neighbour tests, flows sent, flows delivered, peak
flows in transit, largest improved set.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csp_oracle.c")
LIB = os.path.join(HERE, "libcsp_oracle.so")

COUNTER_NAMES = ("C", "U", "D", "E", "R", "P", "I")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 into oracle/libcsp_oracle.so."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-Wextra", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = ctypes.CDLL(LIB)
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.orc_solve_lattice.argtypes = [ctypes.c_int, i64, p, p, p, p, i64, p, p, p, p, i64, p, i64]
        L.orc_solve_lattice.restype = ctypes.c_int
        L.orc_solve_graph.argtypes = [i64, p, p, p, p, p, p, p, i64, p, p, p, p, i64, p, i64]
        L.orc_solve_graph.restype = ctypes.c_int
        L.orc_lattice_adjacency.argtypes = [ctypes.c_int, i64, p, p, p, p, p, p, p]
        L.orc_lattice_adjacency.restype = ctypes.c_int
        L.orc_reconstruct_lattice.argtypes = [ctypes.c_int, i64, p, p, p, p, i64, p, i64, p, p, p, i64]
        L.orc_reconstruct_lattice.restype = ctypes.c_int
        L.orc_reconstruct_lattice_upto.argtypes = [ctypes.c_int, i64, p, p, p, p, i64, p, i64, p, p,
                                                   p, i64, i64, p]
        L.orc_reconstruct_lattice_upto.restype = ctypes.c_int
        L.orc_reconstruct_graph.argtypes = [i64, p, p, p, p, p, p, p, i64, p, i64, p, p, p, i64]
        L.orc_reconstruct_graph.restype = ctypes.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


@dataclass
class Result:
    T: int
    X: int
    x: int
    Y: int
    F2: int
    labels: np.ndarray | None = None
    counters: dict | None = None
    trace: np.ndarray | None = None

    def tuple(self):
        return (self.T, self.X, self.x, self.Y, self.F2)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def solve(d, n, f1, f2, A, B, M, want_labels=True, trace_cap=0, max_cycles=0) -> Result:
    """Run the cycle on an n^d lattice (SoA edge arrays [d][n^d])."""
    f1, f2, A, B = _u8(f1), _u8(f2), _u8(A), _u8(B)
    N = n ** d
    if f1.size != d * N or f2.size != d * N or A.size != N or B.size != N:
        raise ValueError("array sizes do not match d, n")
    labels = np.zeros(N, dtype=np.uint32) if want_labels else None
    res = np.zeros(5, dtype=np.int64)
    cnt = np.zeros(7, dtype=np.int64)
    trace = np.zeros((max(trace_cap, 0), 4), dtype=np.int64) if trace_cap > 0 else None
    tlen = np.zeros(1, dtype=np.int64)
    rc = lib().orc_solve_lattice(d, n, _ptr(f1), _ptr(f2), _ptr(A), _ptr(B), int(M),
                                 _ptr(labels), _ptr(res), _ptr(cnt), _ptr(trace),
                                 trace_cap, _ptr(tlen), max_cycles)
    if rc != 0:
        raise OracleError(f"oracle solve failed: {rc}")
    r = Result(*[int(v) for v in res], labels=labels,
               counters=dict(zip(COUNTER_NAMES, [int(c) for c in cnt])))
    if trace is not None:
        r.trace = trace[:min(int(tlen[0]), trace_cap)].copy()
    return r


def solve_instance(inst, **kw) -> Result:
    return solve(inst.d, inst.n, inst.f1, inst.f2, inst.A, inst.B, inst.M, **kw)


def lattice_adjacency(d, n, f1, f2):
    """Adjacency lists of the lattice: (off, nbr, f1, f2, eid) per directed entry."""
    f1, f2 = _u8(f1), _u8(f2)
    N = n ** d
    off = np.zeros(N + 1, dtype=np.int64)
    if lib().orc_lattice_adjacency(d, n, _ptr(f1), _ptr(f2), _ptr(off), None, None, None, None):
        raise OracleError("bad lattice")
    m = int(off[N])
    nbr = np.zeros(m, dtype=np.int32)
    a1 = np.zeros(m, dtype=np.uint8)
    a2 = np.zeros(m, dtype=np.uint8)
    eid = np.zeros(m, dtype=np.int64)
    if lib().orc_lattice_adjacency(d, n, _ptr(f1), _ptr(f2), _ptr(off), _ptr(nbr), _ptr(a1),
                                   _ptr(a2), _ptr(eid)):
        raise OracleError("bad lattice")
    return off, nbr, a1, a2, eid


def graph_from_edges(nv, edges):
    """Adjacency lists from an undirected edge list [(u, v, f1, f2), ...].

    Edge id = position in the list.  Neighbours are sorted ascending.
    """
    adj = [[] for _ in range(nv)]
    for e, (u, v, w1, w2) in enumerate(edges):
        adj[u].append((v, w1, w2, e))
        adj[v].append((u, w1, w2, e))
    off = np.zeros(nv + 1, dtype=np.int64)
    rows = []
    for u in range(nv):
        adj[u].sort()
        rows.extend(adj[u])
        off[u + 1] = len(rows)
    nbr = np.array([r[0] for r in rows], dtype=np.int32)
    a1 = np.array([r[1] for r in rows], dtype=np.uint8)
    a2 = np.array([r[2] for r in rows], dtype=np.uint8)
    eid = np.array([r[3] for r in rows], dtype=np.int64)
    return off, nbr, a1, a2, eid


def solve_graph(graph, A, B, M, want_labels=True, trace_cap=0, max_cycles=0) -> Result:
    off, nbr, a1, a2, eid = graph
    nv = off.size - 1
    A, B = _u8(A), _u8(B)
    labels = np.zeros(nv, dtype=np.uint32) if want_labels else None
    res = np.zeros(5, dtype=np.int64)
    cnt = np.zeros(7, dtype=np.int64)
    trace = np.zeros((max(trace_cap, 0), 4), dtype=np.int64) if trace_cap > 0 else None
    tlen = np.zeros(1, dtype=np.int64)
    rc = lib().orc_solve_graph(nv, _ptr(off), _ptr(nbr), _ptr(a1), _ptr(a2), _ptr(eid),
                               _ptr(A), _ptr(B), int(M), _ptr(labels), _ptr(res), _ptr(cnt),
                               _ptr(trace), trace_cap, _ptr(tlen), max_cycles)
    if rc != 0:
        raise OracleError(f"oracle solve failed: {rc}")
    r = Result(*[int(v) for v in res], labels=labels,
               counters=dict(zip(COUNTER_NAMES, [int(c) for c in cnt])))
    if trace is not None:
        r.trace = trace[:min(int(tlen[0]), trace_cap)].copy()
    return r


def reconstruct(d, n, f1, f2, A, B, M, cap=None):
    """Vertex path from the A end to X by repeated solves, plus the per-solve rows."""
    f1, f2, A, B = _u8(f1), _u8(f2), _u8(A), _u8(B)
    N = n ** d
    cap = cap if cap is not None else N + 1
    path = np.zeros(cap, dtype=np.int64)
    steps = np.zeros((cap, 5), dtype=np.int64)
    ln = np.zeros(1, dtype=np.int64)
    res = np.zeros(5, dtype=np.int64)
    rc = lib().orc_reconstruct_lattice(d, n, _ptr(f1), _ptr(f2), _ptr(A), _ptr(B), int(M),
                                       _ptr(path), cap, _ptr(ln), _ptr(res), _ptr(steps), cap)
    if rc != 0:
        raise OracleError(f"oracle reconstruct failed: {rc}")
    L = int(ln[0])
    return path[:L].copy(), Result(*[int(v) for v in res]), steps[:max(L - 1, 0)].copy()


def reconstruct_upto(d, n, f1, f2, A, B, M, max_steps):
    """The first max_steps solves of the repeated-solve chain.

    Returns (vertices, result, rows, complete): the vertices found so far in
    path order (ending at X; the whole path from the A end when complete),
    the first solve's result and one {T, X, x, Y, F2} row per solve.
    """
    f1, f2, A, B = _u8(f1), _u8(f2), _u8(A), _u8(B)
    cap = int(max_steps) + 2
    path = np.zeros(cap, dtype=np.int64)
    steps = np.zeros((cap, 5), dtype=np.int64)
    ln = np.zeros(1, dtype=np.int64)
    res = np.zeros(5, dtype=np.int64)
    complete = np.zeros(1, dtype=np.int64)
    rc = lib().orc_reconstruct_lattice_upto(d, n, _ptr(f1), _ptr(f2), _ptr(A), _ptr(B), int(M),
                                            _ptr(path), cap, _ptr(ln), _ptr(res), _ptr(steps),
                                            cap, int(max_steps), _ptr(complete))
    if rc != 0:
        raise OracleError(f"oracle reconstruct failed: {rc}")
    L = int(ln[0])
    done = bool(complete[0])
    nrows = max(L - 1, 0)
    return path[:L].copy(), Result(*[int(v) for v in res]), steps[:nrows].copy(), done


def reconstruct_graph(graph, A, B, M, cap=None):
    off, nbr, a1, a2, eid = graph
    nv = off.size - 1
    A, B = _u8(A), _u8(B)
    cap = cap if cap is not None else nv + 1
    path = np.zeros(cap, dtype=np.int64)
    steps = np.zeros((cap, 5), dtype=np.int64)
    ln = np.zeros(1, dtype=np.int64)
    res = np.zeros(5, dtype=np.int64)
    rc = lib().orc_reconstruct_graph(nv, _ptr(off), _ptr(nbr), _ptr(a1), _ptr(a2), _ptr(eid),
                                     _ptr(A), _ptr(B), int(M), _ptr(path), cap, _ptr(ln),
                                     _ptr(res), _ptr(steps), cap)
    if rc != 0:
        raise OracleError(f"oracle reconstruct failed: {rc}")
    L = int(ln[0])
    return path[:L].copy(), Result(*[int(v) for v in res]), steps[:max(L - 1, 0)].copy()
