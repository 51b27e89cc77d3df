"""The environments of section 7 (passage times in {1, 2}, M infinite)
pinned on the CPU.

With f2 = f1 and M above every path weight, the best water at a vertex is
the earliest: its label is M - dist(v) from time dist(v) on (dist = shortest
f1 distance from the x-axis) and never improves later.  A vertex sends at
dist(v) over each edge to a neighbour not yet reached, and that water is in
transit until dist(v) + f1.  So the labels and the water in transit at every
time follow from one Dijkstra run (scipy), independently of the oracle.

* Lemma 1: the distances have the closed form min(2y, y + 2|x|); the
  lemma's active set A_T lies inside the set of vertices with water in
  transit at T (equality fails: the lemma leaves out vertices reached at
  T - 1 whose water is still travelling).
* Theorem 2's construction and the random environment of Theorem 1: the
  oracle's labels and water in transit at every time equal the Dijkstra
  derivation; the trace rows equal the time-indexed recurrence.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1511_06441_amd import inputs as gen
from tests import pins


def _dist(inst):
    edges = pins.lattice_edge_list(inst.d, inst.n, inst.f1, inst.f2)
    return edges, pins.scipy_multi_source(inst.N, edges, inst.A, edges[2])


def _transit_sources(edges, dist, T0):
    """Directed edges (v, w) carrying water at the end of the sending round
    of time T0, as a boolean per source vertex, and their count."""
    us, vs, w1 = edges[0], edges[1], edges[2]
    act = np.zeros(dist.size, bool)
    count = 0
    for a, b in ((us, vs), (vs, us)):
        m = (dist[a] <= T0) & (dist[b] > dist[a]) & (dist[a] + w1 > T0)
        act[a[m]] = True
        count += int(m.sum())
    return act, count


def _oracle_at(inst, T0):
    """Labels after the sending round of cycle T0 and water in transit then."""
    r = O.solve_instance(inst, max_cycles=T0, trace_cap=1 << 16)
    tr = r.trace
    assert tr[-1, 0] == T0 and len(tr) == T0          # every time unit delivers water
    # water sent from A at t = 0: every edge out of A to a vertex outside A
    edges = pins.lattice_edge_list(inst.d, inst.n, inst.f1, inst.f2)
    a = inst.A.astype(bool)
    sent0 = int((a[edges[0]] != a[edges[1]]).sum())
    transit = sent0 + int(tr[:, 3].sum()) - int(tr[:, 1].sum())
    return r, transit


def _coords(inst):
    n = inst.n
    m = (n - 1) // 2
    v = np.arange(inst.N)
    return v % n - m, v // n


@pytest.mark.parametrize("m", [6, 15])
def test_lemma1_distances_closed_form(m):
    inst = gen.lemma1_environment(m)
    _edges, dist = _dist(inst)
    x, y = _coords(inst)
    assert np.array_equal(dist, np.minimum(2 * y, y + 2 * np.abs(x)))


@pytest.mark.parametrize("m,T0", [(6, 3), (6, 7), (6, 11), (15, 10), (15, 11), (15, 23), (15, 29)])
def test_lemma1_labels_and_active_set(m, T0):
    inst = gen.lemma1_environment(m)
    edges, dist = _dist(inst)
    r, transit = _oracle_at(inst, T0)
    # labels at T0: M - dist where reached
    want = np.where(dist <= T0, inst.M - dist, 0)
    assert np.array_equal(r.labels.astype(np.int64), want.astype(np.int64))
    act, count = _transit_sources(edges, dist, T0)
    assert transit == count
    # the lemma's A_T (section 7, Lemma 1), inside the lattice
    T = T0
    K = (T + 1) // 4
    pts = {(0, T), (0, T - 1)}
    for k in range(1, K + 1):
        pts |= {(-k, T - 2 * k), (k, T - 2 * k)}
    for z in range(-m, m + 1):
        if abs(z) > K:
            pts.add((z, T // 2))
    n = inst.n
    lem = np.zeros(inst.N, bool)
    for (px, py) in pts:
        if -m <= px <= m and 0 <= py < n:
            lem[(px + m) + n * py] = True
    assert (lem & ~act).sum() == 0
    # and the lemma omits some active vertices (reading of section 7)
    if T0 >= 7:
        assert (act & ~lem).sum() > 0


@pytest.mark.parametrize("k,levels", [(4, 1), (4, 4), (5, 3), (6, 6)])
def test_fractal_environment_labels_and_transit(k, levels):
    inst = gen.fractal_environment(k, levels=levels)
    t = 1 << k
    edges, dist = _dist(inst)
    for T0 in (t // 2, t - 1):
        r, transit = _oracle_at(inst, T0)
        want = np.where(dist <= T0, inst.M - dist, 0)
        assert np.array_equal(r.labels.astype(np.int64), want.astype(np.int64))
        assert transit == _transit_sources(edges, dist, T0)[1]
    full = O.solve_instance(inst, want_labels=False)
    assert full.T == t                                  # B = (0, t), up the y-axis
    assert full.counters["U"] == int((dist <= t).sum())  # one improvement per vertex reached by T


@pytest.mark.parametrize("p,seed", [(0.2, 1), (0.5, 2), (0.8, 3)])
def test_binary_environment_vs_recurrence_and_transit(p, seed):
    inst = gen.binary_environment(12, p, seed)
    edges, dist = _dist(inst)
    ref = pins.dp_solve(inst.N, edges, inst.A, inst.B, inst.M)
    r = O.solve_instance(inst, trace_cap=1 << 16)
    assert r.tuple() == (ref["T"], ref["X"], ref["x"], ref["Y"], ref["F2"])
    assert r.counters == ref["counters"]
    assert np.array_equal(r.trace, ref["rows"])
    # every vertex improves exactly once (at its distance), and T is the
    # distance of the top row
    top = inst.B.astype(bool)
    assert r.T == int(dist[top].min())
    assert r.counters["U"] == int((dist <= r.T).sum())
    for T0 in (3, r.T - 1):
        _r, transit = _oracle_at(inst, T0)
        assert transit == _transit_sources(edges, dist, T0)[1]
