"""Independent reference computations that pin the CPU oracle.

None of these share code with the oracle: each computes the problem's plain
definition (section 1 of the paper) a different way.

  L_t(v) = max{ M - F2(pi) : pi a path from A to v, F1(pi) <= t, F2(pi) < M }
           (0 if no such path; M on A)
  T      = least t with L_t(X) > 0 for some X in B (-1 if none)
  X      = the vertex of B with the largest L_T, smallest index on ties
  Y      = the smallest neighbour Y of X with L_{T-f1(Y,X)}(Y) - f2(Y,X) = L_T(X)
  F2     = M - L_T(X)

* ``paths_*``   : enumerate every simple path (tiny graphs).
* ``states_*``  : Dijkstra over the expanded state graph (vertex, quality).
* ``dp_*``      : the time-indexed recurrence
                  L_t(v) = max(L_{t-1}(v), max_u L_{t-f1(u,v)}(u) - f2(u,v)),
                  which also enumerates every flow the cycle sends, so it
                  yields the cycle's counters.
* ``scipy_*``   : textbook Dijkstra (scipy) for the unconstrained and the
                  infeasible special cases.
"""
from __future__ import annotations

import heapq

import numpy as np

from paper_1511_06441_amd import inputs as gen


# ----------------------------------------------------------------------------
# graphs as plain edge lists
# ----------------------------------------------------------------------------

def lattice_edge_list(d, n, f1, f2):
    """Undirected lattice edges as arrays (u, v, f1, f2, eid), built from the
    SoA layout with numpy (no code shared with the oracle)."""
    N = n ** d
    us, vs, w1, w2, ids = [], [], [], [], []
    v_all = np.arange(N, dtype=np.int64)
    for k in range(d):
        c = (v_all // n ** k) % n
        u = v_all[c < n - 1]
        us.append(u)
        vs.append(u + n ** k)
        w1.append(f1[k * N + u].astype(np.int64))
        w2.append(f2[k * N + u].astype(np.int64))
        ids.append(k * N + u)
    return (np.concatenate(us), np.concatenate(vs), np.concatenate(w1),
            np.concatenate(w2), np.concatenate(ids))


def adjacency(nv, edges):
    """adj[u] = sorted list of (v, f1, f2, eid)."""
    us, vs, w1, w2, ids = edges
    adj = [[] for _ in range(nv)]
    for u, v, a, b, e in zip(us.tolist(), vs.tolist(), w1.tolist(), w2.tolist(), ids.tolist()):
        adj[u].append((v, a, b, e))
        adj[v].append((u, a, b, e))
    for lst in adj:
        lst.sort()
    return adj


def edges_from_list(lst):
    """[(u, v, f1, f2), ...] -> edge arrays with eid = position."""
    a = np.array(lst, dtype=np.int64).reshape(-1, 4)
    return a[:, 0], a[:, 1], a[:, 2], a[:, 3], np.arange(len(lst), dtype=np.int64)


def _pick_outputs(adj, Lfun, B, T, M):
    """X, x, Y, F2 from a label oracle Lfun(t, v) at the answer time T."""
    Xs = [v for v in range(len(adj)) if B[v] and Lfun(T, v) > 0]
    X = min(Xs, key=lambda v: (-Lfun(T, v), v))
    LX = Lfun(T, X)
    Y = x = None
    for (y, a, b, e) in adj[X]:
        if T - a >= 0 and Lfun(T - a, y) - b == LX:
            Y, x = y, e
            break
    return X, x, Y, M - LX


# ----------------------------------------------------------------------------
# P1: simple-path enumeration
# ----------------------------------------------------------------------------

def paths_solve(nv, edges, A, B, M):
    """Brute force over all simple paths starting in A.

    Returns (T, X, x, Y, F2, labels_at_T).  Exponential: tiny graphs only.
    """
    adj = adjacency(nv, edges)
    # best[v] = list of (F1, F2) over simple paths from A ending at v
    reach = [[] for _ in range(nv)]

    def dfs(v, F1, F2, seen):
        reach[v].append((F1, F2))
        for (w, a, b, _e) in adj[v]:
            if w not in seen and F2 + b < M:
                seen.add(w)
                dfs(w, F1 + a, F2 + b, seen)
                seen.discard(w)

    for a in range(nv):
        if A[a]:
            dfs(a, 0, 0, {a})

    def Lfun(t, v):
        best = 0
        for (F1, F2) in reach[v]:
            if F1 <= t and F2 < M:
                best = max(best, M - F2)
        return best

    cand = [F1 for v in range(nv) if B[v] for (F1, F2) in reach[v] if F2 < M]
    if not cand:
        Tinf = 1 << 40
        return -1, -1, -1, -1, -1, np.array([Lfun(Tinf, v) for v in range(nv)])
    T = min(cand)
    X, x, Y, F2 = _pick_outputs(adj, Lfun, B, T, M)
    return T, X, x, Y, F2, np.array([Lfun(T, v) for v in range(nv)])


# ----------------------------------------------------------------------------
# P2: Dijkstra over the expanded state graph (vertex, remaining quality)
# ----------------------------------------------------------------------------

def states_dijkstra(nv, edges, A, M):
    """dist[(v, q)] = least time at which water of quality exactly q can be at v."""
    adj = adjacency(nv, edges)
    dist = {}
    heap = [(0, a, M) for a in range(nv) if A[a]]
    heapq.heapify(heap)
    while heap:
        t, v, q = heapq.heappop(heap)
        if (v, q) in dist:
            continue
        dist[(v, q)] = t
        for (w, a, b, _e) in adj[v]:
            q2 = q - b
            if q2 >= 1 and (w, q2) not in dist:
                heapq.heappush(heap, (t + a, w, q2))
    return adj, dist


def states_solve(nv, edges, A, B, M):
    """Returns (T, X, x, Y, F2, labels_at_T, improvements_per_vertex)."""
    adj, dist = states_dijkstra(nv, edges, A, M)
    per_v = [[] for _ in range(nv)]
    for (v, q), t in dist.items():
        per_v[v].append((t, q))
    for lst in per_v:
        lst.sort(key=lambda tq: (tq[0], -tq[1]))

    def Lfun(t, v):
        best = 0
        for (tt, q) in per_v[v]:
            if tt <= t and q > best:
                best = q
        return best

    tB = [t for v in range(nv) if B[v] for (t, q) in per_v[v]]
    T = min(tB) if tB else -1
    horizon = T if T >= 0 else (1 << 40)

    def n_improvements(v):
        best, cnt, last_t = 0, 0, None
        for (t, q) in per_v[v]:
            if t > horizon:
                break
            if q > best:
                best = q
                if t != last_t:
                    cnt += 1
                    last_t = t
        return cnt

    imp = np.array([n_improvements(v) for v in range(nv)], dtype=np.int64)
    labels = np.array([Lfun(horizon, v) for v in range(nv)], dtype=np.int64)
    if T < 0:
        return -1, -1, -1, -1, -1, labels, imp
    X, x, Y, F2 = _pick_outputs(adj, Lfun, B, T, M)
    return T, X, x, Y, F2, labels, imp


# ----------------------------------------------------------------------------
# P3: time-indexed recurrence, with the cycle's counters
# ----------------------------------------------------------------------------

def dp_solve(nv, edges, A, B, M, t_limit=1 << 20):
    """Run L_t for t = 0, 1, ... and enumerate the flows the cycle would send.

    A vertex Q whose label rose at time s (A at s = 0) sends over (Q, P) iff
    L_s(Q) - f2 > L_s(P); the flow arrives at s + f1.  The run stops at the
    answer time T, or when nothing is in transit.

    Returns dict with T, X, x, Y, F2, labels (L_T), counters C U D E R P I.
    """
    us, vs, w1, w2, ids = edges
    # directed copies
    src = np.concatenate([us, vs])
    dst = np.concatenate([vs, us])
    a1 = np.concatenate([w1, w1])
    a2 = np.concatenate([w2, w2])
    deg = np.bincount(src, minlength=nv)
    fmax = int(a1.max()) if a1.size else 1
    Aidx = np.nonzero(A)[0]
    Bm = np.asarray(B).astype(bool)

    hist = []                                   # L_s for every s so far
    L0 = np.zeros(nv, dtype=np.int64)
    L0[Aidx] = M
    hist.append(L0)
    arrivals = {}                               # time -> number of flows arriving
    C = U = D = E = 0
    maxI = 0
    in_transit_by_time = []                     # flows in transit after sending at s
    sent_log = []                               # (send time, arrival time)

    def send(s, Ls, improved):
        nonlocal D, E
        if improved.size == 0:
            return
        D += int(deg[improved].sum())
        mask = np.zeros(nv, dtype=bool)
        mask[improved] = True
        sel = mask[src] & (Ls[src] - a2 > Ls[dst])
        E += int(sel.sum())
        for ta in (s + a1[sel]).tolist():
            arrivals[ta] = arrivals.get(ta, 0) + 1
            sent_log.append((s, ta))

    U += Aidx.size
    send(0, L0, Aidx)
    T = -1
    t = 0
    last_arrival = max(arrivals) if arrivals else 0
    while t < t_limit:
        t += 1
        if t > last_arrival:
            break
        Lt = hist[-1].copy()
        # every edge's contribution: L_{t-f1}(u) - f2 for t - f1 >= 0
        for f in range(1, fmax + 1):
            if t - f < 0:
                break
            sel = a1 == f
            if not sel.any():
                continue
            val = hist[t - f][src[sel]] - a2[sel]
            np.maximum.at(Lt, dst[sel], val)
        Lt = np.maximum(Lt, 0)
        Lt[Aidx] = M
        improved = np.nonzero(Lt > hist[-1])[0]
        hist.append(Lt)
        if arrivals.get(t, 0) > 0:
            C += 1
        U += improved.size
        maxI = max(maxI, improved.size)
        if (Bm[improved]).any():
            T = t
            break
        send(t, Lt, improved)
        if arrivals:
            last_arrival = max(last_arrival, max(arrivals))
    horizon = T if T >= 0 else len(hist) - 1
    R = sum(c for ta, c in arrivals.items() if ta <= horizon)
    # flows in transit right after each sending round s: sent at <= s, arriving > s
    send_rounds = sorted({0} | {ta for ta in arrivals if ta < horizon or T < 0})
    sent_arr = np.array(sent_log, dtype=np.int64).reshape(-1, 2)
    P = 0
    for s in send_rounds:
        if s > horizon or (T >= 0 and s >= T):
            continue
        k = int(((sent_arr[:, 0] <= s) & (sent_arr[:, 1] > s)).sum())
        P = max(P, k)
    out = dict(T=T, labels=hist[horizon].copy(),
               counters=dict(C=C, U=U, D=D, E=E, R=R, P=P, I=maxI))
    if T < 0:
        out.update(X=-1, x=-1, Y=-1, F2=-1)
        return out
    adj = adjacency(nv, edges)

    def Lfun(tt, v):
        return int(hist[tt][v])

    X, x, Y, F2 = _pick_outputs(adj, Lfun, Bm, T, M)
    out.update(X=X, x=x, Y=Y, F2=F2)
    return out


# ----------------------------------------------------------------------------
# P4 / P5: textbook shortest paths (scipy)
# ----------------------------------------------------------------------------

def _csr(nv, edges, weight):
    from scipy.sparse import csr_matrix
    us, vs = edges[0], edges[1]
    w = weight.astype(np.float64)
    rows = np.concatenate([us, vs])
    cols = np.concatenate([vs, us])
    return csr_matrix((np.concatenate([w, w]), (rows, cols)), shape=(nv, nv))


def scipy_multi_source(nv, edges, A, weight):
    from scipy.sparse.csgraph import dijkstra
    g = _csr(nv, edges, weight)
    src = np.nonzero(A)[0]
    d = dijkstra(g, directed=False, indices=src, min_only=True)
    return d


def scipy_unconstrained(nv, edges, A, B):
    """For M above every path weight: T = multi-source Dijkstra on f1; among
    B vertices reached at T, F2 is the lexicographic (f1, f2) optimum."""
    w1, w2 = edges[2], edges[3]
    big = int(w2.sum()) + 1
    dlex = scipy_multi_source(nv, edges, A, w1 * big + w2)
    Bidx = np.nonzero(B)[0]
    lex = np.round(dlex[Bidx]).astype(np.int64)
    T1 = lex // big
    T = int(T1.min())
    cand = Bidx[T1 == T]
    f2s = lex[T1 == T] % big
    j = int(np.argmin(f2s))           # first minimum = smallest index (Bidx ascending)
    return T, int(cand[j]), int(f2s[j])


def scipy_infeasible_labels(nv, edges, A, M):
    """Final labels when no path of weight < M reaches B: max(0, M - dist_f2)."""
    d = scipy_multi_source(nv, edges, A, edges[3])
    lab = np.where(np.isfinite(d), M - d, 0)
    return np.maximum(lab, 0).astype(np.int64), d


# ----------------------------------------------------------------------------
# P6: closed form for f1 == 1 on opposite faces with M > 3 (n-1)
# ----------------------------------------------------------------------------

def straight_line_answer(d, n, f2):
    """With every passage time 1, only straight axis-0 lines reach x = n-1 by
    time n-1.  Returns (T, X, x, Y, F2) in closed form."""
    N = n ** d
    g = f2[:N].reshape((n,) * d).astype(np.int64)      # axis-0 weights [..., c_0]
    sums = g[..., : n - 1].sum(axis=-1).reshape(-1)      # one per line, ascending start index
    j = int(np.argmin(sums))
    X = j * n + (n - 1)
    return n - 1, X, X - 1, X - 1, int(sums[j])
