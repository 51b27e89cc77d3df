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

def _in_slots(nv, edges):
    """Incoming directed edges grouped in slots: slot j holds the j-th
    incoming edge of every vertex that has more than j, so the destinations
    of one slot are distinct.  Each slot: (dst, src, f1, f2) arrays."""
    us, vs, w1, w2, _ids = edges
    src = np.concatenate([us, vs]).astype(np.int64)
    dst = np.concatenate([vs, us]).astype(np.int64)
    a1 = np.concatenate([w1, w1]).astype(np.int64)
    a2 = np.concatenate([w2, w2]).astype(np.int64)
    order = np.lexsort((src, dst))
    src, dst, a1, a2 = src[order], dst[order], a1[order], a2[order]
    first = np.searchsorted(dst, dst, side="left")
    rank = np.arange(dst.size) - first
    slots = []
    for j in range(int(rank.max()) + 1 if rank.size else 0):
        m = rank == j
        slots.append((dst[m], src[m], a1[m], a2[m]))
    deg = np.bincount(src, minlength=nv)
    return slots, deg


def dp_solve(nv, edges, A, B, M, t_limit=1 << 20):
    """Run L_t for t = 0, 1, ... and enumerate the flows the cycle would send.

    A vertex Q whose label rose at time s (A at s = 0) sends over (Q, P) iff
    L_s(Q) - f2 > L_s(P); the flow arrives at s + f1.  The run stops at the
    answer time T, or when nothing is in transit.  Only the last max-f1 + 1
    label vectors are kept, so it scales to lattices of millions of vertices.

    Returns dict with T, X, x, Y, F2, labels (L_T), counters C U D E R P I,
    and rows: one (t, delivered, |I_t|, sent) per time with deliveries.
    """
    us, vs, w1, w2, ids = edges
    slots, deg = _in_slots(nv, edges)
    fmax = max((int(s[2].max()) for s in slots), default=1)
    W = fmax + 1
    Aidx = np.nonzero(A)[0]
    Bm = np.asarray(B).astype(bool)
    # outgoing directed copies, grouped by source (for the sends of I_s)
    osrc = np.concatenate([us, vs]).astype(np.int64)
    odst = np.concatenate([vs, us]).astype(np.int64)
    oa1 = np.concatenate([w1, w1]).astype(np.int64)
    oa2 = np.concatenate([w2, w2]).astype(np.int64)
    order = np.argsort(osrc, kind="stable")
    osrc, odst, oa1, oa2 = osrc[order], odst[order], oa1[order], oa2[order]
    ostart = np.searchsorted(osrc, np.arange(nv + 1))

    ring = np.zeros((W, nv), dtype=np.int64)        # ring[s % W] = L_s
    ring[0, Aidx] = M
    arrive = np.zeros(1024, dtype=np.int64)          # flows arriving at each time
    sent = np.zeros(1024, dtype=np.int64)            # flows sent at each time

    def grow(a, need):
        if need < a.size:
            return a
        b = np.zeros(max(need + 1, 2 * a.size), dtype=np.int64)
        b[:a.size] = a
        return b

    def send(s, Ls, improved):
        """Flows from the vertices of I_s; returns (tests, flows)."""
        nonlocal arrive, sent
        if improved.size == 0:
            return 0, 0
        lo, hi = ostart[improved], ostart[improved + 1]
        cnt = hi - lo
        idx = np.repeat(lo - (np.cumsum(cnt) - cnt), cnt) + np.arange(int(cnt.sum()))
        ok = Ls[osrc[idx]] - oa2[idx] > Ls[odst[idx]]
        ta = s + oa1[idx[ok]]
        if ta.size:
            arrive = grow(arrive, int(ta.max()))
            arrive += np.bincount(ta, minlength=arrive.size)[:arrive.size]
        sent = grow(sent, s)
        sent[s] = int(ok.sum())
        return int(cnt.sum()), int(ok.sum())

    C = D = E = 0
    U = int(Aidx.size)
    maxI = 0
    dd, ee = send(0, ring[0], Aidx)
    D += dd
    E += ee
    rows = []
    T = -1
    t = 0
    while t < t_limit:
        t += 1
        if not arrive[t:].any():
            t -= 1
            break
        prev = ring[(t - 1) % W]
        Lt = prev.copy()
        for (dst, src, a1, a2) in slots:
            ok = a1 <= t
            if not ok.all():
                dst, src, a1, a2 = dst[ok], src[ok], a1[ok], a2[ok]
            val = ring[(t - a1) % W, src] - a2
            Lt[dst] = np.maximum(Lt[dst], val)
        Lt[Aidx] = M
        improved = np.nonzero(Lt > prev)[0]
        ring[t % W] = Lt
        delivered = int(arrive[t]) if t < arrive.size else 0
        if delivered:
            C += 1
        U += int(improved.size)
        maxI = max(maxI, int(improved.size))
        if Bm[improved].any():
            T = t
            if delivered:
                rows.append([t, delivered, int(improved.size), 0])
            break
        dd, ee = send(t, Lt, improved)
        D += dd
        E += ee
        if delivered:
            rows.append([t, delivered, int(improved.size), ee])
    horizon = t
    R = int(arrive[1:horizon + 1].sum())
    # in transit after each sending round s (s = 0 and the cycle times before
    # T): sent at or before s, arriving after s
    tl = max(arrive.size, sent.size)
    cs = np.cumsum(grow(sent, tl)[:tl])
    ca = np.cumsum(grow(arrive, tl)[:tl])
    rounds = [0] + [r[0] for r in rows if T < 0 or r[0] < T]
    P = max(int(cs[s] - ca[s]) for s in rounds)
    out = dict(T=T, labels=ring[horizon % W].copy(),
               counters=dict(C=C, U=U, D=D, E=E, R=R, P=P, I=maxI),
               rows=np.array(rows, dtype=np.int64).reshape(-1, 4))
    if T < 0:
        out.update(X=-1, x=-1, Y=-1, F2=-1)
        return out
    LT = ring[T % W]
    Bidx = np.nonzero(Bm & (LT > 0))[0]
    X = int(Bidx[np.argmax(LT[Bidx])])               # first maximum = smallest index
    LX = int(LT[X])
    # neighbours of X in ascending order: the first that delivers LX at T
    sel = (osrc == X)
    nb = sorted(zip(odst[sel].tolist(), oa1[sel].tolist(), oa2[sel].tolist(),
                    np.concatenate([ids, ids])[order][sel].tolist()))
    Y = x = None
    for (y, a, b, e) in nb:
        if T - a >= 0 and int(ring[(T - a) % W, y]) - b == LX:
            Y, x = y, e
            break
    out.update(X=X, x=int(x), Y=int(Y), F2=M - LX)
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
