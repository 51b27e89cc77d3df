"""Seeded synthetic inputs for lattice constrained-shortest-path instances.

This module is the only code shared by the HIP path, the benchmark and the
CPU oracle's tests.  It draws numbers and builds masks; it holds none of the
method's arithmetic (no labels, no flows, no path sums).

Lattice conventions (the paper treats subgraphs of Z^d with nearest-neighbour
edges, section 1 and section 8):

* N = n**d vertices; vertex v = sum_k c_k * n**k, axis 0 ("x") varies fastest.
* The undirected edge u -- u+e_k has id k*N + u.  Edge arrays are SoA
  ``[d][N]`` uint8; entry (k, u) with c_k(u) == n-1 has no edge and is 0.
* The number of real edges is d * n**(d-1) * (n-1) (section 8 prints this
  count for the 100^3 and 125^3 cubes).

Random numbers: splitmix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  Output i (0-based) of the
stream with state sigma is mix(sigma + (i+1)*gamma), which equals the i-th
output of the sequential generator seeded with sigma.  A value in 1..K is
1 + (((z >> 32) * K) >> 32).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
_C1 = 0xBF58476D1CE4E5B9
_C2 = 0x94D049BB133111EB


def mix64(z: int) -> int:
    """splitmix64 finaliser on one Python int (wraps at 2**64)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * _C1) & MASK64
    z = ((z ^ (z >> 27)) * _C2) & MASK64
    return z ^ (z >> 31)


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * np.uint64(_C1)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(_C2)
    return z ^ (z >> np.uint64(31))


def stream(sigma: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+count-1 of the splitmix64 stream with state sigma."""
    i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64_np(np.uint64(sigma & MASK64) + i * np.uint64(GAMMA))


def stream_at(sigma: int, i: int) -> int:
    """Output i of the stream with state sigma (scalar form of ``stream``)."""
    return mix64((sigma + (i + 1) * GAMMA) & MASK64)


def uniform_int(z: np.ndarray, K: int) -> np.ndarray:
    """Map 64-bit outputs to 1..K by the multiply-high rule."""
    return (np.uint64(1) + (((z >> np.uint64(32)) * np.uint64(K)) >> np.uint64(32)))


def unit_double(z: int) -> float:
    """53-bit uniform double in [0, 1) from one 64-bit output."""
    return float(z >> 11) * (2.0 ** -53)


# ----------------------------------------------------------------------------
# lattice geometry helpers (pure indexing)
# ----------------------------------------------------------------------------

def num_vertices(d: int, n: int) -> int:
    return n ** d


def num_edges(d: int, n: int) -> int:
    return d * n ** (d - 1) * (n - 1)


def _grid(a: np.ndarray, d: int, n: int) -> np.ndarray:
    """View a length-N array as numpy shape (n,)*d indexed [c_{d-1}, ..., c_0]."""
    return a.reshape((n,) * d)


def padding_mask(d: int, n: int) -> np.ndarray:
    """bool [d*N]: True where entry (k, u) has no edge (c_k(u) == n-1)."""
    N = n ** d
    pad = np.zeros(d * N, dtype=bool)
    for k in range(d):
        g = _grid(pad[k * N:(k + 1) * N], d, n)
        idx = [slice(None)] * d
        idx[d - 1 - k] = n - 1
        g[tuple(idx)] = True
    return pad


def face_mask(d: int, n: int, axis: int, coord: int) -> np.ndarray:
    """uint8 [N]: 1 on the face c_axis == coord."""
    m = np.zeros(n ** d, dtype=np.uint8)
    g = _grid(m, d, n)
    idx = [slice(None)] * d
    idx[d - 1 - axis] = coord
    g[tuple(idx)] = 1
    return m


def boundary_mask(d: int, n: int) -> np.ndarray:
    """uint8 [N]: 1 on every vertex with some coordinate equal to 0 or n-1."""
    m = np.zeros(n ** d, dtype=np.uint8)
    g = _grid(m, d, n)
    for ax in range(d):
        for c in (0, n - 1):
            idx = [slice(None)] * d
            idx[ax] = c
            g[tuple(idx)] = 1
    return m


def center_mask(d: int, n: int) -> np.ndarray:
    """uint8 [N]: 1 on the single vertex with every coordinate n//2."""
    m = np.zeros(n ** d, dtype=np.uint8)
    v = sum((n // 2) * n ** k for k in range(d))
    m[v] = 1
    return m


def vertex_index(coords, n: int) -> int:
    """coords = (c_0, c_1, ...) -> linear index."""
    return sum(int(c) * n ** k for k, c in enumerate(coords))


def vertex_coords(v: int, d: int, n: int):
    return tuple((v // n ** k) % n for k in range(d))


# ----------------------------------------------------------------------------
# edge arrays
# ----------------------------------------------------------------------------

def edge_stream_state(seed: int, which: int) -> int:
    """Stream state for f1 (which=1) or f2 (which=2) of instance seed ``seed``."""
    tag = 0xF1 if which == 1 else 0xF2
    return mix64((seed ^ tag) & MASK64)


def lattice_edges(d: int, n: int, seed: int, K1: int, K2: int,
                  f1_const: int | None = None, f2_const: int | None = None,
                  chunk: int = 1 << 23):
    """Return (f1, f2): uint8 SoA [d*N], i.i.d. uniform on 1..K1 / 1..K2.

    Entry i = k*N + v of f1 is draw i of stream edge_stream_state(seed, 1),
    likewise f2 with state edge_stream_state(seed, 2).  A constant overrides
    the draw.  Padding entries are 0.
    """
    if not (1 <= K1 <= 255 and 1 <= K2 <= 255):
        raise ValueError("K must be in 1..255")
    N = n ** d
    total = d * N
    out = []
    for which, K, const in ((1, K1, f1_const), (2, K2, f2_const)):
        f = np.empty(total, dtype=np.uint8)
        if const is not None:
            f[:] = const
        else:
            sigma = edge_stream_state(seed, which)
            for s in range(0, total, chunk):
                c = min(chunk, total - s)
                f[s:s + c] = uniform_int(stream(sigma, c, s), K).astype(np.uint8)
        out.append(f)
    pad = padding_mask(d, n)
    for f in out:
        f[pad] = 0
    return out[0], out[1]


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

@dataclass
class Instance:
    d: int
    n: int
    f1: np.ndarray
    f2: np.ndarray
    A: np.ndarray
    B: np.ndarray
    M: int
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.n ** self.d


def opposite_faces(d: int, n: int, seed: int, K1: int, K2: int, M: int,
                   name: str = "", f1_const=None, f2_const=None) -> Instance:
    f1, f2 = lattice_edges(d, n, seed, K1, K2, f1_const, f2_const)
    return Instance(d, n, f1, f2, face_mask(d, n, 0, 0), face_mask(d, n, 0, n - 1), M,
                    name=name, meta=dict(seed=seed, K1=K1, K2=K2))


def square64(seed: int = 1, M: int = 200) -> Instance:
    """2-D 64x64, f1,f2 uniform 1..5, A = column x=0, B = column x=63."""
    return opposite_faces(2, 64, seed, 5, 5, M, name=f"square64_s{seed}_M{M}")


def cube128(seed: int = 11, M: int = 700) -> Instance:
    """3-D 128^3, f1,f2 uniform 1..10, A = face x=0, B = face x=127."""
    return opposite_faces(3, 128, seed, 10, 10, M, name=f"cube128_s{seed}_M{M}")


def cube256(seed: int = 21, M: int = 10000) -> Instance:
    """3-D 256^3, f1,f2 uniform 1..100 (long edge timers), faces x=0 / x=255."""
    return opposite_faces(3, 256, seed, 100, 100, M, name=f"cube256_s{seed}_M{M}")


def cube256_stress(seed: int = 22, M: int = 10000) -> Instance:
    """3-D 256^3, f1 == 1, f2 uniform 1..3 (thick, BFS-like frontier)."""
    return opposite_faces(3, 256, seed, 1, 3, M, name=f"cube256stress_s{seed}_M{M}",
                          f1_const=1)


def cube_boundary_to_center(n: int, seed: int, K: int = 100, M: int = 10000) -> Instance:
    """3-D n^3 with water on the cube boundary and B the centre (section 8's runs)."""
    f1, f2 = lattice_edges(3, n, seed, K, K)
    return Instance(3, n, f1, f2, boundary_mask(3, n), center_mask(3, n), M,
                    name=f"cube{n}_boundary_s{seed}", meta=dict(seed=seed, K1=K, K2=K))


# ----------------------------------------------------------------------------
# the environments of section 7 (passage times in {1, 2})
# ----------------------------------------------------------------------------

def _unit_weights_plane(m: int):
    """A (2m+1) x (2m+1) square standing for [-m, m] x [0, 2m]: vertex
    (x, y) is index (x + m) + (2m+1) y.  Returns (n, f1) with every edge at 2
    (padding 0) and a setter for single edges."""
    n = 2 * m + 1
    N = n * n
    f1 = np.full(2 * N, 2, dtype=np.uint8)
    f1[padding_mask(2, n)] = 0
    return n, N, f1


def _mark_edge(f1, n, N, a, b, value=1):
    """Set f1 of the lattice edge joining plane points a and b (unit step)."""
    (xa, ya), (xb, yb) = a, b
    m = (n - 1) // 2
    if ya == yb and abs(xa - xb) == 1:
        x0 = min(xa, xb)
        if -m <= x0 < m and 0 <= ya < n:
            f1[0 * N + (x0 + m) + n * ya] = value
    elif xa == xb and abs(ya - yb) == 1:
        y0 = min(ya, yb)
        if -m <= xa <= m and 0 <= y0 < n - 1:
            f1[1 * N + (xa + m) + n * y0] = value
    else:
        raise ValueError("not a unit step")


def _staircase(p, q):
    """Lattice points of a monotone staircase from p to q (integer points)
    that stays within half a step of the straight segment pq."""
    (x0, y0), (x1, y1) = p, q
    dx, dy = x1 - x0, y1 - y0
    sx, sy = (1 if dx > 0 else -1), (1 if dy > 0 else -1)
    ax, ay = abs(dx), abs(dy)
    pts = [(x0, y0)]
    x, y, i, j = x0, y0, 0, 0
    while i < ax or j < ay:
        # step in the direction whose next point lies closer to the segment
        if j == ay or (i < ax and (2 * i + 1) * ay < (2 * j + 1) * ax):
            x += sx
            i += 1
        else:
            y += sy
            j += 1
        pts.append((x, y))
    return pts


def lemma1_environment(m: int, M: int | None = None) -> Instance:
    """Section 7, Lemma 1: on [-m, m] x [0, 2m] every edge of the y-axis has
    passage time 1 and every other edge 2; water starts on the whole x-axis.
    The lemma takes M infinite: here f2 = f1 and M exceeds every path weight,
    so a label is M minus the first arrival time.  B is the top of the
    y-axis, (0, 2m), reached at T = 2m."""
    n, N, f1 = _unit_weights_plane(m)
    for y in range(n - 1):
        _mark_edge(f1, n, N, (0, y), (0, y + 1))
    f2 = f1.copy()
    A = np.zeros(N, np.uint8)
    A[:n] = 1
    B = np.zeros(N, np.uint8)
    B[m + n * (n - 1)] = 1
    M = M if M is not None else 2 * N + 1
    return Instance(2, n, f1, f2, A, B, M, name=f"lemma1_m{m}", meta=dict(m=m))


def fractal_environment(k: int, M: int | None = None, levels: int | None = None) -> Instance:
    """Section 7, Theorem 2's construction at t = 2^k: the y-axis and the
    segment LO (L = (-t/2, 0), O = (0, t/2), T = (0, t)) get passage time 1,
    then k-1 times every triangle (L, O, T) of the current set gets time 1 on
    L0 X and T0 X (L0, T0 the midpoints of LO and TO, X the midpoint of LT)
    and is replaced by (L, L0, X) and (X, T0, T); the whole is mirrored in
    the y-axis.  Segments are laid on the lattice as monotone staircases.
    Every other edge has time 2; f2 = f1, M above every path weight, water
    starts on the x-axis and B is T.  The lattice is [-t, t] x [0, 2t].
    `levels` (1..k, default k) stops the refinement early: omega_levels."""
    t = 1 << k
    levels = k if levels is None else levels
    if not 1 <= levels <= k:
        raise ValueError("levels must be in 1..k")
    m = t
    n, N, f1 = _unit_weights_plane(m)
    marked = set()

    def seg(p, q):
        pts = _staircase((round(p[0]), round(p[1])), (round(q[0]), round(q[1])))
        for a, b in zip(pts[:-1], pts[1:]):
            for sgn in (1, -1):
                marked.add(((sgn * a[0], a[1]), (sgn * b[0], b[1])))

    for y in range(t):
        marked.add(((0, y), (0, y + 1)))
    L, O, T = (-t / 2, 0.0), (0.0, t / 2), (0.0, float(t))
    seg(L, O)
    tris = [(L, O, T)]

    def mid(a, b):
        return ((a[0] + b[0]) / 2, (a[1] + b[1]) / 2)

    for _ in range(levels - 1):
        nxt = []
        for (l, o, tt) in tris:
            l0, t0, x = mid(l, o), mid(tt, o), mid(l, tt)
            seg(l0, x)
            seg(t0, x)
            nxt += [(l, l0, x), (x, t0, tt)]
        tris = nxt
    for a, b in marked:
        _mark_edge(f1, n, N, a, b)
    f2 = f1.copy()
    A = np.zeros(N, np.uint8)
    A[:n] = 1
    B = np.zeros(N, np.uint8)
    B[m + n * t] = 1
    M = M if M is not None else 2 * N + 1
    return Instance(2, n, f1, f2, A, B, M, name=f"fractal_k{k}_l{levels}", meta=dict(k=k, t=t, levels=levels))


def binary_environment(m: int, p: float, seed: int, M: int | None = None) -> Instance:
    """Section 7's random environment: on [-m, m] x [0, 2m] every edge has
    passage time 1 with probability p and 2 otherwise, independently (draw
    i of stream edge_stream_state(seed, 1) over the SoA index, 1 when its top
    53 bits as a fraction fall below p).  f2 = f1 and M above every path
    weight (the section's M = infinity); water starts on the x-axis and B is
    the top row."""
    n, N, f1 = _unit_weights_plane(m)
    z = stream(edge_stream_state(seed, 1), 2 * N)
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    pad = f1 == 0
    f1 = np.where(u < p, 1, 2).astype(np.uint8)
    f1[pad] = 0
    f2 = f1.copy()
    A = np.zeros(N, np.uint8)
    A[:n] = 1
    B = np.zeros(N, np.uint8)
    B[n * (n - 1):] = 1
    M = M if M is not None else 2 * N + 1
    return Instance(2, n, f1, f2, A, B, M, name=f"binary_m{m}_p{p}_s{seed}", meta=dict(m=m, p=p, seed=seed))


def _round_half_up(x: float) -> int:
    return int(math.floor(x + 0.5))


def mixed_params(master: int, j: int, lo2=(32, 512), lo3=(16, 160)):
    """Parameters (seed, d, n, K, M) of instance j of a mixed batch.

    s_j is output j of the stream with state ``master``; outputs g0..g3 of the
    stream with state s_j give d, n (log-uniform), K (3..50) and
    M = round((1.5 + 2.5 u') * n * (K+1) / 2).
    """
    s = stream_at(master, j)
    g0, g1, g2, g3 = (stream_at(s, i) for i in range(4))
    d = 2 + (g0 >> 63)
    lo, hi = lo2 if d == 2 else lo3
    u = unit_double(g1)
    n = _round_half_up(lo * (hi / lo) ** u)
    K = 3 + (((g2 >> 32) * 48) >> 32)
    u2 = unit_double(g3)
    M = _round_half_up((1.5 + 2.5 * u2) * n * (K + 1) / 2)
    return s, int(d), int(n), int(K), int(M)


def mixed_instance(master: int, j: int, lo2=(32, 512), lo3=(16, 160)) -> Instance:
    s, d, n, K, M = mixed_params(master, j, lo2, lo3)
    inst = opposite_faces(d, n, s, K, K, M, name=f"mixed{master}_{j}")
    inst.meta.update(K=K, j=j)
    return inst


def batch_params(count: int = 1024, master: int = 41):
    """Mixed batch: d in {2,3}, n log-uniform in [32,512] (2-D) / [16,160] (3-D)."""
    return [mixed_params(master, j) for j in range(count)]


def serving_params(count: int, master: int = 51):
    """Serving mix: sides log-uniform 64..1024 (2-D) and 32..256 (3-D)."""
    return [mixed_params(master, j, (64, 1024), (32, 256)) for j in range(count)]


def poisson_arrivals(count: int, qps: float, seed: int = 52) -> np.ndarray:
    """Arrival times (s) of a Poisson stream: exponential gaps from stream ``seed``."""
    z = stream(mix64(seed), count)
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    gaps = -np.log1p(-u) / qps
    return np.cumsum(gaps)


# ----------------------------------------------------------------------------
# the same draws, generated on a torch device (for large workloads)
# ----------------------------------------------------------------------------

def _i64(v: int) -> int:
    """Two's-complement int64 value of a 64-bit pattern."""
    v &= MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def _shr(z, k):
    """Logical right shift of int64 tensors holding 64-bit patterns."""
    return (z >> k) & ((1 << (64 - k)) - 1)


def _mix64_t(z):
    z = (z ^ _shr(z, 30)) * _i64(_C1)
    z = (z ^ _shr(z, 27)) * _i64(_C2)
    return z ^ _shr(z, 31)


def lattice_edges_torch(d: int, n: int, seed: int, K1: int, K2: int, device="cuda",
                        f1_const=None, f2_const=None, chunk: int = 1 << 24):
    """Same arrays as ``lattice_edges`` (bit for bit), built with torch on ``device``."""
    import torch
    N = n ** d
    total = d * N
    out = []
    for which, K, const in ((1, K1, f1_const), (2, K2, f2_const)):
        f = torch.empty(total, dtype=torch.uint8, device=device)
        if const is not None:
            f.fill_(const)
        else:
            sigma = _i64(edge_stream_state(seed, which))
            for s0 in range(0, total, chunk):
                c = min(chunk, total - s0)
                i = torch.arange(s0 + 1, s0 + c + 1, dtype=torch.int64, device=device)
                z = _mix64_t(sigma + i * _i64(GAMMA))
                f[s0:s0 + c] = (1 + ((_shr(z, 32) * K) >> 32)).to(torch.uint8)
        out.append(f)
    # zero the padding entries: (k, u) with c_k(u) == n-1
    for f in out:
        for k in range(d):
            g = f[k * N:(k + 1) * N].view(*([n] * d))
            idx = [slice(None)] * d
            idx[d - 1 - k] = n - 1
            g[tuple(idx)] = 0
    return out[0], out[1]


def face_mask_torch(d: int, n: int, axis: int, coord: int, device="cuda"):
    import torch
    m = torch.zeros((n,) * d, dtype=torch.uint8, device=device)
    idx = [slice(None)] * d
    idx[d - 1 - axis] = coord
    m[tuple(idx)] = 1
    return m.reshape(-1)


# ----------------------------------------------------------------------------
# general graphs (adjacency lists)
# ----------------------------------------------------------------------------

def graph_csr(nv: int, us, vs, f1, f2, ids=None):
    """Adjacency arrays of an undirected graph from its edge list: both
    directions of every edge, neighbours of each vertex in ascending order
    (ties by edge id), edge id = position in the list unless given.
    Returns off int64 [nv+1], nbr int32, f1 uint8, f2 uint8, eid int64."""
    us = np.asarray(us, dtype=np.int64)
    vs = np.asarray(vs, dtype=np.int64)
    f1 = np.asarray(f1, dtype=np.uint8)
    f2 = np.asarray(f2, dtype=np.uint8)
    ids = np.arange(us.size, dtype=np.int64) if ids is None else np.asarray(ids, dtype=np.int64)
    src = np.concatenate([us, vs])
    dst = np.concatenate([vs, us])
    a1 = np.concatenate([f1, f1])
    a2 = np.concatenate([f2, f2])
    e = np.concatenate([ids, ids])
    order = np.lexsort((e, dst, src))
    src, dst, a1, a2, e = src[order], dst[order], a1[order], a2[order], e[order]
    off = np.zeros(nv + 1, dtype=np.int64)
    np.add.at(off, src + 1, 1)
    off = np.cumsum(off)
    return off, dst.astype(np.int32), a1, a2, e


def random_graph(nv: int, seed: int, K1: int, K2: int, max_deg: int = 6, chords: int = 2):
    """A connected bounded-degree graph: a path 0-1-...-(nv-1) plus `chords`
    random chords per vertex (skipped when they would exceed max_deg or
    repeat an edge).  f1, f2 i.i.d. uniform on 1..K from the same streams as
    the lattices.  Returns (us, vs, f1, f2) as arrays."""
    z = stream(mix64(seed ^ 0xC0), nv * chords)
    deg = np.zeros(nv, dtype=np.int64)
    seen = set()
    us, vs = [], []
    for u in range(nv - 1):
        us.append(u)
        vs.append(u + 1)
        seen.add((u, u + 1))
        deg[u] += 1
        deg[u + 1] += 1
    for k in range(nv * chords):
        u = k // chords
        v = int(z[k] % np.uint64(nv))
        a, b = min(u, v), max(u, v)
        if a == b or (a, b) in seen or deg[a] >= max_deg or deg[b] >= max_deg:
            continue
        seen.add((a, b))
        us.append(a)
        vs.append(b)
        deg[a] += 1
        deg[b] += 1
    m = len(us)
    f1 = uniform_int(stream(mix64(seed ^ 0xF1), m), K1).astype(np.uint8)
    f2 = uniform_int(stream(mix64(seed ^ 0xF2), m), K2).astype(np.uint8)
    return np.array(us, dtype=np.int64), np.array(vs, dtype=np.int64), f1, f2
