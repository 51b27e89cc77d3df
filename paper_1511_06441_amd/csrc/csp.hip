// csp.hip -- libcsp: the water-flow constrained-shortest-path cycle on
// lattice cubes in Z^d, written for MI355X (gfx950, CDNA4, wave64).
//
// Method: I. Matic, "A parallel algorithm for the constrained shortest path
// problem on lattice graphs" (arXiv:1511.06441), sections 4-6,
// Algorithms 1-11.  The paper keeps per-edge records (time remaining,
// source, state) plus a separate phantom list and runs nine barrier-separated
// steps per time unit.  Here every unit of water in transit is a flow record
// (destination, quality, arriving direction) filed in a timing wheel by its
// arrival time, so regular and phantom edges are the same thing, and Step 1's
// time skip is the first non-empty bucket after t.  A cycle is:
//
//   arrival   (Steps 1-3, 8): deliver the bucket of time t; raise each
//             destination's label to the best quality delivered; the vertices
//             whose label rose form the improved set I_t.  A vertex of B in
//             I_t ends the run (Step 6).
//   departure (Steps 4-5): every Q in I_t tests its 2d lattice neighbours;
//             if Label(Q) - f2 > Label(P), a flow (P, Label(Q) - f2) is filed
//             in bucket (t + f1) mod W.  Delivered flows simply leave their
//             bucket (Steps 7, 9).
//
// Two single-solve kernels, chosen per problem:
//
//  * k_ranges (range-owned, the usual one).  The lattice is cut into g
//    contiguous index ranges, one per workgroup; ranges of one XCD are
//    contiguous.  A workgroup keeps its range's labels (16 or 32 bits), the
//    frontier bitmap, the B bitmap and the wheel fill counts in LDS and owns
//    its own wheel in HBM, so every label test, delivery and commit is an
//    LDS operation and the wheel needs no device-wide counter.  A neighbour
//    test whose target lies in another range is shipped to the owner as a
//    candidate (local index, f1, direction, quality) and tested there after
//    the next barrier against labels that are still those of the sending
//    time.  One combining barrier per cycle (a two-level tree, one group per
//    XCD, one release line per member) returns the next event time, flags,
//    counts and the best B key.
//  * k_solve (global labels, for lattices whose ranges do not fit LDS).
//    Label words in HBM pack (label << 2) | inB << 1 | idle; a delivery is one
//    atomicMax that raises the label and elects the first improver; frontier
//    segments are balanced by an LDS prefix sum; two grid barriers per cycle.
//
// k_batch runs many range-owned solves in one persistent launch (a gang of
// workgroups per problem) and k_serve keeps such workers alive while a host
// feeds them requests, including the reconstruction chain of section 1 and section 5 ("Termination").
//
// Measured on MI355X, and the reason for the shapes above: device atomics on
// one address serialise at ~11 ns each; scattered atomicMax reaches ~27 G/s;
// a grid barrier costs several microseconds and grows with the number of
// participants and with the dirty data each must write back.
//
// All arithmetic is integer; results are bit-identical to the CPU oracle.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "csp.h"

namespace {

constexpr int BLOCK = 1024;
constexpr int NWAVES = BLOCK / 64;
constexpr int MAXW = 256;          // f1 <= 255, so 256 buckets always suffice
constexpr int GMAX = 512;          // workgroups per launch
constexpr int NGRP = 8;            // barrier groups (one per XCD)
constexpr unsigned IDLE = 1u;
constexpr unsigned INB = 2u;
constexpr unsigned QB_INB = 0x80000000u;   // frontier entry: vertex is in B

// slot flags
constexpr unsigned SF_BHIT = 1u << 31;
constexpr unsigned SF_OVER = 1u << 30;
constexpr unsigned SF_INVAL = 1u << 29;
constexpr unsigned SF_MASK = 0x1FFFFFFFu;

// Per-instance outputs of a range-owned solve.
struct Out {
    long long res[5];              // T X x Y F2
    unsigned long long ctr[8];     // C U D E R P I
    unsigned long long prof[8];    // wall-clock ticks per phase (range 0)
    unsigned long long psum[8];    // per-phase ticks summed over ranges (phase timing 2)
    unsigned long long pmax[8];    // per-phase ticks, largest range (phase timing 2)
    long long trace_rows;          // cycle rows produced (may exceed the trace capacity)
    long long xrec;                // improvement record of X at T (logging runs)
    int status;
    int log_over;                  // the improvement log ran out (logging runs)
};

// State of one combining barrier among the g workgroups of a gang; the
// header is followed by g member slot lines and g flag lines (16 x u64 each).
struct BarHdr {
    unsigned grp[NGRP][32];        // group counters, one per 128-byte line
    unsigned root[32];
    unsigned long long gslot[NGRP][16];
    unsigned long long res[2][16]; // sums and maximum of the last two barriers
    int broken;
    int pad[31];
    // gang_or (the cycle loop's barrier): arrival words of the groups and of
    // the root by barrier parity (word 0 of each line), per-barrier sums for
    // member 0 (words 0-2 of a ring of four lines) and the best B key
    unsigned long long ow[2][16][16];
    unsigned long long oroot[2][16];
    unsigned long long ring[4][16][3][16];   // [barrier & 3][group][sum] (word 0 of each line)
    unsigned long long bkey[16];
};

__host__ __device__ inline size_t bar_bytes(unsigned g) { return sizeof(BarHdr) + (size_t)2 * g * 128; }

struct Ctl {
    unsigned grp[NGRP][32];        // barrier group counters, one per 128-byte line
    unsigned root[32];
    unsigned flag[GMAX][32];       // per-workgroup release flags
    unsigned qslot[GMAX];          // arrival: frontier size | flags
    unsigned nslot[GMAX];          // departure: next delta (0 = none) | flags
    unsigned tslot[GMAX];          // departure: flows in transit
    unsigned long long xkey;
    unsigned ydir;
    unsigned bad;                  // set by the packing kernel
    unsigned maxf1;
    unsigned pad0;
    unsigned long long ctr[8];     // C U D E R P I
    long long res[5];              // T X x Y F2
    unsigned long long prof[8];    // wall-clock ticks per phase (workgroup 0)
    int status;
    int broken;
    // range-owned solves
    Out rout;
    BarHdr rbar;
    unsigned long long rbar_lines[2 * GMAX][16];
};

enum { ST_RUNNING = 0, ST_DONE = 1, ST_OVERFLOW = 2, ST_CANCELED = 3, ST_BROKEN = 4, ST_INVAL = 5 };

struct Params {
    long long N;
    long long off[8];              // neighbour offset per direction
    const void *rec;               // packed (f1, f2) per vertex and direction
    const uint8_t *A, *B;
    unsigned M;
    unsigned qs;                   // frontier capacity per workgroup
    unsigned long long pool_flows; // total wheel capacity in flows
    unsigned *lab;
    unsigned *queue;               // [G][qs]
    uint2 *pool;
    Ctl *ctl;
    unsigned *labels_out;
    long long max_cycles;
    unsigned long long wait_limit; // wall-clock ticks a barrier wait may take
    int prof;                      // record per-phase time of workgroup 0
};

// record type per dimension: 2d (f1, f2) byte pairs
template <int D> struct Rec;
template <> struct Rec<1> { using T = uint32_t; };
template <> struct Rec<2> { using T = uint2; };
template <> struct Rec<3> { using T = uint4; };
template <> struct Rec<4> { using T = uint4; };

template <int D>
__device__ __forceinline__ void rec_get(const typename Rec<D>::T &r, int dir, unsigned &a1, unsigned &a2)
{
    unsigned w;
    if constexpr (D == 1) {
        w = r;
    } else if constexpr (D == 2) {
        w = dir < 2 ? r.x : r.y;
    } else {
        const int q = dir >> 1;
        w = q == 0 ? r.x : (q == 1 ? r.y : (q == 2 ? r.z : r.w));
    }
    const unsigned sh = (dir & 1) ? 16u : 0u;
    const unsigned pr = (D == 1) ? (w >> (16u * dir)) : (w >> sh);
    a1 = pr & 0xFFu;
    a2 = (pr >> 8) & 0xFFu;
}

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ unsigned ld_rlx(const unsigned *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_rlx(unsigned *p, unsigned v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// Two-level tree barrier over a cooperative grid.  Thread 0 of each
// workgroup publishes the group's writes with an agent-scope release fence
// and counts itself in its XCD group; the last arriver of a group counts the
// group at the root; the last group releases every workgroup by writing the
// new epoch into its private flag line.  Waiters spin on their own flag and
// finish with an acquire fence.  Every wait is bounded by `limit` wall-clock
// ticks; on expiry the run is marked broken and the call returns false, so a
// logic error drains the grid instead of hanging it.
__device__ bool grid_sync(Ctl *ctl, unsigned &epoch, unsigned long long limit)
{
    __shared__ int s_ok;
    __syncthreads();
    ++epoch;
    const unsigned G = gridDim.x;
    if (G == 1) return true;
    if (threadIdx.x < 64) {
        int releaser = 0;
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const unsigned grp = blockIdx.x % NGRP;
            const unsigned ngrp = G < NGRP ? G : NGRP;
            const unsigned members = (G - grp + NGRP - 1) / NGRP;
            const unsigned a = __hip_atomic_fetch_add(&ctl->grp[grp][0], 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            if (a == members - 1) {
                st_rlx(&ctl->grp[grp][0], 0u);
                const unsigned r = __hip_atomic_fetch_add(&ctl->root[0], 1u, __ATOMIC_ACQ_REL,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                if (r == ngrp - 1) {
                    st_rlx(&ctl->root[0], 0u);
                    releaser = 1;
                }
            }
        }
        releaser = __shfl(releaser, 0);
        if (releaser) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            for (unsigned i = threadIdx.x; i < G; i += 64) st_rlx(&ctl->flag[i][0], epoch);
        }
        if (threadIdx.x == 0) {
            int ok = 1;
            const unsigned long long t0 = wall_clock64();
            while (ld_rlx(&ctl->flag[blockIdx.x][0]) < epoch) {
                __builtin_amdgcn_s_sleep(1);
                if (wall_clock64() - t0 > limit) {
                    __hip_atomic_store(&ctl->broken, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (__hip_atomic_load(&ctl->broken, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
            s_ok = ok;
        }
    }
    __syncthreads();
    return s_ok != 0;
}

// Exclusive prefix sum over one value per thread (BLOCK threads); returns
// the exclusive prefix and writes the total to *total (all threads).
__device__ unsigned block_scan(unsigned v, unsigned *s_wave, unsigned *total)
{
    const unsigned lane = lane_id(), wv = threadIdx.x >> 6;
    unsigned x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned y = __shfl_up(x, o);
        if (lane >= (unsigned)o) x += y;
    }
    if (lane == 63) s_wave[wv] = x;
    __syncthreads();
    if (wv == 0) {
        unsigned w = lane < NWAVES ? s_wave[lane] : 0u;
#pragma unroll
        for (int o = 1; o < NWAVES; o <<= 1) {
            const unsigned y = __shfl_up(w, o);
            if (lane >= (unsigned)o) w += y;
        }
        if (lane < NWAVES) s_wave[lane] = w;      // inclusive wave totals
    }
    __syncthreads();
    const unsigned before = wv ? s_wave[wv - 1] : 0u;
    *total = s_wave[NWAVES - 1];
    const unsigned r = before + x - v;
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Clear the control block (a kernel rather than a memset, so the sequence
// stays valid inside captured graphs).
__global__ void __launch_bounds__(BLOCK) k_reset_ctl(Ctl *ctl)
{
    unsigned *w = reinterpret_cast<unsigned *>(ctl);
    for (unsigned i = threadIdx.x; i < sizeof(Ctl) / 4; i += BLOCK) w[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) ctl->ydir = 0xFFFFFFFFu;
}

// Repack SoA edge arrays into per-vertex records of 2d (f1, f2) pairs in
// direction order (-n^(d-1) .. -1, +1 .. +n^(d-1)); zero where no edge.
// Also checks that every real edge has positive f1 and f2 and records the
// largest f1 (it sizes the timing wheel).
template <int D>
__global__ void __launch_bounds__(256) k_pack(long long n, long long N, const uint8_t *f1,
                                              const uint8_t *f2, typename Rec<D>::T *rec, Ctl *ctl)
{
    const long long gs = (long long)gridDim.x * blockDim.x;
    unsigned bad = 0, mx = 0;
    long long stride[D];
    {
        long long s = 1;
        for (int k = 0; k < D; ++k) {
            stride[k] = s;
            s *= n;
        }
    }
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += gs) {
        long long c[D];
        long long rem = v;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            c[k] = rem % n;
            rem /= n;
        }
        unsigned pr[2 * D];
#pragma unroll
        for (int dir = 0; dir < 2 * D; ++dir) {
            const bool lower = dir < D;
            const int k = lower ? D - 1 - dir : dir - D;
            const bool exists = lower ? (c[k] >= 1) : (c[k] <= n - 2);
            pr[dir] = 0;
            if (exists) {
                const long long e = (long long)k * N + (lower ? v - stride[k] : v);
                const unsigned a = f1[e], b = f2[e];
                if (a == 0 || b == 0) bad = 1;
                mx = a > mx ? a : mx;
                pr[dir] = a | (b << 8);
            }
        }
        typename Rec<D>::T r;
        if constexpr (D == 1) {
            r = pr[0] | (pr[1] << 16);
        } else if constexpr (D == 2) {
            r = make_uint2(pr[0] | (pr[1] << 16), pr[2] | (pr[3] << 16));
        } else if constexpr (D == 3) {
            r = make_uint4(pr[0] | (pr[1] << 16), pr[2] | (pr[3] << 16), pr[4] | (pr[5] << 16), 0u);
        } else {
            r = make_uint4(pr[0] | (pr[1] << 16), pr[2] | (pr[3] << 16), pr[4] | (pr[5] << 16),
                           pr[6] | (pr[7] << 16));
        }
        rec[v] = r;
    }
    for (int o = 32; o > 0; o >>= 1) {
        bad |= __shfl_xor(bad, o);
        mx = max(mx, (unsigned)__shfl_xor(mx, o));
    }
    if (lane_id() == 0) {
        if (bad) atomicOr(&ctl->bad, 1u);
        if (mx) atomicMax(&ctl->maxf1, mx);
    }
}

template <int D>
__global__ void __launch_bounds__(BLOCK) k_solve(Params p)
{
    using RT = typename Rec<D>::T;
    __shared__ unsigned s_cnt[MAXW];           // this workgroup's fill per bucket
    __shared__ unsigned s_pref[GMAX + 1];      // frontier prefix sums over workgroups
    __shared__ unsigned s_wave[NWAVES];
    __shared__ unsigned s_qn;                  // this workgroup's frontier fill
    __shared__ unsigned s_flags;
    __shared__ unsigned s_min;
    __shared__ unsigned long long s_red[4];

    Ctl *ctl = p.ctl;
    const unsigned tid = threadIdx.x, lane = lane_id();
    const unsigned g = blockIdx.x, G = gridDim.x;
    const bool lead = g == 0;
    const long long N = p.N;
    const RT *rec = static_cast<const RT *>(p.rec);
    unsigned epoch = 0;

    unsigned W = 2;
    while (W <= ctl->maxf1) W <<= 1;
    const unsigned Wm = W - 1;
    const unsigned long long S = p.pool_flows / ((unsigned long long)W * G);   // flows per segment
    const unsigned QS = p.qs;
    unsigned *myq = p.queue + (unsigned long long)g * QS;

    unsigned long long cU = 0, cD = 0, cE = 0, cR = 0;      // per thread
    unsigned long long cC = 0, cP = 0, cI = 0;              // lead workgroup, thread 0
    // phase clock of workgroup 0: departure, departure barrier, next time,
    // arrival, arrival barrier, frontier gather
    unsigned long long ph[6] = {0, 0, 0, 0, 0, 0}, ph_t = 0;
    const bool timing = p.prof && lead && tid == 0;
#define PHASE(k)                                         \
    do {                                                 \
        if (timing) {                                    \
            const unsigned long long now_ = wall_clock64(); \
            ph[k] += now_ - ph_t;                        \
            ph_t = now_;                                 \
        }                                                \
    } while (0)

    for (unsigned i = tid; i < MAXW; i += BLOCK) s_cnt[i] = 0;
    if (tid == 0) {
        s_qn = 0;
        s_flags = 0;
        for (int i = 0; i < 4; ++i) s_red[i] = 0;
    }
    __syncthreads();

    int status = ST_RUNNING;
    if (ctl->bad) status = ST_INVAL;                       // read by every workgroup alike

    // ---- Initialization (Algorithm 3): Label = M on A, 0 elsewhere; A is I_0.
    if (status == ST_RUNNING) {
        const long long chunk = (N + G - 1) / G;
        const long long lo = (long long)g * chunk, hi = min(N, lo + chunk);
        for (long long v = lo + tid; v < hi; v += BLOCK) {
            const bool a = p.A[v] != 0, b = p.B[v] != 0;
            if (a && b) atomicOr(&s_flags, SF_INVAL);
            p.lab[v] = (a ? (p.M << 2) : 0u) | (b ? INB : 0u) | IDLE;
            const unsigned long long m = __ballot(a);
            if (m) {
                const int ld = __ffsll((long long)m) - 1;
                unsigned base = 0;
                if ((int)lane == ld) base = atomicAdd(&s_qn, (unsigned)__popcll(m));
                base = __shfl(base, ld);
                const unsigned slot = base + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
                if (a) myq[slot] = (unsigned)v;                   // chunk <= QS
            }
        }
        __syncthreads();
        if (tid == 0) st_rlx(&ctl->qslot[g], s_qn | s_flags);
    }
    if (status == ST_RUNNING && !grid_sync(ctl, epoch, p.wait_limit)) status = ST_BROKEN;

    long long t = 0;
    unsigned cyc = 0;
    unsigned bucket_n = 0;      // flows this workgroup delivered in the last arrival
    unsigned b_cur = 0;
    unsigned Qtot = 0;

    // frontier sizes -> prefix sums (every workgroup computes the same)
    auto gather_frontier = [&](unsigned &flags) {
        const unsigned raw = tid < G ? ld_rlx(&ctl->qslot[tid]) : 0u;
        const unsigned v = raw & SF_MASK;
        const unsigned fl = __syncthreads_or((int)(raw & ~SF_MASK)) ? 1u : 0u;
        unsigned any = 0;
        if (fl) {
            if (tid == 0) s_min = 0;
            __syncthreads();
            if (raw & ~SF_MASK) atomicOr(&s_min, raw & ~SF_MASK);
            __syncthreads();
            any = s_min;
            __syncthreads();
        }
        unsigned total;
        const unsigned ex = block_scan(v, s_wave, &total);
        if (tid < G) s_pref[tid] = ex;
        if (tid == 0) s_pref[G] = total;
        __syncthreads();
        flags = any;
        return total;
    };

    if (status == ST_RUNNING) {
        unsigned fl;
        Qtot = gather_frontier(fl);
        if (fl & SF_INVAL) status = ST_INVAL;
        cU += (g == 0 && tid == 0) ? Qtot : 0;
    }

    if (timing) ph_t = wall_clock64();
    while (status == ST_RUNNING) {
        // ---- Departure (Steps 4-5, Algorithms 7-8): an equal slice of I_t.
        {
            const unsigned lo = (unsigned)(((unsigned long long)Qtot * g) / G);
            const unsigned hi = (unsigned)(((unsigned long long)Qtot * (g + 1)) / G);
            for (unsigned i = lo + tid; i < hi; i += BLOCK) {
                // segment s with s_pref[s] <= i < s_pref[s+1]
                unsigned a = 0, b = G;
                while (b - a > 1) {
                    const unsigned m = (a + b) >> 1;
                    if (s_pref[m] <= i) a = m;
                    else b = m;
                }
                const unsigned e = p.queue[(unsigned long long)a * QS + (i - s_pref[a])];
                const unsigned Q = e & ~QB_INB;
                const unsigned L = p.lab[Q] >> 2;
                p.lab[Q] = (L << 2) | ((e & QB_INB) ? INB : 0u) | IDLE;
                const RT r = rec[Q];
                unsigned lp[2 * D];
#pragma unroll
                for (int dir = 0; dir < 2 * D; ++dir) {
                    unsigned a1, a2;
                    rec_get<D>(r, dir, a1, a2);
                    lp[dir] = a1 ? p.lab[(long long)Q + p.off[dir]] : 0xFFFFFFFFu;
                }
#pragma unroll
                for (int dir = 0; dir < 2 * D; ++dir) {
                    unsigned a1, a2;
                    rec_get<D>(r, dir, a1, a2);
                    if (a1) {
                        ++cD;
                        const int q = (int)L - (int)a2;
                        if (q > (int)(lp[dir] >> 2)) {
                            const unsigned bk = (unsigned)((t + a1) & Wm);
                            const unsigned pos = atomicAdd(&s_cnt[bk], 1u);
                            if (pos < S) {
                                // the receiver sees the sender in the opposite direction
                                p.pool[((unsigned long long)bk * G + g) * S + pos] =
                                    make_uint2((unsigned)((long long)Q + p.off[dir]),
                                               ((unsigned)q << 3) | (unsigned)(2 * D - 1 - dir));
                            } else {
                                atomicOr(&s_flags, SF_OVER);
                            }
                            ++cE;
                        }
                    }
                }
            }
        }
        __syncthreads();
        // next non-empty bucket of this workgroup, flows it holds in transit
        if (tid < 64) {
            unsigned best = 0xFFFFFFFFu, over = 0;
            unsigned long long tr = 0;
            for (unsigned j = tid; j + 1 < W; j += 64) {
                const unsigned c = s_cnt[(unsigned)((t + 1 + j) & Wm)];
                tr += c;
                if (c > S) over = 1;
                if (c && best == 0xFFFFFFFFu) best = j + 1;
            }
            for (int o = 32; o > 0; o >>= 1) {
                best = min(best, (unsigned)__shfl_xor(best, o));
                tr += __shfl_xor(tr, o);
                over |= __shfl_xor(over, o);
            }
            if (tid == 0) {
                const unsigned fl = (s_flags & SF_OVER) | (over ? SF_OVER : 0u);
                st_rlx(&ctl->nslot[g], (best == 0xFFFFFFFFu ? 0u : best) | fl);
                st_rlx(&ctl->tslot[g], (unsigned)min(tr, 0xFFFFFFFFull));
            }
        }
        PHASE(0);
        if (!grid_sync(ctl, epoch, p.wait_limit)) { status = ST_BROKEN; break; }
        PHASE(1);

        // ---- Step 1 (Algorithm 4): next delivery time = earliest bucket anywhere.
        {
            const unsigned raw = tid < G ? ld_rlx(&ctl->nslot[tid]) : 0u;
            if (tid == 0) { s_min = 0xFFFFFFFFu; s_flags = 0; }
            __syncthreads();
            const unsigned d0 = raw & SF_MASK;
            if (tid < G && d0) atomicMin(&s_min, d0);
            if (tid < G && (raw & SF_OVER)) atomicOr(&s_flags, SF_OVER);
            if (lead && tid < G) {
                const unsigned tr = ld_rlx(&ctl->tslot[tid]);
                atomicAdd(&s_red[3], (unsigned long long)tr);   // s_red[3] zeroed below
            }
            __syncthreads();
        }
        const unsigned dmin = s_min;
        const bool over = (s_flags & SF_OVER) != 0;
        if (lead && tid == 0) {
            cP = s_red[3] > cP ? s_red[3] : cP;
            s_red[3] = 0;
        }
        __syncthreads();
        if (over) { status = ST_OVERFLOW; break; }
        if (dmin == 0xFFFFFFFFu) { status = ST_DONE; break; }            // condition 2
        if (p.max_cycles > 0 && (long long)cyc >= p.max_cycles) { status = ST_CANCELED; break; }
        t += dmin;
        ++cyc;
        if (lead && tid == 0) ++cC;
        PHASE(2);

        // ---- Arrival (Steps 1-3 and 8, Algorithms 4-6, 10): own segment of bucket t.
        b_cur = (unsigned)(t & Wm);
        bucket_n = s_cnt[b_cur];
        if (tid == 0) s_qn = 0;
        __syncthreads();
        {
            const uint2 *seg = p.pool + ((unsigned long long)b_cur * G + g) * S;
            for (unsigned j = tid; j < bucket_n; j += BLOCK) {
                const uint2 f = seg[j];
                const unsigned P = f.x, q = f.y >> 3;
                bool imp = false;
                unsigned inb = 0;
                if (q > (p.lab[P] >> 2)) {
                    const unsigned old = atomicMax(&p.lab[P], q << 2);
                    imp = (q > (old >> 2)) && (old & IDLE);
                    inb = old & INB;
                }
                const unsigned long long m = __ballot(imp);
                if (m) {
                    const int ld = __ffsll((long long)m) - 1;
                    unsigned base = 0;
                    if ((int)lane == ld) base = atomicAdd(&s_qn, (unsigned)__popcll(m));
                    base = __shfl(base, ld);
                    if (imp) {
                        const unsigned slot = base + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
                        if (slot < QS) myq[slot] = P | (inb ? QB_INB : 0u);
                        else atomicOr(&s_flags, SF_OVER);
                        if (inb) atomicOr(&s_flags, SF_BHIT);
                        ++cU;
                    }
                }
            }
        }
        if (tid == 0) cR += bucket_n;
        __syncthreads();
        if (tid == 0) {
            s_cnt[b_cur] = 0;
            st_rlx(&ctl->qslot[g], min(s_qn, QS) | (s_flags & (SF_OVER | SF_BHIT)));
            s_flags = 0;
        }
        PHASE(3);
        if (!grid_sync(ctl, epoch, p.wait_limit)) { status = ST_BROKEN; break; }
        PHASE(4);
        unsigned fl;
        Qtot = gather_frontier(fl);
        PHASE(5);
        if (lead && tid == 0) cI = Qtot > cI ? Qtot : cI;
        if (fl & SF_OVER) { status = ST_OVERFLOW; break; }

        // ---- Step 6 (Algorithm 2): a vertex of B improved -> T = t.
        if (fl & SF_BHIT) {
            // X = best label among improved B vertices, smallest index on ties
            {
                const unsigned nq = min(s_qn, QS);
                unsigned long long best = 0;
                for (unsigned j = tid; j < nq; j += BLOCK) {
                    const unsigned e = myq[j];
                    if (e & QB_INB) {
                        const unsigned P = e & ~QB_INB;
                        const unsigned long long key =
                            ((unsigned long long)(p.lab[P] >> 2) << 32) | (0xFFFFFFFFull - P);
                        best = key > best ? key : best;
                    }
                }
                for (int o = 32; o > 0; o >>= 1) {
                    const unsigned long long ob = __shfl_xor(best, o);
                    best = ob > best ? ob : best;
                }
                if (tid == 0) s_red[0] = 0;
                __syncthreads();
                if (lane == 0 && best) atomicMax(&s_red[0], best);
                __syncthreads();
                if (tid == 0 && s_red[0]) atomicMax(&ctl->xkey, s_red[0]);
            }
            if (!grid_sync(ctl, epoch, p.wait_limit)) { status = ST_BROKEN; break; }
            const unsigned long long xk = __hip_atomic_load(&ctl->xkey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned X = (unsigned)(0xFFFFFFFFull - (xk & 0xFFFFFFFFull));
            const unsigned LX = (unsigned)(xk >> 32);
            // x = the delivery to X at T carrying LX, smallest sender
            {
                const uint2 *seg = p.pool + ((unsigned long long)b_cur * G + g) * S;
                for (unsigned j = tid; j < bucket_n; j += BLOCK) {
                    const uint2 f = seg[j];
                    if (f.x == X && (f.y >> 3) == LX) atomicMin(&ctl->ydir, f.y & 7u);
                }
            }
            if (!grid_sync(ctl, epoch, p.wait_limit)) { status = ST_BROKEN; break; }
            if (lead && tid == 0 && ld_rlx(&ctl->ydir) >= 2u * D) {
                __hip_atomic_store(&ctl->broken, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else if (lead && tid == 0) {
                const unsigned yd = ld_rlx(&ctl->ydir);
                const long long Y = (long long)X + p.off[yd];
                const bool lower = (int)yd < D;
                const int k = lower ? D - 1 - (int)yd : (int)yd - D;
                ctl->res[0] = t;
                ctl->res[1] = X;
                ctl->res[2] = (long long)k * N + (lower ? Y : (long long)X);
                ctl->res[3] = Y;
                ctl->res[4] = (long long)p.M - (long long)LX;
            }
            status = ST_DONE;
            break;
        }
    }

    // ---- outputs
    if (status == ST_DONE && p.labels_out) {
        const long long chunk = (N + G - 1) / G;
        const long long lo = (long long)g * chunk, hi = min(N, lo + chunk);
        for (long long v = lo + tid; v < hi; v += BLOCK) p.labels_out[v] = p.lab[v] >> 2;
    }
    __syncthreads();
    if (tid == 0) {
        s_red[0] = 0;
        s_red[1] = 0;
        s_red[2] = 0;
        s_red[3] = 0;
    }
    __syncthreads();
    if (cU) atomicAdd(&s_red[0], cU);
    if (cD) atomicAdd(&s_red[1], cD);
    if (cE) atomicAdd(&s_red[2], cE);
    if (cR) atomicAdd(&s_red[3], cR);
    __syncthreads();
    if (tid == 0) {
        if (s_red[0]) atomicAdd(&ctl->ctr[1], s_red[0]);
        if (s_red[1]) atomicAdd(&ctl->ctr[2], s_red[1]);
        if (s_red[2]) atomicAdd(&ctl->ctr[3], s_red[2]);
        if (s_red[3]) atomicAdd(&ctl->ctr[4], s_red[3]);
        if (lead) {
            for (int i = 0; i < 6; ++i) ctl->prof[i] = ph[i];
            ctl->ctr[0] = cC;
            ctl->ctr[5] = cP;
            ctl->ctr[6] = cI;
            const int br = __hip_atomic_load(&ctl->broken, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ctl->status = br ? ST_BROKEN : status;
            if (status == ST_DONE && ctl->xkey == 0) {
                for (int i = 0; i < 5; ++i) ctl->res[i] = -1;
            }
        }
    }
}

// ===========================================================================
// Range-owned cycle kernel
//
// Workgroup r owns the contiguous vertex range [r*c, r*c + c) (ranges are
// laid out so each XCD holds a contiguous run of them).  It keeps the
// range's labels, a frontier bitmap and a B bitmap in LDS, and it alone
// delivers water to the range, so deliveries are LDS atomics and every label
// it reads for a neighbour test inside the range is already final.
//
// A neighbour test across ranges is shipped instead: the sender writes a
// candidate (vertex, quality, f1, direction) to the neighbouring range, and
// that range's owner runs the test against its own labels before its next
// delivery can change them, filing the flow itself if it passes.  All flows
// into a range therefore sit in that range's own wheel (per-bucket fills in
// LDS), and a cycle needs one grid barrier:
//
//   send from I_t inside the range, ship candidates out (Steps 4-5)
//   arrive at the barrier; once the neighbouring ranges have arrived, accept
//     the candidates they shipped at t (Steps 4-5 across ranges)
//   barrier release, combining the next event time, flags, counts and the
//     best B key
//   deliver the next bucket, commit labels, build I_t (Steps 1-3, 8)
//
// The barrier's result decides termination (Steps 6 and 1) identically in
// every workgroup; the departure of the terminal cycle is discarded.
// ===========================================================================

constexpr int KMAX = 4;                 // neighbours lie within KMAX ranges
constexpr unsigned DENSE_NEVER = 0xFFFFFFFFu;   // dense threshold: keep the append list
constexpr int NOMAX = 2 * KMAX + 1;

// What a gang barrier combines.  mn is below 0xFFFF or 0xFFFFFFFF (none);
// only the top four bits of orf are combined.
struct Comb {
    unsigned mn;                        // minimum (0xFFFFFFFF = none)
    unsigned orf;                       // bitwise or (bits 28-31)
    unsigned long long s0, s1, s2;      // sums
    unsigned long long mx;              // maximum
    const unsigned long long *rest;     // where s0, s1, s2, mx of this barrier lie (null: in the fields)
};

__device__ __forceinline__ unsigned long long *bar_slot(BarHdr *b, unsigned i)
{
    return reinterpret_cast<unsigned long long *>(b + 1) + (size_t)i * 16;
}

__device__ __forceinline__ unsigned long long *bar_flag(BarHdr *b, unsigned g, unsigned i)
{
    return reinterpret_cast<unsigned long long *>(b + 1) + ((size_t)g + i) * 16;
}

__device__ __forceinline__ unsigned long long ld64(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st64(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void comb_wave(unsigned &mn, unsigned &orf, unsigned long long &s0,
                                          unsigned long long &s1, unsigned long long &s2,
                                          unsigned long long &mx)
{
    for (int o = 32; o > 0; o >>= 1) {
        mn = min(mn, (unsigned)__shfl_xor(mn, o));
        orf |= __shfl_xor(orf, o);
        s0 += __shfl_xor(s0, o);
        s1 += __shfl_xor(s1, o);
        s2 += __shfl_xor(s2, o);
        const unsigned long long om = __shfl_xor(mx, o);
        mx = om > mx ? om : mx;
    }
}

// Wait until every memory access the calling wave has issued is complete.
// The compiler may not move memory accesses across it.
__device__ __forceinline__ void vm_drain()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Tree barrier among the g workgroups of a gang (member m is the caller)
// that combines one Comb per member.  Members write their Comb to a private
// slot line, publish with an agent-scope release fence and count themselves
// in group m % 8; the group's last arriver combines the group's slots with
// one wavefront, writes the group slot and counts the group at the root; the
// last group combines the group slots and writes the result, then the new
// epoch, into every member's flag line.  Waiters spin on their own line; a
// wait that outlasts `limit` wall-clock ticks marks the gang broken and the
// call returns false, so a logic error drains the gang instead of hanging.
// The cycle loop uses gang_or instead; this one publishes the plain stores
// made before it (edge records, fills cleared at initialisation, results).
__device__ bool gang_combine(BarHdr *bh, unsigned g, unsigned m, unsigned &epoch, unsigned long long limit,
                             const Comb &mine, Comb &out, bool need_rest, unsigned long long *tpub = nullptr)
{
    __shared__ int s_ok;
    __shared__ unsigned long long s_o[5];
    __syncthreads();
    ++epoch;
    if (g == 1) {
        out = mine;
        out.rest = nullptr;
        return true;
    }
    if (threadIdx.x < 64) {
        const unsigned lane = threadIdx.x;
        const unsigned grp = m % NGRP;
        const unsigned ngrp = g < NGRP ? g : NGRP;
        const unsigned members = (g - grp + NGRP - 1) / NGRP;
        int leader = 0;
        if (lane == 0) {
            unsigned long long *sl = bar_slot(bh, m);
            st64(&sl[0], (unsigned long long)mine.mn | ((unsigned long long)mine.orf << 32));
            st64(&sl[1], mine.s0);
            st64(&sl[2], mine.s1);
            st64(&sl[3], mine.s2);
            st64(&sl[4], mine.mx);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const unsigned a = __hip_atomic_fetch_add(&bh->grp[grp][0], 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            leader = a == members - 1;
            if (leader) st_rlx(&bh->grp[grp][0], 0u);
        }
        leader = __shfl(leader, 0);
        if (leader) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            unsigned mn = 0xFFFFFFFFu, orf = 0;
            unsigned long long s0 = 0, s1 = 0, s2 = 0, mx = 0;
            for (unsigned j = lane; j < members; j += 64) {
                const unsigned long long *sl = bar_slot(bh, grp + NGRP * j);
                const unsigned long long w0 = ld64(&sl[0]);
                mn = min(mn, (unsigned)w0);
                orf |= (unsigned)(w0 >> 32);
                s0 += ld64(&sl[1]);
                s1 += ld64(&sl[2]);
                s2 += ld64(&sl[3]);
                const unsigned long long v = ld64(&sl[4]);
                mx = v > mx ? v : mx;
            }
            comb_wave(mn, orf, s0, s1, s2, mx);
            int releaser = 0;
            if (lane == 0) {
                unsigned long long *gs = bh->gslot[grp];
                st64(&gs[0], (unsigned long long)mn | ((unsigned long long)orf << 32));
                st64(&gs[1], s0);
                st64(&gs[2], s1);
                st64(&gs[3], s2);
                st64(&gs[4], mx);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                const unsigned rr = __hip_atomic_fetch_add(&bh->root[0], 1u, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
                releaser = rr == ngrp - 1;
                if (releaser) st_rlx(&bh->root[0], 0u);
            }
            releaser = __shfl(releaser, 0);
            if (releaser) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                mn = 0xFFFFFFFFu;
                orf = 0;
                s0 = s1 = s2 = mx = 0;
                if (lane < ngrp) {
                    const unsigned long long *gs = bh->gslot[lane];
                    const unsigned long long w0 = ld64(&gs[0]);
                    mn = (unsigned)w0;
                    orf = (unsigned)(w0 >> 32);
                    s0 = ld64(&gs[1]);
                    s1 = ld64(&gs[2]);
                    s2 = ld64(&gs[3]);
                    mx = ld64(&gs[4]);
                }
                comb_wave(mn, orf, s0, s1, s2, mx);
                // sums and maximum once per gang; the release word of every
                // member carries the epoch, the flags and the minimum
                unsigned long long *rs = bh->res[epoch & 1];
                if (lane == 0) {
                    st64(&rs[0], s0);
                    st64(&rs[1], s1);
                    st64(&rs[2], s2);
                    st64(&rs[3], mx);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                const unsigned long long w = ((unsigned long long)epoch << 32) |
                                             ((unsigned long long)(orf >> 28) << 16) | (mn < 0xFFFFu ? mn : 0xFFFFu);
                for (unsigned i = lane; i < g; i += 64) st64(&bar_flag(bh, g, i)[0], w);
            }
        }
        if (lane == 0) {
            int ok = 1;
            unsigned long long *fl = bar_flag(bh, g, m);
            const unsigned long long t0 = wall_clock64();
            if (tpub) *tpub = t0;           // published (and combined, if the last): the wait starts
            unsigned long long w;
            while (((w = ld64(&fl[0])) >> 32) < (unsigned long long)epoch) {
                __builtin_amdgcn_s_sleep(1);
                if (wall_clock64() - t0 > limit) {
                    __hip_atomic_store(&bh->broken, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (__hip_atomic_load(&bh->broken, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
            const unsigned mn16 = (unsigned)(w & 0xFFFFu), orf = (unsigned)((w >> 16) & 0xFu) << 28;
            s_o[0] = (unsigned long long)(mn16 == 0xFFFFu ? 0xFFFFFFFFu : mn16) | ((unsigned long long)orf << 32);
            if (need_rest || (orf & SF_BHIT)) {
                const unsigned long long *rs = bh->res[epoch & 1];
                for (int k = 0; k < 4; ++k) s_o[1 + k] = ld64(&rs[k]);
            }
            s_ok = ok;
        }
    }
    __syncthreads();
    out.mn = (unsigned)s_o[0];
    out.orf = (unsigned)(s_o[0] >> 32);
    out.s0 = s_o[1];
    out.s1 = s_o[2];
    out.s2 = s_o[3];
    out.mx = s_o[4];
    out.rest = bh->res[epoch & 1];
    const bool ok = s_ok != 0;
    __syncthreads();
    return ok;
}

// Barrier of the cycle loop.  Everything the members exchange around it
// (the words below, the caller's candidates and their fills) goes through
// agent-scope atomics, which are coherent across the XCDs' L2 caches by
// themselves, so it writes back and invalidates no cache; each wave only
// waits for its own accesses to complete before the workgroup arrives.
//
// Arrival is one fetch-or per level.  A member's word holds its arrival bit
// (bits 0-31), the four flag bits (32-35), a "far" bit (36) and the bit of
// its next event delta when that is 1..27 (bits 37-63); groups are up to 32
// consecutive members.  The fetch-or that completes a group's arrival bits
// forwards the or of the group's words (with the group's own arrival bit)
// to the root word, and the one that completes the root releases every
// member with (epoch, flags, least delta).  A member whose next delta is
// 28 or more sets "far" and first writes the delta, tagged with the epoch,
// to its slot line; only when no member has a near delta does the releaser
// read the slots.  So from the last member's arrival to everyone's wake-up
// there are two atomic round trips and one store-to-load delay.
//
// Sums (s0, s1, s2) and the B key (mx) bypass the barrier: the caller
// (gang_or_post) adds its sums to this barrier's line of a ring of four and
// raises the B key with an atomic maximum as soon as they are known, well
// before it arrives; member 0 reads the sums after the barrier (out.rest,
// final then) and clears the line, and everyone reads the B key after a
// barrier whose flags carry SF_BHIT.  Member 0 clears the ring lines, the B
// key and the arrival words at the start of each solve, before the solve's
// first (fully fenced) barrier.  A wait beyond `limit` ticks marks the gang
// broken, as in gang_combine.
constexpr unsigned OR_FAR = 36, OR_D0 = 37, OR_ND = 27;

__device__ __forceinline__ unsigned or_group_size(unsigned g) { return g <= 256 ? 16u : 32u; }

// What member m contributes to the next gang_or outside its arrival word:
// its sums, added to its group's lines of that barrier (so at most 32
// members add to one word), and its B key.
__device__ __forceinline__ void gang_or_post(BarHdr *bh, unsigned g, unsigned m, unsigned epoch,
                                             unsigned long long s0, unsigned long long s1, unsigned long long s2,
                                             unsigned long long mx)
{
    if (g == 1) return;
    unsigned long long(*ln)[16] = bh->ring[(epoch + 1) & 3][m / or_group_size(g)];
    if (s0) __hip_atomic_fetch_add(&ln[0][0], s0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (s1) __hip_atomic_fetch_add(&ln[1][0], s1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (s2) __hip_atomic_fetch_add(&ln[2][0], s2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (mx) __hip_atomic_fetch_max(&bh->bkey[0], mx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Member 0, after gang_or with epoch e: the sums of that barrier over all
// groups (wave 0), and the ring lines cleared for barrier e + 4.
__device__ __forceinline__ void gang_or_sums(BarHdr *bh, unsigned g, unsigned e, unsigned long long &s0,
                                             unsigned long long &s1, unsigned long long &s2)
{
    const unsigned lane = threadIdx.x & 63u, ngr = (g + or_group_size(g) - 1) / or_group_size(g);
    unsigned long long v[3] = {0, 0, 0};
    if (lane < ngr) {
        unsigned long long(*ln)[16] = bh->ring[e & 3][lane];
        for (int k = 0; k < 3; ++k) {
            v[k] = ld64(&ln[k][0]);
            st64(&ln[k][0], 0ull);
        }
    }
    for (int o = 32; o > 0; o >>= 1)
        for (int k = 0; k < 3; ++k) v[k] += __shfl_xor(v[k], o);
    s0 = v[0];
    s1 = v[1];
    s2 = v[2];
}

// First half of gang_or: member m arrives at barrier epoch + 1 (epoch is
// advanced) once every access of the workgroup has completed; waves 1 and
// up return at once, wave 0 arrives.  The member that completes the root
// releases everyone here.
__device__ void gang_or_arrive(BarHdr *bh, unsigned g, unsigned m, unsigned &epoch, const Comb &mine,
                               unsigned long long *tpub = nullptr)
{
    const unsigned e = epoch + 1;
    if (g > 1 && threadIdx.x == 0) {
        if (mine.mn != 0xFFFFFFFFu && mine.mn > OR_ND)
            st64(&bar_slot(bh, m)[8], ((unsigned long long)e << 32) | mine.mn);
    }
    vm_drain();
    __syncthreads();
    epoch = e;
    if (g == 1 || threadIdx.x >= 64) return;
    const unsigned lane = threadIdx.x;
    const unsigned MG = or_group_size(g);                      // members per group
    const unsigned ngr = (g + MG - 1) / MG;
    const unsigned grp = m / MG, gsz = min(MG, g - grp * MG);
    const unsigned long long tag = (unsigned long long)e << 32;
    if (tpub && lane == 0) *tpub = wall_clock64();
    unsigned long long comb = 0, rel = 2;  // rel: 2 not the releaser, 1 releaser reading far deltas, 0 releaser
    if (lane == 0) {
        unsigned long long w = (1ull << (m - grp * MG)) | ((unsigned long long)(mine.orf >> 28) << 32);
        if (mine.mn != 0xFFFFFFFFu) w |= mine.mn <= OR_ND ? 1ull << (OR_D0 + mine.mn - 1) : 1ull << OR_FAR;
        unsigned long long *gw = &bh->ow[e & 1][grp][0];
        const unsigned long long full_g = gsz == 64 ? ~0ull : (1ull << gsz) - 1;
        const unsigned long long og = __hip_atomic_fetch_or(gw, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) | w;
        if ((og & 0xFFFFFFFFull) == full_g) {
            // last of its group: forward the group to the root
            const unsigned long long rw = (og & ~0xFFFFFFFFull) | (1ull << grp);
            const unsigned long long full_r = (1ull << ngr) - 1;
            const unsigned long long orr =
                __hip_atomic_fetch_or(&bh->oroot[e & 1][0], rw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) | rw;
            if ((orr & 0xFFFFFFFFull) == full_r) {
                // last group: combine and release.  The arrival words of
                // this parity are cleared for the barrier after next.
                for (unsigned k = 0; k < ngr; ++k) st64(&bh->ow[e & 1][k][0], 0ull);
                st64(&bh->oroot[e & 1][0], 0ull);
                const unsigned long long near = (orr >> OR_D0) & ((1ull << OR_ND) - 1);
                unsigned mn = 0xFFFFFFFFu;
                if (near) mn = (unsigned)__builtin_ctzll(near) + 1;
                rel = ((orr >> OR_FAR) & 1ull) && !near ? 1 : 0;
                comb = ((unsigned long long)((orr >> 32) & 0xFull) << 32) | mn;
            }
        }
    }
    // the releaser reads the far deltas when there is no near one
    rel = __shfl(rel, 0);
    if (rel != 2) {
        comb = __shfl(comb, 0);
        unsigned mn = (unsigned)comb, orf4 = (unsigned)(comb >> 32);
        if (rel == 1) {
            unsigned fm = 0xFFFFFFFFu;
            for (unsigned i = lane; i < g; i += 64) {
                const unsigned long long v = ld64(&bar_slot(bh, i)[8]);
                if ((v & 0xFFFFFFFF00000000ull) == tag) fm = min(fm, (unsigned)v);
            }
            for (int o = 32; o > 0; o >>= 1) fm = min(fm, (unsigned)__shfl_xor(fm, o));
            mn = fm;
        }
        const unsigned long long rw = tag | ((unsigned long long)orf4 << 16) | (mn < 0xFFFFu ? mn : 0xFFFFu);
        for (unsigned i = lane; i < g; i += 64) st64(&bar_flag(bh, g, i)[0], rw);
    }
}

// Second half of gang_or: wait for the release of barrier epoch (the one
// gang_or_arrive entered) and return its flags, least delta and B key.
__device__ bool gang_or_wait(BarHdr *bh, unsigned g, unsigned m, unsigned epoch, unsigned long long limit,
                             const Comb &mine, Comb &out)
{
    __shared__ int s_ok;
    __shared__ unsigned long long s_o[2];
    if (g == 1) {
        out = mine;
        out.rest = nullptr;
        return true;
    }
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned long long t0 = wall_clock64();
        unsigned long long *fl = bar_flag(bh, g, m);
        unsigned long long w;
        while (((w = ld64(&fl[0])) >> 32) < (unsigned long long)epoch) {
            __builtin_amdgcn_s_sleep(1);
            if (wall_clock64() - t0 > limit) {
                __hip_atomic_store(&bh->broken, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
        }
        if (__hip_atomic_load(&bh->broken, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
        const unsigned mn16 = (unsigned)(w & 0xFFFFu), orf = (unsigned)((w >> 16) & 0xFu) << 28;
        s_o[0] = (unsigned long long)(mn16 == 0xFFFFu ? 0xFFFFFFFFu : mn16) | ((unsigned long long)orf << 32);
        s_o[1] = (orf & SF_BHIT) ? ld64(&bh->bkey[0]) : 0;
        s_ok = ok;
    }
    __syncthreads();
    out.mn = (unsigned)s_o[0];
    out.orf = (unsigned)(s_o[0] >> 32);
    out.s0 = out.s1 = out.s2 = 0;
    out.mx = s_o[1];
    out.rest = nullptr;
    const bool ok = s_ok != 0;
    __syncthreads();
    return ok;
}

__device__ bool gang_or(BarHdr *bh, unsigned g, unsigned m, unsigned &epoch, unsigned long long limit,
                        const Comb &mine, Comb &out, unsigned long long *tpub = nullptr)
{
    gang_or_arrive(bh, g, m, epoch, mine, tpub);
    return gang_or_wait(bh, g, m, epoch, limit, mine, out);
}

// Offset of the neighbour in direction dir (0..D-1: -stride[D-1..0],
// D..2D-1: +stride[0..D-1]).
template <int D> __device__ __forceinline__ long long dir_offset(long long n, int dir)
{
    const int k = dir < D ? D - 1 - dir : dir - D;
    long long st = 1;
    for (int j = 0; j < k; ++j) st *= n;
    return dir < D ? -st : st;
}

// One range-owned solve (a "job"): everything a gang of g workgroups needs.
struct RJ {
    long long n, N;
    long long c;                   // vertices per range
    int d;
    int K;                         // neighbours lie within K ranges
    int lt;                        // LDS label bytes (2 or 4)
    int llist;                     // frontier list entries kept in LDS (16-bit local indices); the rest in lists
    unsigned dense_thr;            // a range delivering more flows in a cycle builds I_t by a bitmap sweep
    int tile;                      // 1 (d = 3): ranges are x-pencils of n x ty x tz vertices
    int ty, tz;                    // pencil extent along y and z
    unsigned nty;                  // pencils along y
    unsigned g;                    // ranges (workgroups) in the gang
    const uint8_t *f1, *f2;        // SoA edge arrays [d][N]
    const uint8_t *A, *B;
    unsigned M;
    unsigned cand_cap;
    void *rec;                     // packed edge records, written by the owners
    unsigned *lists;               // [g][c] frontier list per range (when not in LDS)
    uint2 *pool;                   // [g][W][S] wheel of each range
    unsigned long long pool_flows;
    uint2 *cand;                   // [2][g][NO][cand_cap] candidates by sender and offset
    unsigned long long *pubc;      // [2][g][NOMAX] candidate fills, tagged with the barrier epoch
    BarHdr *bar;
    Out *out;
    unsigned *labels_out;
    long long max_cycles;
    unsigned long long wait_limit;
    int prof;
    long long *trace;              // [trace_cap][4] per delivery cycle: t, delivered, |I_t|, sent (nullable)
    long long trace_cap;
    // improvement log (reconstruction by walking back instead of re-solving)
    unsigned *wptr;                // [pool] record of the sender of each wheel flow
    unsigned *cptr;                // [2][g][NO][cand_cap] record of the sender of each candidate
    unsigned long long *winner;    // [g][c] (quality, -direction, sender record) of the best delivery
    unsigned *cur;                 // [g][c] latest improvement record of each vertex
    uint4 *log;                    // [g][log_cap] records (parent record, vertex, t, label)
    unsigned long long log_cap;    // records per range
};

template <typename LT> __device__ __forceinline__ unsigned lab_get(const LT *lab, unsigned i) { return lab[i]; }

// pencil-face flags kept in the spare word of a 3-d record
template <typename RT> __device__ __forceinline__ unsigned rec_cross(const RT &) { return 0; }
template <> __device__ __forceinline__ unsigned rec_cross<uint4>(const uint4 &v) { return v.w; }

// raise lab[i] to q; true when this call raised it
__device__ __forceinline__ bool lab_raise(unsigned *lab, unsigned i, unsigned q)
{
    if (q <= lab[i]) return false;
    return atomicMax(&lab[i], q) < q;
}

__device__ __forceinline__ bool lab_raise(uint16_t *lab, unsigned i, unsigned q)
{
    unsigned *w = reinterpret_cast<unsigned *>(lab) + (i >> 1);
    const unsigned sh = (i & 1u) * 16u;
    unsigned old = *w;
    for (;;) {
        const unsigned cur = (old >> sh) & 0xFFFFu;
        if (q <= cur) return false;
        const unsigned nw = (old & ~(0xFFFFu << sh)) | (q << sh);
        const unsigned prev = atomicCAS(w, old, nw);
        if (prev == old) return true;
        old = prev;
    }
}

// LDS labels of a range are 16 or 32 bits wide (uniform per workgroup).
__device__ __forceinline__ unsigned lget(const unsigned *lw, bool l16, unsigned i)
{
    return l16 ? (unsigned)reinterpret_cast<const uint16_t *>(lw)[i] : lw[i];
}

__device__ __forceinline__ void lset(unsigned *lw, bool l16, unsigned i, unsigned v)
{
    if (l16) reinterpret_cast<uint16_t *>(lw)[i] = (uint16_t)v;
    else lw[i] = v;
}

__device__ __forceinline__ bool lraise(unsigned *lw, bool l16, unsigned i, unsigned q)
{
    return l16 ? lab_raise(reinterpret_cast<uint16_t *>(lw), i, q) : lab_raise(lw, i, q);
}

constexpr unsigned CAND_LI = 0x1FFFFu;     // candidate word 0: local index | f1 << 17 | dir << 25

// Candidates cross workgroups inside the cycle loop, whose barrier writes
// back no cache: they are stored and loaded with agent-scope atomics.
__device__ __forceinline__ void cand_put(uint2 *p, unsigned w0, unsigned w1)
{
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), (unsigned long long)w0 | ((unsigned long long)w1 << 32),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint2 cand_get(const uint2 *p)
{
    const unsigned long long v =
        __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_uint2((unsigned)v, (unsigned)(v >> 32));
}
constexpr unsigned SF_BAD = 1u << 28;      // an edge with f1 or f2 equal to 0

// Range r of job p, run by the calling workgroup.  smem is the dynamic LDS
// block: labels | frontier bitmap | B bitmap | wheel fills [MAXW] | frontier
// list (the first p.llist entries, 16-bit local indices).
//
// Initialisation (Algorithm 3) packs the range's edge records (per vertex,
// (f1, f2) of its 2d edges in direction order, zero where the lattice ends),
// checks the edges, sets labels (M on A) and the A and B bitmaps.  A first
// barrier combines the largest f1 (it sizes the wheel) and input errors.
// Then each cycle:
//   departure (Steps 4-5) from I_t: inside the range, test and file flows;
//     across ranges, ship candidates to the owning range
//   barrier arrival; once the neighbouring ranges have arrived, accept the
//     candidates they shipped at t against this range's labels
//   barrier release: next event time, flags, counts, best B key (Steps 1, 6)
//   arrival (Steps 1-3, 8): deliver the next bucket, commit labels, build I_t
// What every member of the gang knows when a solve ends; yd (direction of
// the last edge seen from X) is known only to X's owner.
struct RunRes {
    int status;
    int found;
    long long t;
    unsigned X, LX, yd;
    unsigned mf;                   // largest f1 of the lattice
};

// M and B of the solve are arguments so that a chain of solves on one
// lattice (reconstruction) can change them: B is the mask p.B, or the single
// vertex bvert when bvert >= 0.  epoch continues over the gang's barriers.
// abits (nullable, [g][cw] words) keeps the A bitmap of each range: a full
// initialisation (reinit_mf == 0) writes it; a later solve of the same
// lattice passes the largest f1 seen before as reinit_mf and starts from
// abits, without re-reading or re-packing the edges.
template <int D, bool TILE = false, bool LOG = false>
__device__ RunRes range_run(const RJ &p, unsigned r, unsigned *smem, unsigned M, long long bvert, unsigned &epoch,
                            Out *out, unsigned *abits = nullptr, unsigned reinit_mf = 0)
{
    using RT = typename Rec<D>::T;
    __shared__ unsigned s_wave[NWAVES];
    __shared__ unsigned s_flags;
    __shared__ unsigned s_min;
    __shared__ unsigned s_ydir;
    __shared__ unsigned s_mf;
    __shared__ unsigned long long s_xkey;
    __shared__ unsigned long long s_sum;
    __shared__ unsigned long long s_red[4];
    __shared__ unsigned s_ccnt[NOMAX];        // candidates shipped / received this cycle
    __shared__ unsigned s_nl, s_bhn;          // size of I_t; improved vertices of B
    __shared__ unsigned s_nbad;               // a neighbour never arrived (gang broken)
    __shared__ unsigned s_sink;               // keeps the prefetch loads
    __shared__ unsigned s_cpre[NOMAX + 1];

    const unsigned tid = threadIdx.x, lane = lane_id();
    const unsigned G = p.g;
    const bool lead = r == 0;
    const long long n = p.n, N = p.N, c = p.c;
    // neighbour offsets split into whole ranges (floor) and a remainder in [0, c)
    long long offq[2 * D], offr[2 * D], offv[2 * D];
#pragma unroll
    for (int dir = 0; dir < 2 * D; ++dir) {
        const long long o = dir_offset<D>(n, dir);
        const long long q = o >= 0 ? o / c : -((-o + c - 1) / c);
        offv[dir] = o;
        offq[dir] = q;
        offr[dir] = o - q * c;
    }
    const long long base = (long long)r * c;
    // Pencil ranges (d = 3): range r holds x = 0..n-1, y in [ry ty, ry ty + ty),
    // z in [rz tz, rz tz + tz), local index x + n (ly + ty lz); a range at the
    // far faces can be partial.  Contiguous ranges hold vertices base..base+c-1.
    constexpr bool tile = D == 3 && TILE;
    const long long ty = p.ty, tz = p.tz;
    const long long ry = tile ? (long long)(r % p.nty) : 0, rz = tile ? (long long)(r / p.nty) : 0;
    const unsigned cr = tile ? (unsigned)c : (unsigned)max(0ll, min(c, N - base));
    const int K = p.K, NO = tile ? 2 * D : 2 * K + 1;
    // global index of local vertex i (-1 outside the lattice)
    auto gvert = [=](unsigned i) -> long long {
        if (!tile) return base + i;
        const long long x = i % n, q = i / n, y = ry * ty + q % ty, z = rz * tz + q / ty;
        return (y < n && z < n) ? x + n * (y + n * z) : -1;
    };
    // range and local index of global vertex v
    auto locate = [=](long long v, long long &li) -> long long {
        if (!tile) {
            li = v % c;
            return v / c;
        }
        const long long x = v % n, y = (v / n) % n, z = v / (n * n);
        const long long qy = y / ty, qz = z / tz;
        li = x + n * ((y - qy * ty) + ty * (z - qz * tz));
        return qy + (long long)p.nty * qz;
    };
    // target range offset of candidate slot s (a receiver reads slot s from range r - soff(s))
    auto soff = [=](int sl) -> long long {
        if (!tile) return (long long)(sl - K);
        return sl == 0 ? -(long long)p.nty : sl == 1 ? -1 : sl == 2 * D - 2 ? 1 : sl == 2 * D - 1 ? (long long)p.nty : 0;
    };
    RT *rec = static_cast<RT *>(p.rec);

    const unsigned cw = (unsigned)((c + 31) / 32);
    const bool l16 = p.lt == 2;
    const unsigned lab_words = (unsigned)((c * (long long)(l16 ? 2 : 4) + 3) / 4);
    unsigned *lab = smem;
    unsigned *fb = smem + lab_words;
    unsigned *bb = fb + cw;
    unsigned *cnt = bb + cw;
    unsigned *mylist = p.lists + (unsigned long long)r * c;
    uint16_t *lds_list = reinterpret_cast<uint16_t *>(smem + lab_words + 2 * cw + MAXW);
    const unsigned lcap = (unsigned)p.llist;
    auto list_put = [=](unsigned k, unsigned i) {
        if (k < lcap) lds_list[k] = (uint16_t)i;
        else mylist[k] = i;
    };
    auto list_get = [=](unsigned k) -> unsigned { return k < lcap ? (unsigned)lds_list[k] : mylist[k]; };
    uint2 *const cand = p.cand;
    unsigned long long *const pubc_base = p.pubc;
    const unsigned long long ccap = p.cand_cap;
    auto candbuf = [=](unsigned par, unsigned long long src, unsigned oi) {
        return cand + (((unsigned long long)par * G + src) * NO + oi) * ccap;
    };
    auto pubc = [=](unsigned par, unsigned long long src, unsigned oi) {
        return pubc_base + ((unsigned long long)par * G + src) * NOMAX + oi;
    };

    unsigned long long cU = 0, cD = 0, cE = 0, cR = 0;      // per thread, committed
    // counters C, P, I and the cycle trace state, kept by the lead's thread 0
    // (in LDS, so they cost no registers): C P I | rows, in transit before the
    // open row's sending round, its deliveries, open flag
    __shared__ unsigned long long s_lc[7];
    if (tid < 7) s_lc[tid] = 0;
    unsigned long long ph[6] = {0, 0, 0, 0, 0, 0}, ph_t = 0;
    // phase timing 1: range 0 only; 2: every range (sums and maxima)
    const bool timing = tid == 0 && (p.prof == 2 || (p.prof && lead));
#define PHASE4(k)                                            \
    do {                                                     \
        if (timing) {                                        \
            const unsigned long long now_ = wall_clock64();  \
            ph[k] += now_ - ph_t;                            \
            ph_t = now_;                                     \
        }                                                    \
    } while (0)

    for (unsigned i = tid; i < lab_words + 2 * cw + MAXW; i += BLOCK) smem[i] = 0;
    if (tid < 2 * NOMAX) p.pubc[((unsigned long long)(tid / NOMAX) * G + r) * NOMAX + tid % NOMAX] = 0;
    if (tid == 0) {
        s_flags = 0;
        s_xkey = 0;
        s_ydir = 0xFFFFFFFFu;
        s_mf = 0;
    }
    __syncthreads();

    // ---- Initialization (Algorithm 3): pack and check the range's edges;
    // Label = M on A, 0 elsewhere; A is I_0.
    if (reinit_mf) {
        for (unsigned w = tid; w < cw; w += BLOCK) {
            unsigned bits = abits[(unsigned long long)r * cw + w];
            fb[w] = bits;
            while (bits) {
                const unsigned bt = (unsigned)(__ffs(bits) - 1);
                bits &= bits - 1u;
                lset(lab, l16, w * 32u + bt, M);
            }
        }
        if (tid == 0) {
            s_mf = reinit_mf;
            long long bl = 0;
            if (bvert >= 0 && locate(bvert, bl) == (long long)r) {
                const unsigned i = (unsigned)bl;
                bb[i >> 5] |= 1u << (i & 31);
            }
        }
    } else {
        unsigned mf = 0, bad = 0;
        long long stride[D];
        {
            long long sv = 1;
            for (int k = 0; k < D; ++k) {
                stride[k] = sv;
                sv *= n;
            }
        }
        for (unsigned i = tid; i < cr; i += BLOCK) {
            const long long v = gvert(i);
            if (v < 0) {
                rec[base + i] = RT{};       // outside the lattice: no edges
                continue;
            }
            long long cc[D];
            long long rem = v;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                cc[k] = rem % n;
                rem /= n;
            }
            unsigned pr[2 * D];
#pragma unroll
            for (int dir = 0; dir < 2 * D; ++dir) {
                const bool lower = dir < D;
                const int k = lower ? D - 1 - dir : dir - D;
                const bool exists = lower ? (cc[k] >= 1) : (cc[k] <= n - 2);
                pr[dir] = 0;
                if (exists) {
                    const long long e = (long long)k * N + (lower ? v - stride[k] : v);
                    const unsigned a = p.f1[e], b = p.f2[e];
                    if (a == 0 || b == 0) bad = 1;
                    mf = a > mf ? a : mf;
                    pr[dir] = a | (b << 8);
                }
            }
            RT rv;
            if constexpr (D == 1) {
                rv = pr[0] | (pr[1] << 16);
            } else if constexpr (D == 2) {
                rv = make_uint2(pr[0] | (pr[1] << 16), pr[2] | (pr[3] << 16));
            } else if constexpr (D == 3) {
                // word 3: directions whose neighbour lies in another pencil
                unsigned cross = 0;
                if (tile) {
                    const long long q = (long long)i / n, ly = q % ty, lz = q / ty;
                    cross = (lz == 0 ? 1u : 0u) | (ly == 0 ? 2u : 0u) | (ly == ty - 1 ? 16u : 0u) |
                            (lz == tz - 1 ? 32u : 0u);
                }
                rv = make_uint4(pr[0] | (pr[1] << 16), pr[2] | (pr[3] << 16), pr[4] | (pr[5] << 16), cross);
            } else {
                rv = make_uint4(pr[0] | (pr[1] << 16), pr[2] | (pr[3] << 16), pr[4] | (pr[5] << 16),
                                pr[6] | (pr[7] << 16));
            }
            rec[base + i] = rv;
            const bool a = p.A[v] != 0, b = bvert >= 0 ? v == bvert : p.B[v] != 0;
            if (a && b) bad |= 2;
            if (a) {
                lset(lab, l16, i, M);
                atomicOr(&fb[i >> 5], 1u << (i & 31));
            }
            if (b) atomicOr(&bb[i >> 5], 1u << (i & 31));
        }
        for (int o = 32; o > 0; o >>= 1) {
            mf = max(mf, (unsigned)__shfl_xor(mf, o));
            bad |= __shfl_xor(bad, o);
        }
        if (lane == 0) {
            if (mf) atomicMax(&s_mf, mf);
            if (bad & 1) atomicOr(&s_flags, SF_BAD);
            if (bad & 2) atomicOr(&s_flags, SF_INVAL);
        }
    }
    __syncthreads();
    if (abits && !reinit_mf) {
        for (unsigned w = tid; w < cw; w += BLOCK) abits[(unsigned long long)r * cw + w] = fb[w];
    }

    // Frontier bitmap -> sorted list of local indices; clear the bitmap;
    // best (label, -index) over the B members in it.
    auto compact = [=]() -> unsigned {
        unsigned total = 0;
        unsigned long long bestB = 0;
        for (unsigned w0 = 0; w0 < cw; w0 += BLOCK) {
            const unsigned wi = w0 + tid;
            unsigned bits = 0, bm = 0;
            if (wi < cw) {
                bits = fb[wi];
                bm = bits & bb[wi];
                fb[wi] = 0;
            }
            unsigned tot;
            const unsigned ex = block_scan((unsigned)__popc(bits), s_wave, &tot);
            unsigned k = total + ex;
            while (bits) {
                const unsigned bt = (unsigned)(__ffs(bits) - 1);
                bits &= bits - 1u;
                const unsigned i = wi * 32u + bt;
                list_put(k++, i);
                if ((bm >> bt) & 1u) {
                    const unsigned long long key = ((unsigned long long)lget(lab, l16, i) << 32) |
                                                   (0xFFFFFFFFull - (unsigned long long)gvert(i));
                    bestB = key > bestB ? key : bestB;
                }
            }
            total += tot;
        }
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long ob = __shfl_xor(bestB, o);
            bestB = ob > bestB ? ob : bestB;
        }
        if (lane == 0 && bestB) {
            atomicMax(&s_xkey, bestB);
            atomicOr(&s_flags, SF_BHIT);
        }
        __syncthreads();
        return total;
    };

    // Dense form of I_t (Step 8's condensed list in vertex order): the
    // deliveries only set the frontier bitmap, and this sweep packs it, two
    // words per thread, into the list; each wave writes the set bits of its
    // words in ascending local index at an offset taken from a shared
    // counter (s_sw, zero on entry).  It also finds the best (label, -index)
    // over the improved vertices of B.  The bitmap is left as it is (the
    // departure clears it).
    __shared__ unsigned s_sw;
    auto sweep = [=]() -> unsigned {
        unsigned long long bestB = 0;
        for (unsigned w0 = 0; w0 < cw; w0 += 2 * BLOCK) {
            const unsigned wi = w0 + 2 * tid;
            const unsigned b0 = wi < cw ? fb[wi] : 0u, b1 = wi + 1 < cw ? fb[wi + 1] : 0u;
            const unsigned nb = (unsigned)(__popc(b0) + __popc(b1));
            unsigned x = nb;                        // inclusive scan over the wave
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const unsigned y = __shfl_up(x, o);
                if (lane >= (unsigned)o) x += y;
            }
            const unsigned wtot = __shfl(x, 63);
            unsigned wbase = 0;
            if (lane == 0 && wtot) wbase = atomicAdd(&s_sw, wtot);
            unsigned k = __shfl(wbase, 0) + x - nb;
            unsigned bits = b0;
            while (bits) {
                const unsigned bt = (unsigned)(__ffs(bits) - 1);
                bits &= bits - 1u;
                list_put(k++, wi * 32u + bt);
            }
            bits = b1;
            while (bits) {
                const unsigned bt = (unsigned)(__ffs(bits) - 1);
                bits &= bits - 1u;
                list_put(k++, (wi + 1) * 32u + bt);
            }
            // improved vertices of B: best (label, -index)
            for (int h = 0; h < 2; ++h) {
                const unsigned wh = wi + (unsigned)h, bh = h ? b1 : b0;
                unsigned bm = bh ? bh & bb[wh] : 0u;
                while (bm) {
                    const unsigned bt = (unsigned)(__ffs(bm) - 1);
                    bm &= bm - 1u;
                    const unsigned i = wh * 32u + bt;
                    const unsigned long long key = ((unsigned long long)lget(lab, l16, i) << 32) |
                                                   (0xFFFFFFFFull - (unsigned long long)gvert(i));
                    bestB = key > bestB ? key : bestB;
                }
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long ob = __shfl_xor(bestB, o);
            bestB = ob > bestB ? ob : bestB;
        }
        if (lane == 0 && bestB) {
            atomicMax(&s_xkey, bestB);
            atomicOr(&s_flags, SF_BHIT);
        }
        __syncthreads();
        return s_sw;
    };

    unsigned nlist = compact();
    if (tid == 0) cU += nlist;
    // improvement log: this range's records are log[r * log_cap ...]
    __shared__ unsigned long long s_logn;
    const unsigned long long logbase = LOG ? (unsigned long long)r * p.log_cap : 0;
    auto log_improved = [&](long long tt, unsigned nl, bool first) {
        // one record per vertex of I_t, parent = sender record of its best delivery
        const unsigned long long used = s_logn;
        if (used + nl > p.log_cap) {
            if (tid == 0) {
                atomicOr(&s_flags, SF_OVER);
                atomicOr(&out->log_over, 1);
            }
            return;
        }
        for (unsigned j = tid; j < nl; j += BLOCK) {
            const unsigned i = list_get(j);
            // the best delivery was combined by atomics in L2: read it there
            const unsigned parent =
                first ? 0xFFFFFFFFu
                      : (unsigned)(__hip_atomic_load(&p.winner[base + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                                   0xFFFFFFFFull);
            const unsigned idx = (unsigned)(logbase + used + j);
            p.log[idx] = make_uint4(parent, (unsigned)gvert(i), (unsigned)tt, lget(lab, l16, i));
            p.cur[base + i] = idx;
        }
        __syncthreads();
        if (tid == 0) s_logn = used + nl;
        __syncthreads();
    };
    if constexpr (LOG) {
        for (unsigned i = tid; i < (unsigned)c; i += BLOCK) p.winner[base + i] = 0;
        if (tid == 0) s_logn = 0;
        __syncthreads();
        log_improved(0, nlist, true);
    }

    if (lead) {
        // gang_or's arrival words, sums ring and B key start from zero in
        // every solve (published by the fully fenced barrier below)
        BarHdr *bh = p.bar;
        for (unsigned i = tid; i < 2 * 16 + 2 + 4 * 16 * 3 + 1; i += BLOCK) {
            unsigned long long *w = i < 32 ? &bh->ow[i / 16][i % 16][0]
                                    : i < 34 ? &bh->oroot[i - 32][0]
                                    : i < 34 + 192 ? &bh->ring[(i - 34) / 48][(i - 34) / 3 % 16][(i - 34) % 3][0]
                                                   : &bh->bkey[0];
            st64(w, 0ull);
        }
    }
    int status = ST_RUNNING;
    unsigned W = 2;
    RunRes rr;
    {
        Comb mine, all;
        mine.mn = 0xFFFFFFFFu;
        mine.orf = s_flags & (SF_BAD | SF_INVAL);
        mine.s0 = mine.s1 = mine.s2 = 0;
        mine.mx = s_mf;
        if (!gang_combine(p.bar, G, r, epoch, p.wait_limit, mine, all, true)) status = ST_BROKEN;
        else if (all.orf & (SF_BAD | SF_INVAL)) status = ST_INVAL;
        while (W <= (unsigned)all.mx) W <<= 1;
        rr.mf = (unsigned)all.mx;
        if (tid == 0) s_flags = 0;                   // an A member of B is an error, not a hit
        __syncthreads();
    }
    const unsigned Wm = W - 1;
    const unsigned long long S = p.pool_flows / ((unsigned long long)G * W);
    const unsigned CS = p.cand_cap;
    uint2 *wheel = p.pool + (unsigned long long)r * W * S;
    unsigned *wptr = LOG ? p.wptr + (unsigned long long)r * W * S : nullptr;

    rr.X = rr.LX = 0;
    long long t = 0;
    unsigned cyc = 0, par = 0;
    unsigned F = 0;                     // flows delivered this cycle
    unsigned long long transit = 0;     // flows in transit after the previous sending round
    bool found = false;
    if (timing) ph_t = wall_clock64();

    while (status == ST_RUNNING) {
        // ---- Departure (Steps 4-5, Algorithms 7-8) from I_t in this range.
        unsigned long long dD = 0, dE = 0;
        if (tid < NOMAX) s_ccnt[tid] = 0;
        if (tid == 0) s_min = 0xFFFFFFFFu;
        __syncthreads();
        unsigned amin = 0xFFFFFFFFu;      // least f1 of a shipped candidate
        // the record of the next frontier vertex is in flight while one is
        // processed
        auto front = [&](unsigned j, unsigned &i, RT &rv) {
            if (j < nlist) {
                i = list_get(j);
                rv = rec[base + i];
            }
        };
        unsigned i1 = 0, i2 = 0;
        RT r1{}, r2{};
        front(tid, i1, r1);
        front(tid + BLOCK, i2, r2);
        for (unsigned j = tid; j < nlist; j += BLOCK) {
            const unsigned i = i1;
            const RT rv = r1;
            i1 = i2;
            r1 = r2;
            front(j + 2 * BLOCK, i2, r2);
            fb[i >> 5] = 0;                 // every vertex of the word is in this list
            const unsigned L = lget(lab, l16, i);
            const unsigned myrec = LOG ? p.cur[base + i] : 0u;
#pragma unroll
            for (int dir = 0; dir < 2 * D; ++dir) {
                unsigned a1, a2;
                rec_get<D>(rv, dir, a1, a2);
                if (!a1) continue;
                ++dD;
                const int q = (int)L - (int)a2;
                if (q <= 0) continue;
                bool wrap;
                int o;
                unsigned li;                                            // index in the owner's range
                if (tile) {
                    // within the pencil, or across its y / z face
                    long long lstep = 1, span = 1;
                    if (dir == 0 || dir == 2 * D - 1) { lstep = n * ty; span = tz; }
                    if (dir == 1 || dir == 2 * D - 2) { lstep = n; span = ty; }
                    const bool up = dir >= D;
                    wrap = false;
                    if (rec_cross(rv) & (1u << dir)) {
                        o = 1;                                          // any nonzero: candidate slot dir
                        li = (unsigned)((long long)i + (up ? -(span - 1) : (span - 1)) * lstep);
                    } else {
                        o = 0;
                        li = (unsigned)((long long)i + (up ? lstep : -lstep));
                    }
                } else {
                    const long long lo = (long long)i + offr[dir];
                    wrap = lo >= c;
                    o = (int)offq[dir] + (wrap ? 1 : 0);
                    li = (unsigned)(wrap ? lo - c : lo);
                }
                const unsigned rdir = (unsigned)(2 * D - 1 - dir);      // sender seen from the receiver
                if (o == 0) {
                    if ((unsigned)q > lget(lab, l16, li)) {
                        const unsigned bk = (unsigned)((t + a1) & Wm);
                        const unsigned pos = atomicAdd(&cnt[bk], 1u);
                        if (pos < S) {
                            wheel[(unsigned long long)bk * S + pos] =
                                make_uint2((unsigned)(base + li), ((unsigned)q << 3) | rdir);
                            if constexpr (LOG) wptr[(unsigned long long)bk * S + pos] = myrec;
                        } else {
                            atomicOr(&s_flags, SF_OVER);
                        }
                        ++dE;
                    }
                } else {
                    const unsigned oi = tile ? (unsigned)dir : (unsigned)(o + K);
                    // for one direction a wave ships to at most two receivers:
                    // the lanes of each share one LDS atomic
                    const unsigned long long mw = __ballot(wrap), ma = __ballot(1);
                    const unsigned long long grp = wrap ? mw : (ma & ~mw);
                    const int leader = __ffsll((long long)grp) - 1;
                    unsigned first = 0;
                    if ((int)lane == leader) first = atomicAdd(&s_ccnt[oi], (unsigned)__popcll(grp));
                    first = __shfl(first, leader);
                    const unsigned pos = first + (unsigned)__popcll(grp & ((1ull << lane) - 1ull));
                    if (pos < CS) {
                        cand_put(candbuf(par, r, oi) + pos, li | (a1 << 17) | (rdir << 25), (unsigned)q);
                        if constexpr (LOG)
                            __hip_atomic_store(&p.cptr[(candbuf(par, r, oi) - cand) + pos], myrec, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                    } else {
                        atomicOr(&s_flags, SF_OVER);
                    }
                    amin = a1 < amin ? a1 : amin;
                }
            }
        }
        for (int o = 32; o > 0; o >>= 1) amin = min(amin, (unsigned)__shfl_xor(amin, o));
        if (lane == 0 && amin != 0xFFFFFFFFu) atomicMin(&s_min, amin);
        __syncthreads();
        // candidate fills (published after the barrier arrival); next
        // delivery time seen from this range
        if (tid < (unsigned)NO && soff((int)tid) != 0 && s_ccnt[tid] > CS) atomicOr(&s_flags, SF_OVER);
        {
            unsigned best = 0xFFFFFFFFu, over = 0;
            for (unsigned bk = tid; bk < W; bk += BLOCK) {
                const unsigned v = cnt[bk];
                if (v) {
                    const unsigned delta = (unsigned)((bk - (unsigned)t) & Wm);
                    best = min(best, delta);
                    if (v > S) over = 1;
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                best = min(best, (unsigned)__shfl_xor(best, o));
                over |= __shfl_xor(over, o);
            }
            if (lane == 0) {
                if (best != 0xFFFFFFFFu) atomicMin(&s_min, best);
                if (over) atomicOr(&s_flags, SF_OVER);
            }
        }
        __syncthreads();
        PHASE4(0);
        Comb mine, all;
        mine.mn = s_min;
        mine.orf = s_flags & (SF_OVER | SF_BHIT);
        mine.s0 = F;
        mine.s1 = nlist;
        mine.s2 = transit;
        mine.mx = s_xkey;
        if (tid == 0) s_nbad = 0;
        gang_or_arrive(p.bar, G, r, epoch, mine);
        PHASE4(1);
        // ---- Steps 4-5 across ranges: test the candidates the neighbours
        // shipped at t against this range's labels (still L_t) and file the
        // flows, while the barrier completes.  Every access of the departure
        // has completed (gang_or_arrive waited for them), so each fill count
        // is published now, tagged with the barrier's epoch; a neighbour's
        // candidates are complete once its count with this epoch is seen.  A
        // run that ends at this barrier (T found, overflow) discards what is
        // filed here; it is counted (cEx) only when the run goes on.
        unsigned long long cEx = 0;
        if (tid >= 64 && tid - 64 < (unsigned)NO) {      // wave 1: wave 0 is arriving
            const unsigned sl = tid - 64;
            const long long so = soff((int)sl);           // slot sl comes from range r - so
            if (so != 0)
                st64(pubc(par, r, sl), ((unsigned long long)epoch << 32) | min(s_ccnt[sl], CS));
            const long long src = (long long)r - so;
            unsigned v = 0;
            if (so != 0 && src >= 0 && src < (long long)G) {
                const unsigned long long *w = pubc(par, (unsigned long long)src, sl);
                unsigned long long x = ld64(w);
                if ((x >> 32) < (unsigned long long)epoch) {
                    const unsigned long long t0 = wall_clock64();
                    for (;;) {
                        __builtin_amdgcn_s_sleep(1);
                        x = ld64(w);
                        if ((x >> 32) >= (unsigned long long)epoch) break;
                        if (wall_clock64() - t0 > p.wait_limit ||
                            __hip_atomic_load(&p.bar->broken, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                            __hip_atomic_store(&p.bar->broken, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            s_nbad = 1;
                            x = 0;
                            break;
                        }
                    }
                }
                v = (unsigned)x;
            }
            s_ccnt[sl] = v;
        }
        __syncthreads();
        if (tid == 0) {
            s_cpre[0] = 0;
            for (int oi = 0; oi < NO; ++oi) s_cpre[oi + 1] = s_cpre[oi] + s_ccnt[oi];
        }
        __syncthreads();
        {
            const unsigned FC = s_cpre[NO];
            constexpr int UC = 4;                   // candidate loads in flight per thread
            for (unsigned j0 = tid; j0 < FC; j0 += BLOCK * UC) {
              uint2 cdu[UC];
              unsigned cpu[UC];
#pragma unroll
              for (int u = 0; u < UC; ++u) {
                const unsigned j = j0 + u * BLOCK;
                if (j < FC) {
                    int oi = 0;
                    while (j >= s_cpre[oi + 1]) ++oi;
                    const long long src = (long long)r - soff(oi);
                    const uint2 *cb = candbuf(par, (unsigned long long)src, (unsigned)oi);
                    cdu[u] = cand_get(cb + (j - s_cpre[oi]));
                    if constexpr (LOG)
                        cpu[u] = __hip_atomic_load(&p.cptr[(cb - cand) + (j - s_cpre[oi])], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                }
              }
#pragma unroll
              for (int u = 0; u < UC; ++u) {
                if (j0 + u * BLOCK >= FC) continue;
                const uint2 cd = cdu[u];
                const unsigned li = cd.x & CAND_LI, a1 = (cd.x >> 17) & 0xFFu, rdir = cd.x >> 25;
                if (cd.y > lget(lab, l16, li)) {
                    const unsigned bk = (unsigned)((t + a1) & Wm);
                    const unsigned pos = atomicAdd(&cnt[bk], 1u);
                    if (pos < S) {
                        wheel[(unsigned long long)bk * S + pos] = make_uint2((unsigned)(base + li), (cd.y << 3) | rdir);
                        if constexpr (LOG) wptr[(unsigned long long)bk * S + pos] = cpu[u];
                    } else {
                        atomicOr(&s_flags, SF_OVER);
                    }
                    ++cEx;
                }
              }
            }
        }
        par ^= 1u;
        PHASE4(2);
        // While the release is on its way, bring the bucket of t + 1 (the
        // usual next delivery time) into the L2: one word per 128-byte line,
        // loaded by waves 1-15 (wave 0 waits for the release), consumed
        // after it.
        unsigned xb = 0;
        {
            const unsigned bk1 = (unsigned)((t + 1) & Wm);
            const unsigned c1 = __hip_atomic_load(&cnt[bk1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const unsigned n1 = (unsigned)min((unsigned long long)c1, S);
            if (tid >= 64 && (tid - 64) * 16u < n1) xb = wheel[(unsigned long long)bk1 * S + (tid - 64) * 16u].x;
        }
        if (!gang_or_wait(p.bar, G, r, epoch, p.wait_limit, mine, all) || s_nbad) {
            status = ST_BROKEN;
            break;
        }
        if (xb == 0x9E3779B9u) *(volatile unsigned *)&s_sink = xb;
        PHASE4(4);

        // the counters' sums are needed by the lead only; it clears the
        // ring line they came in for a later barrier
        unsigned long long a0 = all.s0, a1 = all.s1, a2 = all.s2;
        if (lead && tid < 64 && G > 1) gang_or_sums(p.bar, G, epoch, a0, a1, a2);
        if (all.orf & SF_OVER) { status = ST_OVERFLOW; break; }
        if (cyc > 0 && lead && tid == 0) {
            s_lc[0] += a0 > 0 ? 1 : 0;
            s_lc[2] = a1 > s_lc[2] ? a1 : s_lc[2];
            s_lc[1] = a2 > s_lc[1] ? a2 : s_lc[1];
            if (p.trace) {
                // a0, a1: delivered and |I_t| at t; a2: in transit after the
                // sending round of the previous cycle, which completes that
                // cycle's row: sent = a2 - (in transit before it) + delivered
                const long long rows = (long long)s_lc[3];
                if (s_lc[6]) {
                    if (rows <= p.trace_cap) p.trace[4 * (rows - 1) + 3] = (long long)(a2 - s_lc[4] + s_lc[5]);
                    s_lc[6] = 0;
                }
                if (a0 > 0) {
                    if (rows + 1 <= p.trace_cap) {
                        long long *row = p.trace + 4 * rows;
                        row[0] = t;
                        row[1] = (long long)a0;
                        row[2] = (long long)a1;
                        row[3] = 0;             // the last row keeps 0: nothing is sent at the end
                    }
                    s_lc[3] = (unsigned long long)(rows + 1);
                    s_lc[5] = a0;
                    s_lc[6] = 1;
                }
                s_lc[4] = a2;
            }
        }
        if (all.orf & SF_BHIT) {
            // ---- Step 6 (Algorithm 2): T = t.  The departure just made is
            // not part of the run; x is the delivery to X carrying its label
            // from the smallest sender, found by X's owner.
            found = true;
            const unsigned X = (unsigned)(0xFFFFFFFFull - (all.mx & 0xFFFFFFFFull));
            const unsigned LX = (unsigned)(all.mx >> 32);
            long long xl = 0;
            if (locate((long long)X, xl) == (long long)r) {
                const unsigned Xr = (unsigned)(base + xl);              // X as a wheel entry names it
                const uint2 *bkt = wheel + (unsigned long long)(t & Wm) * S;
                for (unsigned j = tid; j < F; j += BLOCK) {
                    const uint2 f = bkt[j];
                    if (f.x == Xr && (f.y >> 3) == LX) atomicMin(&s_ydir, f.y & 7u);
                }
                __syncthreads();
                if (tid == 0) {
                    const unsigned yd = s_ydir;
                    if (yd >= 2u * D) {
                        __hip_atomic_store(&p.bar->broken, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    } else {
                        long long oy = 0;
#pragma unroll
                        for (int dd = 0; dd < 2 * D; ++dd)
                            if ((unsigned)dd == yd) oy = offv[dd];
                        const long long Y = (long long)X + oy;
                        const bool lower = (int)yd < D;
                        const int k = lower ? D - 1 - (int)yd : (int)yd - D;
                        out->res[0] = t;
                        out->res[1] = X;
                        out->res[2] = (long long)k * N + (lower ? Y : (long long)X);
                        out->res[3] = Y;
                        out->res[4] = (long long)M - (long long)LX;
                        if constexpr (LOG) out->xrec = p.cur[base + xl];
                    }
                }
            }
            rr.X = X;
            rr.LX = LX;
            status = ST_DONE;
            break;
        }
        cD += dD;
        cE += dE + cEx;
        if (all.mn == 0xFFFFFFFFu) { status = ST_DONE; break; }          // condition 2
        if (p.max_cycles > 0 && (long long)cyc >= p.max_cycles) { status = ST_CANCELED; break; }
        t += all.mn;
        ++cyc;

        if (tid == 0) {
            s_sum = 0;
            s_nl = 0;
            s_sw = 0;
            s_bhn = 0;
            // atomic: other threads may still be flagging an overflow of the
            // candidate phase, and a lost flag would drop flows silently
            atomicAnd(&s_flags, SF_OVER);
            s_xkey = 0;
        }
        __syncthreads();
        // flows in transit after the sending round of the previous time
        {
            unsigned long long tr = 0;
            for (unsigned bk = tid; bk < W; bk += BLOCK) tr += cnt[bk];
            for (int o = 32; o > 0; o >>= 1) tr += __shfl_xor(tr, o);
            if (lane == 0 && tr) atomicAdd(&s_sum, tr);
        }

        // ---- Arrival (Steps 1-3 and 8, Algorithms 4-6, 10): deliver bucket t.
        {
            const unsigned bk = (unsigned)(t & Wm);
            F = (unsigned)min((unsigned long long)cnt[bk], S);
            // dense form when the bucket is large: the deliveries only mark
            // the bitmap, and a sweep builds the list (and the B check) after
            const bool dense = F > p.dense_thr;
            const uint2 *bkt = wheel + (unsigned long long)bk * S;
            constexpr int UA = 4;                   // flow loads in flight per thread
            for (unsigned j0 = tid; j0 < F; j0 += BLOCK * UA) {
                uint2 f[UA];
                unsigned fp[UA];
#pragma unroll
                for (int u = 0; u < UA; ++u) {
                    const unsigned j = j0 + u * BLOCK;
                    if (j < F) {
                        f[u] = bkt[j];
                        if constexpr (LOG) fp[u] = wptr[(unsigned long long)bk * S + j];
                    }
                }
#pragma unroll
                for (int u = 0; u < UA; ++u) {
                    if (j0 + u * BLOCK < F) {
                        const unsigned i = (unsigned)((long long)f[u].x - base);
                        const bool raised = lraise(lab, l16, i, f[u].y >> 3);
                        if constexpr (LOG) {
                            const unsigned q = f[u].y >> 3;
                            if (q >= lget(lab, l16, i))
                                atomicMax(&p.winner[base + i], ((unsigned long long)q << 35) |
                                                                   ((unsigned long long)(7u - (f[u].y & 7u)) << 32) | fp[u]);
                        }
                        if (raised) {
                            // the first raise of a vertex this cycle puts it in I_t
                            const unsigned bit = 1u << (i & 31);
                            if (dense) {
                                atomicOr(&fb[i >> 5], bit);
                            } else if (!(atomicOr(&fb[i >> 5], bit) & bit)) {
                                const unsigned long long am = __ballot(1);
                                const int ld = __ffsll((long long)am) - 1;
                                unsigned k0 = 0;
                                if ((int)lane == ld) k0 = atomicAdd(&s_nl, (unsigned)__popcll(am));
                                const unsigned k = (unsigned)__builtin_amdgcn_readlane((int)k0, ld) + (unsigned)__popcll(am & ((1ull << lane) - 1ull));
                                list_put(k, i);
                                if (bb[i >> 5] & bit) atomicAdd(&s_bhn, 1u);
                            }
                        }
                    }
                }
            }
            if (tid == 0) cR += F;
            __syncthreads();
            nlist = s_nl;
            if (s_bhn) {
                // a vertex of B improved: best (label, -index) over them, with
                // the labels after every delivery of this cycle
                unsigned long long bestB = 0;
                for (unsigned j = tid; j < nlist; j += BLOCK) {
                    const unsigned i = list_get(j);
                    if (bb[i >> 5] & (1u << (i & 31))) {
                        const unsigned long long key = ((unsigned long long)lget(lab, l16, i) << 32) |
                                                       (0xFFFFFFFFull - (unsigned long long)gvert(i));
                        bestB = key > bestB ? key : bestB;
                    }
                }
                for (int o = 32; o > 0; o >>= 1) {
                    const unsigned long long ob = __shfl_xor(bestB, o);
                    bestB = ob > bestB ? ob : bestB;
                }
                if (lane == 0 && bestB) {
                    atomicMax(&s_xkey, bestB);
                    atomicOr(&s_flags, SF_BHIT);
                }
            }
            // a large I_t is rebuilt in vertex order (the same set)
            if (dense) nlist = sweep();
            if (tid == 0) {
                cnt[bk] = 0;
                cU += nlist;
            }
            __syncthreads();
            transit = s_sum;
            // the next barrier's sums and B key, long before it
            if (tid == 0) gang_or_post(p.bar, G, r, epoch, F, nlist, transit, s_xkey);
            if constexpr (LOG) log_improved(t, nlist, false);
        }
        PHASE4(3);
    }
#undef PHASE4

    // ---- outputs
    if (status == ST_DONE && p.labels_out) {
        for (unsigned i = tid; i < cr; i += BLOCK) {
            const long long v = gvert(i);
            if (v >= 0) p.labels_out[v] = lget(lab, l16, i);
        }
    }
    __syncthreads();
    if (tid == 0) {
        for (int i = 0; i < 4; ++i) s_red[i] = 0;
    }
    __syncthreads();
    if (cU) atomicAdd(&s_red[0], cU);
    if (cD) atomicAdd(&s_red[1], cD);
    if (cE) atomicAdd(&s_red[2], cE);
    if (cR) atomicAdd(&s_red[3], cR);
    __syncthreads();
    if (tid == 0) {
        if (s_red[0]) atomicAdd(&out->ctr[1], s_red[0]);
        if (s_red[1]) atomicAdd(&out->ctr[2], s_red[1]);
        if (s_red[2]) atomicAdd(&out->ctr[3], s_red[2]);
        if (s_red[3]) atomicAdd(&out->ctr[4], s_red[3]);
        if (p.prof == 2) {
            for (int i = 0; i < 6; ++i) {
                atomicAdd(&out->psum[i], ph[i]);
                atomicMax(&out->pmax[i], ph[i]);
            }
        }
        if (lead) {
            for (int i = 0; i < 6; ++i) out->prof[i] = ph[i];
            out->ctr[0] = s_lc[0];
            out->ctr[5] = s_lc[1];
            out->ctr[6] = s_lc[2];
            out->trace_rows = (long long)s_lc[3];
            const int br = __hip_atomic_load(&p.bar->broken, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            out->status = br ? ST_BROKEN : status;
            if (status == ST_DONE && !found) {
                for (int i = 0; i < 5; ++i) out->res[i] = -1;
            }
        }
    }
    __syncthreads();
    rr.status = status;
    rr.found = found ? 1 : 0;
    rr.t = t;
    rr.yd = s_ydir;
    __syncthreads();
    return rr;
}

// Single solve: the whole grid is one gang; range r of physical block b is
// chosen so that each XCD (blocks b = x mod 8) holds a contiguous run.
template <int D, bool TILE = false, bool LOG = false>
__global__ void __launch_bounds__(BLOCK) k_ranges(RJ p)
{
    extern __shared__ unsigned smem[];
    const unsigned G = gridDim.x;
    const unsigned r = (G % NGRP) == 0 ? (blockIdx.x % NGRP) * (G / NGRP) + blockIdx.x / NGRP : blockIdx.x;
    unsigned epoch = 0;
    (void)range_run<D, TILE, LOG>(p, r, smem, p.M, -1, epoch, p.out);
}

// Path of a logged solve, from X back to A: follow the parent records.
// Stops after cap vertices (a path never has more than min(M, N)) or at a
// record index outside the log (then *len = -1).
__global__ void k_walk(const uint4 *log, unsigned long long nlog, long long xrec, long long *path, long long cap,
                       long long *len)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    long long k = 0;
    unsigned idx = (unsigned)xrec;
    while (k < cap && idx != 0xFFFFFFFFu && idx < nlog) {
        const uint4 rec = log[idx];
        path[k++] = rec.y;
        idx = rec.x;
    }
    *len = idx == 0xFFFFFFFFu ? k : -1;
}

// Batched solves in one persistent launch.  Work is a list of (job, range)
// slots ordered so that each job's ranges are consecutive and large jobs
// come first; a workgroup takes the next slot with one atomic and runs that
// range, meeting the rest of the job's gang at its barriers.  Every slot of
// a gang is taken by a workgroup that finishes its earlier slots without
// waiting on later ones, so every gang completes.
struct BatchArgs {
    const RJ *jobs;
    const unsigned *slot_job;
    const unsigned *slot_range;
    unsigned nslots;
    unsigned *next;                // slot counter
};

template <int D>
__global__ void __launch_bounds__(BLOCK) k_batch(BatchArgs a)
{
    extern __shared__ unsigned smem[];
    __shared__ unsigned s_slot;
    for (;;) {
        if (threadIdx.x == 0) s_slot = atomicAdd(a.next, 1u);
        __syncthreads();
        const unsigned sl = __builtin_amdgcn_readfirstlane(s_slot);
        __syncthreads();
        if (sl >= a.nslots) break;
        const unsigned jb = __builtin_amdgcn_readfirstlane(a.slot_job[sl]);
        const unsigned r = __builtin_amdgcn_readfirstlane(a.slot_range[sl]);
        const RJ &job = a.jobs[jb];
        unsigned epoch = 0;
        (void)range_run<D>(job, r, smem, job.M, -1, epoch, job.out);
    }
}

// ---------------------------------------------------------------------------
// Serving: one persistent, cooperative launch (every worker resident) that
// keeps taking solves while it runs.
//
// The host publishes jobs in host-coherent (fine-grained) memory: a job
// table, a ring of (job, range) slots and a tail counter.  Workers (one
// workgroup per CU) claim slots in order by compare-and-swap on a device
// word that holds the number of claimed slots, so a slot is taken only once
// it is published, and the host publishes all slots of a job at once.  One
// idle worker at a time (the watcher) reads the host's tail and mirrors it
// into device memory, so idle workers spin on L2 rather than on the bus.
// A job is the solve of its range, then, when asked, the reconstruction
// chain of section 1 and section 5 "Termination" (re-solve with B' = {Y} and M' = F2 - f2(x) + 1 until
// Y is in A), run by the same gang with the lattice still resident.  The
// last member to finish writes the completion record to host memory.
// Workers leave when the host raises stop, or when the host has not beaten
// its heartbeat for `stale` ticks, and only when every published slot has
// been claimed, so no gang is ever left short of members.
// ---------------------------------------------------------------------------

// Completion record of a served job (host-coherent memory).
struct Done {
    long long res[5];                  // T X x Y F2 of the first solve
    unsigned long long ctr[8];         // counters of the first solve
    unsigned long long ctr_chain[8];   // reconstruction solves (U D E R summed)
    long long path_len;
    long long solves;
    int status;
    int pad;
    unsigned long long seq;            // written last; the host waits for it
};

struct SJ {
    RJ rj;
    Out *out0;                         // first solve
    Out *outc;                         // reconstruction solves
    unsigned *done_cnt;                // members finished (zero between jobs)
    long long *path;                   // host-coherent; X, Y, Y', ... until A
    long long path_cap;
    unsigned *abits;                   // [g][cw] A bitmap of each range
    Done *done;                        // host-coherent
    unsigned long long seq;
    int recon;
    int pad;
};

// Host-coherent control block.
struct SrvCtl {
    unsigned long long tail;           // slots published
    unsigned long long heartbeat;
    unsigned stop;
    unsigned pad[27];
};

constexpr unsigned long long SRV_QUIT = 1ull << 63;

struct ServeArgs {
    const SJ *jobs;                    // host-coherent [max jobs]
    const unsigned *slots;             // host-coherent [ring][2] (job, range)
    unsigned ring;                     // power of two
    const SrvCtl *ctl;
    unsigned long long *state;         // device: claimed slots | SRV_QUIT
    unsigned long long *dtail;         // device mirror of ctl->tail
    unsigned *watch;                   // device: 1 while a watcher polls the host
    unsigned long long stale;          // wall-clock ticks
    unsigned max_jobs;
};

__device__ __forceinline__ unsigned long long ld_sys64(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ unsigned ld_sys32(const unsigned *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ void st_sys64(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ void st_sys64(long long *p, long long v)
{
    st_sys64(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v);
}

__device__ __forceinline__ bool cas64(unsigned long long *p, unsigned long long expect, unsigned long long want)
{
    return __hip_atomic_compare_exchange_strong(p, &expect, want, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
}

// Next slot for the calling worker (thread 0), or ~0 when the worker leaves.
__device__ unsigned long long serve_claim(const ServeArgs &a)
{
    bool watcher = false;
    unsigned long long hb_last = 0, t_seen = wall_clock64();
    for (;;) {
        const unsigned long long st = __hip_atomic_load(a.state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (st & SRV_QUIT) {
            if (watcher) __hip_atomic_store(a.watch, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return ~0ull;
        }
        unsigned long long tl = __hip_atomic_load(a.dtail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!watcher && st >= tl) {
            unsigned z = 0;
            watcher = __hip_atomic_compare_exchange_strong(a.watch, &z, 1u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
            if (watcher) {
                hb_last = ld_sys64(&a.ctl->heartbeat);
                t_seen = wall_clock64();
            }
        }
        if (watcher) {
            tl = ld_sys64(&a.ctl->tail);
            if (tl > __hip_atomic_load(a.dtail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                __hip_atomic_store(a.dtail, tl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (st < tl) {
            if (cas64(a.state, st, st + 1)) {
                if (watcher) __hip_atomic_store(a.watch, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                return st;
            }
            continue;
        }
        if (watcher) {
            const unsigned long long hb = ld_sys64(&a.ctl->heartbeat), now = wall_clock64();
            if (hb != hb_last) {
                hb_last = hb;
                t_seen = now;
            }
            if (ld_sys32(&a.ctl->stop) || now - t_seen > a.stale) {
                (void)cas64(a.state, st, st | SRV_QUIT);   // fails if a slot was claimed meanwhile
                continue;
            }
            __builtin_amdgcn_s_sleep(32);
        } else {
            __builtin_amdgcn_s_sleep(127);
        }
    }
}

template <int D>
__device__ __forceinline__ void serve_job(const SJ &sj, unsigned r, unsigned *smem)
{
    const RJ &p = sj.rj;
    const unsigned tid = threadIdx.x, G = p.g;
    if (r == 0 && tid == 0) {
        // before the gang's first barrier, which publishes it
        Out *o[2] = {sj.out0, sj.outc};
        for (int k = 0; k < 2; ++k) {
            for (int i = 0; i < 5; ++i) o[k]->res[i] = 0;
            for (int i = 0; i < 8; ++i) o[k]->ctr[i] = 0;
            o[k]->status = 0;
        }
    }
    unsigned epoch = 0;
    int status = ST_DONE;
    long long plen = 0, solves = 0;
    long long X = -1, T = 0, F2 = 0, bvert = -1;
    unsigned Mc = p.M, f1x = 0, f2x = 0, mf = 0;
    for (;;) {
        const RunRes rr = range_run<D>(p, r, smem, Mc, bvert, epoch, solves ? sj.outc : sj.out0, sj.abits, mf);
        mf = rr.mf;
        if (rr.status != ST_DONE) { status = rr.status; break; }
        if (solves == 0) {
            if (!rr.found || !sj.recon) break;
            if (r == 0 && tid == 0) st_sys64(&sj.path[0], (long long)rr.X);
            plen = 1;
        } else if (!rr.found || (long long)rr.X != bvert || rr.t != T - (long long)f1x ||
                   (long long)Mc - (long long)rr.LX != F2 - (long long)f2x) {
            status = ST_BROKEN;         // a re-solve must end at Y, f1(x) and f2(x) earlier
            break;
        }
        ++solves;
        X = rr.X;
        T = rr.t;
        F2 = (long long)Mc - (long long)rr.LX;
        // the direction of x is known to X's owner only
        Comb mine, all;
        mine.mn = rr.yd;
        mine.orf = 0;
        mine.s0 = mine.s1 = mine.s2 = mine.mx = 0;
        if (!gang_combine(p.bar, G, r, epoch, p.wait_limit, mine, all, false)) { status = ST_BROKEN; break; }
        const unsigned yd = all.mn;
        if (yd >= 2u * D || plen >= sj.path_cap) { status = ST_BROKEN; break; }
        long long oy = 0;
#pragma unroll
        for (int dd = 0; dd < 2 * D; ++dd)
            if ((unsigned)dd == yd) oy = dir_offset<D>(p.n, dd);
        const long long Y = X + oy;
        const bool lower = (int)yd < D;
        const int k = lower ? D - 1 - (int)yd : (int)yd - D;
        const long long x = (long long)k * p.N + (lower ? Y : X);
        if (r == 0 && tid == 0) st_sys64(&sj.path[plen], Y);
        ++plen;
        if (p.A[Y]) break;
        f1x = p.f1[x];
        f2x = p.f2[x];
        Mc = (unsigned)(F2 - (long long)f2x + 1);
        bvert = Y;
    }
    if (solves == 0) solves = 1;
    // Leave the barrier lines zero for the next job, then count out; the last
    // member publishes the completion.
    __syncthreads();
    if (tid == 0) {
        if (G > 1) {
            unsigned long long *sl = bar_slot(p.bar, r), *fl = bar_flag(p.bar, G, r);
            for (int k = 0; k < 16; ++k) {
                st64(&sl[k], 0);
                st64(&fl[k], 0);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        const unsigned a = __hip_atomic_fetch_add(sj.done_cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a == G - 1) {
            __hip_atomic_store(sj.done_cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const int br = __hip_atomic_load(&p.bar->broken, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            Done *dn = sj.done;
            for (int i = 0; i < 5; ++i) st_sys64(&dn->res[i], ld64(reinterpret_cast<const unsigned long long *>(&sj.out0->res[i])));
            for (int i = 0; i < 8; ++i) {
                st_sys64(&dn->ctr[i], ld64(&sj.out0->ctr[i]));
                st_sys64(&dn->ctr_chain[i], ld64(&sj.outc->ctr[i]));
            }
            st_sys64(&dn->path_len, plen);
            st_sys64(&dn->solves, solves);
            __hip_atomic_store(&dn->status, br ? (int)ST_BROKEN : status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
            st_sys64(&dn->seq, sj.seq);
        }
    }
    __syncthreads();
}

__global__ void __launch_bounds__(BLOCK) k_serve(ServeArgs a)
{
    extern __shared__ unsigned smem[];
    __shared__ SJ s_job;
    __shared__ unsigned long long s_slot;
    __shared__ unsigned s_jr[2];
    constexpr unsigned JW = sizeof(SJ) / 8;
    static_assert(sizeof(SJ) % 8 == 0, "job words");
    for (;;) {
        if (threadIdx.x == 0) s_slot = serve_claim(a);
        __syncthreads();
        const unsigned long long sl = s_slot;
        if (sl == ~0ull) break;
        if (threadIdx.x < 2) s_jr[threadIdx.x] = ld_sys32(&a.slots[2 * (sl & (a.ring - 1)) + threadIdx.x]);
        __syncthreads();
        const unsigned j = __builtin_amdgcn_readfirstlane(s_jr[0]), r = __builtin_amdgcn_readfirstlane(s_jr[1]);
        if (j >= a.max_jobs) continue;      // not a slot the host wrote
        const unsigned long long *src = reinterpret_cast<const unsigned long long *>(a.jobs + j);
        unsigned long long *dst = reinterpret_cast<unsigned long long *>(&s_job);
        for (unsigned i = threadIdx.x; i < JW; i += BLOCK) dst[i] = ld_sys64(src + i);
        __syncthreads();
        // the job's fields as wave-uniform values
        SJ pj;
        const unsigned *sw = reinterpret_cast<const unsigned *>(&s_job);
        unsigned *pw = reinterpret_cast<unsigned *>(&pj);
#pragma unroll
        for (unsigned i = 0; i < sizeof(SJ) / 4; ++i) pw[i] = __builtin_amdgcn_readfirstlane(sw[i]);
        __syncthreads();
        if (r >= pj.rj.g) continue;         // not a slot the host wrote
        switch (pj.rj.d) {
        case 1: serve_job<1>(pj, r, smem); break;
        case 2: serve_job<2>(pj, r, smem); break;
        case 3: serve_job<3>(pj, r, smem); break;
        default: serve_job<4>(pj, r, smem); break;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// General bounded-degree graphs (section 1 poses the problem on any graph;
// the lattice is the case studied).  Adjacency lists replace the lattice
// arithmetic: off[v] .. off[v+1] index nbr, f1, f2 and the edge id of each
// directed entry (both directions of every edge present).  Labels live in
// HBM and are raised with atomicMax; each workgroup files the flows it sends
// in its own wheel segment.  A delivery that raises a label stamps the
// vertex with the cycle; after the barrier each workgroup lists the stamped
// vertices of its own contiguous chunk, so departures follow the static
// partition whichever workgroup delivered.  A flow is (destination,
// quality, sender, adjacency entry), so the last edge x and its sender Y
// come out of the bucket delivered at T.  Per cycle: an arrival phase, a
// barrier (so departures read every delivery of t), the listing of I_t, the
// departure phase, and a combining barrier that returns the next time, the
// best B key and the counts.
// ---------------------------------------------------------------------------

struct GJ {
    long long nv, m;
    const long long *off;
    const int *nbr;
    const uint8_t *f1, *f2;
    const long long *eid;
    const uint8_t *A, *B;
    unsigned M;
    unsigned *lab;                 // [nv]
    unsigned *stamp;               // [nv] last cycle in which a delivery raised the label
    unsigned *lists;               // [G][qcap] I_t of each workgroup's chunk of vertices
    unsigned long long qcap;
    uint4 *pool;                   // [G][W][S] flows (dst, q, sender, adjacency entry)
    unsigned long long pool_flows;
    BarHdr *bar;
    Out *out;
    unsigned long long *xsel;      // (sender << 32 | entry) of x, by atomicMin
    unsigned *labels_out;
    long long max_cycles;
    unsigned long long wait_limit;
    int prof;                      // accumulate phase times in workgroup 0
};

__global__ void __launch_bounds__(BLOCK) k_graph(GJ p)
{
    __shared__ unsigned s_cnt[MAXW];
    __shared__ unsigned s_nl, s_flags, s_min, s_mf;
    __shared__ unsigned long long s_xkey, s_red[4];
    __shared__ unsigned long long s_lc[3];          // lead: C, P, I
    const unsigned tid = threadIdx.x, lane = lane_id();
    const unsigned G = gridDim.x;
    const unsigned r = (G % NGRP) == 0 ? (blockIdx.x % NGRP) * (G / NGRP) + blockIdx.x / NGRP : blockIdx.x;
    const bool lead = r == 0;
    const long long nv = p.nv;
    unsigned epoch = 0;
    unsigned *const list = p.lists + (unsigned long long)r * p.qcap;
    const long long c_chunk = (nv + G - 1) / G;
    const long long c_lo = min(nv, (long long)r * c_chunk), c_hi = min(nv, c_lo + c_chunk);
    unsigned long long cU = 0, cD = 0, cE = 0, cR = 0;

    for (unsigned i = tid; i < MAXW; i += BLOCK) s_cnt[i] = 0;
    if (tid == 0) {
        s_nl = 0;
        s_flags = 0;
        s_mf = 0;
        s_xkey = 0;
        for (int k = 0; k < 3; ++k) s_lc[k] = 0;
        if (lead) *p.xsel = ~0ull;          // published by the first barrier
    }
    __syncthreads();

    // append v to this workgroup's list (one LDS atomic per wave); over
    // capacity sets SF_OVER
    auto append = [&](unsigned v) {
        const unsigned long long am = __ballot(1);
        const int ld = __ffsll((long long)am) - 1;
        unsigned k0 = 0;
        if ((int)lane == ld) k0 = atomicAdd(&s_nl, (unsigned)__popcll(am));
        const unsigned k = __shfl(k0, ld) + (unsigned)__popcll(am & ((1ull << lane) - 1ull));
        if (k < p.qcap) list[k] = v;
        else atomicOr(&s_flags, SF_OVER);
    };

    // ---- Initialization (Algorithm 3) of this workgroup's chunk of vertices
    {
        const long long chunk = (nv + G - 1) / G;
        const long long lo = (long long)r * chunk, hi = min(nv, lo + chunk);
        unsigned mf = 0, bad = 0;
        for (long long v = lo + tid; v < hi; v += BLOCK) {
            const bool a = p.A[v] != 0, b = p.B[v] != 0;
            if (a && b) bad |= 2;
            // the adjacency arrays are checked here, before any cycle reads
            // them: entries j0 .. j1 - 1 must lie in [0, m) and name vertices
            const long long j0 = p.off[v], j1 = p.off[v + 1];
            if (j0 < 0 || j1 < j0 || j1 > p.m) {
                bad |= 2;
                continue;
            }
            for (long long j = j0; j < j1; ++j) {
                const unsigned x1 = p.f1[j], x2 = p.f2[j];
                if (!x1 || !x2) bad |= 1;
                if (p.nbr[j] < 0 || (long long)p.nbr[j] >= nv) bad |= 2;
                mf = x1 > mf ? x1 : mf;
            }
            p.lab[v] = a ? p.M : 0u;
            p.stamp[v] = 0xFFFFFFFFu;
            if (a) append((unsigned)v);
        }
        for (int o = 32; o > 0; o >>= 1) {
            mf = max(mf, (unsigned)__shfl_xor(mf, o));
            bad |= __shfl_xor(bad, o);
        }
        if (lane == 0) {
            if (mf) atomicMax(&s_mf, mf);
            if (bad & 1) atomicOr(&s_flags, SF_BAD);
            if (bad & 2) atomicOr(&s_flags, SF_INVAL);
        }
    }
    int status = ST_RUNNING;
    unsigned W = 2;
    {
        Comb mine, all;
        mine.mn = 0xFFFFFFFFu;
        __syncthreads();
        mine.orf = s_flags & (SF_BAD | SF_INVAL | SF_OVER);
        mine.s0 = mine.s1 = mine.s2 = 0;
        mine.mx = s_mf;
        if (!gang_combine(p.bar, G, r, epoch, p.wait_limit, mine, all, true)) status = ST_BROKEN;
        else if (all.orf & (SF_BAD | SF_INVAL)) status = ST_INVAL;
        else if (all.orf & SF_OVER) status = ST_OVERFLOW;
        while (W <= (unsigned)all.mx) W <<= 1;
    }
    const unsigned Wm = W - 1;
    const unsigned long long S = p.pool_flows / ((unsigned long long)G * W);
    uint4 *wheel = p.pool + (unsigned long long)r * W * S;
    unsigned nl = s_nl, F = 0, cyc = 0;
    long long t = 0;
    bool found = false;
    unsigned X = 0, LX = 0;
    unsigned long long ph[6] = {0, 0, 0, 0, 0, 0}, ph_t = 0;
    const bool timing = p.prof && lead && tid == 0;
#define GPHASE(k)                                            \
    do {                                                     \
        if (timing) {                                        \
            const unsigned long long now_ = wall_clock64();  \
            ph[k] += now_ - ph_t;                            \
            ph_t = now_;                                     \
        }                                                    \
    } while (0)
    if (timing) ph_t = wall_clock64();
    __syncthreads();

    while (status == ST_RUNNING) {
        // ---- Departure (Steps 4-5) from this workgroup's part of I_t; its
        // counts are committed unless the cycle turns out to be the last
        unsigned long long dD = 0, dE = 0;
        if (tid == 0) s_min = 0xFFFFFFFFu;
        __syncthreads();
        for (unsigned k = tid; k < nl; k += BLOCK) {
            const unsigned Q = list[k];
            const unsigned L = p.lab[Q];
            const long long j0 = p.off[Q], j1 = p.off[Q + 1];
            // neighbours in groups of GU: their entries, then their labels, are
            // loaded together, so a group costs two memory round trips
            constexpr int GU = 4;
            for (long long jb = j0; jb < j1; jb += GU) {
                unsigned P[GU], a1[GU], a2[GU], lp[GU];
#pragma unroll
                for (int u = 0; u < GU; ++u) {
                    const long long j = jb + u;
                    P[u] = j < j1 ? (unsigned)p.nbr[j] : 0u;
                    a1[u] = j < j1 ? (unsigned)p.f1[j] : 0u;
                    a2[u] = j < j1 ? (unsigned)p.f2[j] : 0u;
                }
#pragma unroll
                for (int u = 0; u < GU; ++u) lp[u] = jb + u < j1 ? p.lab[P[u]] : 0xFFFFFFFFu;
#pragma unroll
                for (int u = 0; u < GU; ++u) {
                    const long long j = jb + u;
                    if (j >= j1) continue;
                    ++dD;
                    const int q = (int)L - (int)a2[u];
                    if (q > 0 && (unsigned)q > lp[u]) {
                        const unsigned bk = (unsigned)((t + a1[u]) & Wm);
                        const unsigned pos = atomicAdd(&s_cnt[bk], 1u);
                        if (pos < S)
                            wheel[(unsigned long long)bk * S + pos] = make_uint4(P[u], (unsigned)q, Q, (unsigned)j);
                        else
                            atomicOr(&s_flags, SF_OVER);
                        ++dE;
                    }
                }
            }
        }
        __syncthreads();
        GPHASE(0);
        unsigned long long transit = 0;
        {
            unsigned best = 0xFFFFFFFFu;
            for (unsigned bk = tid; bk < W; bk += BLOCK) {
                const unsigned v = s_cnt[bk];
                if (v) {
                    best = min(best, (unsigned)((bk - (unsigned)t) & Wm));
                    transit += v;
                    if (v > S) atomicOr(&s_flags, SF_OVER);
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                best = min(best, (unsigned)__shfl_xor(best, o));
                transit += __shfl_xor(transit, o);
            }
            if (tid == 0) s_red[0] = 0;
            __syncthreads();
            if (lane == 0) {
                if (best != 0xFFFFFFFFu) atomicMin(&s_min, best);
                if (transit) atomicAdd(&s_red[0], transit);
            }
            __syncthreads();
            transit = s_red[0];
        }
        Comb mine, all;
        mine.mn = s_min;
        mine.orf = s_flags & (SF_OVER | SF_BHIT);
        mine.s0 = F;
        mine.s1 = nl;
        mine.s2 = transit;
        mine.mx = s_xkey;
        if (!gang_combine(p.bar, G, r, epoch, p.wait_limit, mine, all, false)) { status = ST_BROKEN; break; }
        GPHASE(1);
        if (all.orf & SF_OVER) { status = ST_OVERFLOW; break; }
        if (lead && tid == 0) {
            const unsigned long long a0 = all.rest ? ld64(&all.rest[0]) : all.s0;
            const unsigned long long a1 = all.rest ? ld64(&all.rest[1]) : all.s1;
            const unsigned long long a2 = all.rest ? ld64(&all.rest[2]) : all.s2;
            cU += a1;
            if (cyc > 0) {
                s_lc[0] += a0 > 0 ? 1 : 0;
                s_lc[2] = a1 > s_lc[2] ? a1 : s_lc[2];
            }
            // in transit after this sending round, unless the round is the last
            if (!(all.orf & SF_BHIT)) s_lc[1] = a2 > s_lc[1] ? a2 : s_lc[1];
        }
        if (all.orf & SF_BHIT) {
            // ---- Step 6 (Algorithm 2): T = t; x from the bucket delivered at t.
            found = true;
            X = (unsigned)(0xFFFFFFFFull - (all.mx & 0xFFFFFFFFull));
            LX = (unsigned)(all.mx >> 32);
            const uint4 *bkt = wheel + (unsigned long long)(t & Wm) * S;
            for (unsigned k = tid; k < F; k += BLOCK) {
                const uint4 f = bkt[k];
                if (f.x == X && f.y == LX) atomicMin(p.xsel, ((unsigned long long)f.z << 32) | f.w);
            }
            status = ST_DONE;
            break;
        }
        cD += dD;
        cE += dE;
        if (all.mn == 0xFFFFFFFFu) { status = ST_DONE; break; }            // condition 2
        if (p.max_cycles > 0 && (long long)cyc >= p.max_cycles) { status = ST_CANCELED; break; }
        t += all.mn;
        ++cyc;

        // ---- Arrival (Steps 1-3, 8): deliver this workgroup's bucket t
        const unsigned bk = (unsigned)(t & Wm);
        F = (unsigned)min((unsigned long long)s_cnt[bk], S);
        const uint4 *bkt = wheel + (unsigned long long)bk * S;
        if (tid == 0) {
            s_nl = 0;
            s_flags &= SF_OVER;
            s_xkey = 0;
        }
        __syncthreads();
        for (unsigned k0 = tid; k0 < F; k0 += 4 * BLOCK) {
            uint4 f[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (k0 + u * BLOCK < F) f[u] = bkt[k0 + u * BLOCK];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (k0 + u * BLOCK >= F) continue;
                if (f[u].y <= p.lab[f[u].x]) continue;          // cannot raise the label
                const unsigned old = atomicMax(&p.lab[f[u].x], f[u].y);
                if (f[u].y > old) p.stamp[f[u].x] = cyc;        // joins I_t; its owner lists it
            }
        }
        cR += tid == 0 ? F : 0;
        __syncthreads();
        GPHASE(3);
        if (tid == 0) s_cnt[bk] = 0;
        // every delivery of t lands before any departure reads a label
        {
            Comb m2, a2;
            m2.mn = 0xFFFFFFFFu;
            m2.orf = s_flags & SF_OVER;
            m2.s0 = m2.s1 = m2.s2 = m2.mx = 0;
            if (!gang_combine(p.bar, G, r, epoch, p.wait_limit, m2, a2, false)) { status = ST_BROKEN; break; }
            if (a2.orf & SF_OVER) { status = ST_OVERFLOW; break; }
        }
        GPHASE(4);
        // I_t of this workgroup's vertices: those stamped with this cycle, listed
        // by their owner so the departures follow the static partition; with it,
        // the vertices of B among them: best (label, -index) with final labels
        {
            unsigned long long bestB = 0;
            for (long long v0 = c_lo + tid; v0 < c_hi; v0 += 4 * BLOCK) {
                unsigned st[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) st[u] = v0 + u * BLOCK < c_hi ? p.stamp[v0 + u * BLOCK] : 0xFFFFFFFFu;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const long long v = v0 + u * BLOCK;
                    if (__ballot(st[u] == cyc) == 0) continue;      // wave-uniform skip
                    if (st[u] != cyc) continue;
                    append((unsigned)v);
                    if (p.B[v]) {
                        const unsigned long long key = ((unsigned long long)p.lab[v] << 32) | (0xFFFFFFFFull - v);
                        bestB = key > bestB ? key : bestB;
                    }
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const unsigned long long ob = __shfl_xor(bestB, o);
                bestB = ob > bestB ? ob : bestB;
            }
            if (lane == 0 && bestB) {
                atomicMax(&s_xkey, bestB);
                atomicOr(&s_flags, SF_BHIT);
            }
            __syncthreads();
            nl = s_nl;
        }
        GPHASE(5);
    }
#undef GPHASE

    // ---- outputs; the selection of x needs every workgroup's bucket scan
    if (found) {
        Comb m3, a3;
        m3.mn = 0xFFFFFFFFu;
        m3.orf = 0;
        m3.s0 = m3.s1 = m3.s2 = m3.mx = 0;
        if (!gang_combine(p.bar, G, r, epoch, p.wait_limit, m3, a3, false)) status = ST_BROKEN;
    }
    if (status == ST_DONE && p.labels_out) {
        const long long chunk = (nv + G - 1) / G;
        const long long lo = (long long)r * chunk, hi = min(nv, lo + chunk);
        for (long long v = lo + tid; v < hi; v += BLOCK) p.labels_out[v] = p.lab[v];
    }
    __syncthreads();
    if (tid == 0)
        for (int i = 0; i < 4; ++i) s_red[i] = 0;
    __syncthreads();
    if (cD) atomicAdd(&s_red[1], cD);
    if (cE) atomicAdd(&s_red[2], cE);
    if (cR) atomicAdd(&s_red[3], cR);
    __syncthreads();
    if (tid == 0) {
        Out *out = p.out;
        if (s_red[1]) atomicAdd(&out->ctr[2], s_red[1]);
        if (s_red[2]) atomicAdd(&out->ctr[3], s_red[2]);
        if (s_red[3]) atomicAdd(&out->ctr[4], s_red[3]);
        if (p.prof == 2) {
            for (int i = 0; i < 6; ++i) {
                atomicAdd(&out->psum[i], ph[i]);
                atomicMax(&out->pmax[i], ph[i]);
            }
        }
        if (lead) {
            for (int i = 0; i < 6; ++i) out->prof[i] = ph[i];
            out->ctr[0] = s_lc[0];
            out->ctr[1] = cU;
            out->ctr[5] = s_lc[1];
            out->ctr[6] = s_lc[2];
            const int br = __hip_atomic_load(&p.bar->broken, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            out->status = br ? ST_BROKEN : status;
            if (status == ST_DONE && found) {
                const unsigned long long xs = __hip_atomic_load(p.xsel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const unsigned Y = (unsigned)(xs >> 32), j = (unsigned)xs;
                if (xs == ~0ull || (long long)j >= p.m) {
                    out->status = ST_BROKEN;
                } else {
                    out->res[0] = t;
                    out->res[1] = X;
                    out->res[2] = p.eid[j];
                    out->res[3] = Y;
                    out->res[4] = (long long)p.M - (long long)LX;
                }
            } else if (status == ST_DONE) {
                for (int i = 0; i < 5; ++i) out->res[i] = -1;
            }
        }
    }
}

// Clear the quit bit and the watcher flag before a serving launch.
// ---------------------------------------------------------------------------
// Micro-benchmarks of the device resources the cycle is bound by (csp_microbench)
// ---------------------------------------------------------------------------

__device__ __forceinline__ unsigned mb_hash(unsigned x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

__global__ void __launch_bounds__(256) k_mb_copy(const uint4 *src, uint4 *dst, unsigned long long n)
{
    for (unsigned long long i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (unsigned long long)gridDim.x * 256ull)
        dst[i] = src[i];
}

// n atomic maxima at hashed positions of an array of `words` (a power of two)
__global__ void __launch_bounds__(256) k_mb_atomic(unsigned *a, unsigned long long words, unsigned long long n)
{
    for (unsigned long long i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (unsigned long long)gridDim.x * 256ull)
        atomicMax(&a[mb_hash((unsigned)i) & (words - 1)], (unsigned)i);
}

// per workgroup and round, nr 16-byte loads at hashed positions of its own
// slab of 65,536 records (1 MiB), four in flight per thread
__global__ void __launch_bounds__(BLOCK) k_mb_loads(const uint4 *rec, int nr, int rounds, int lg, unsigned *sink)
{
    const unsigned tid = threadIdx.x, r = blockIdx.x, mask = (1u << lg) - 1u;
    const uint4 *my = rec + ((size_t)r << lg);
    unsigned acc = 0;
    for (int it = 0; it < rounds; ++it) {
        for (int j0 = (int)tid; j0 < nr; j0 += BLOCK * 4) {
            uint4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = j0 + u * BLOCK;
                if (j < nr) v[u] = my[mb_hash((unsigned)(j * 977 + it * 131) + r) & mask];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (j0 + u * BLOCK < nr) acc ^= v[u].x ^ v[u].w;
        }
        __syncthreads();
    }
    if (acc == 0x9E3779B9u) sink[0] = acc;      // keeps the loads
}

// `iters` barriers among the grid: kind 0 the cycle loop's (gang_or), kind 1
// the fully fenced tree (gang_combine) after each member wrote `dirty_words`
// words of its own region with plain stores.  Every barrier's combined
// minimum is checked; a wrong one marks the gang broken.
__global__ void __launch_bounds__(BLOCK) k_mb_barrier(BarHdr *bh, int kind, int iters, unsigned *dirty,
                                                      unsigned long long dirty_words, unsigned long long limit)
{
    const unsigned G = gridDim.x, m = blockIdx.x;
    unsigned epoch = 0;
    if (m == 0) {
        for (unsigned i = threadIdx.x; i < 2 * 16 + 2 + 4 * 16 * 3 + 1; i += BLOCK) {
            unsigned long long *w = i < 32 ? &bh->ow[i / 16][i % 16][0]
                                    : i < 34 ? &bh->oroot[i - 32][0]
                                    : i < 34 + 192 ? &bh->ring[(i - 34) / 48][(i - 34) / 3 % 16][(i - 34) % 3][0]
                                                   : &bh->bkey[0];
            st64(w, 0ull);
        }
    }
    Comb mine, all;
    mine.orf = 0;
    mine.s0 = mine.s1 = mine.s2 = mine.mx = 0;
    mine.mn = 0xFFFFFFFFu;
    if (!gang_combine(bh, G, m, epoch, limit, mine, all, false)) return;
    for (int it = 0; it < iters; ++it) {
        // member (it mod G) has the least delta, 1 + (it mod 5); the others 30
        mine.mn = m == (unsigned)it % G ? 1u + (unsigned)it % 5u : 30u;
        bool ok;
        if (kind == 0) {
            ok = gang_or(bh, G, m, epoch, limit, mine, all);
        } else {
            unsigned *d = dirty + (size_t)m * dirty_words;
            for (unsigned long long i = threadIdx.x; i < dirty_words; i += BLOCK) d[i] = (unsigned)it;
            ok = gang_combine(bh, G, m, epoch, limit, mine, all, false);
        }
        if (!ok) return;
        if (all.mn != 1u + (unsigned)it % 5u) {
            if (threadIdx.x == 0) __hip_atomic_store(&bh->broken, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
    }
}

__global__ void k_serve_reset(unsigned long long *state, unsigned *watch)
{
    *state &= ~SRV_QUIT;
    *watch = 0;
}

__global__ void k_set_byte(uint8_t *p, long long i, uint8_t v) { p[i] = v; }

// Zero `words` 32-bit words (a kernel rather than a memset, so the sequence
// stays valid inside captured graphs).
__global__ void __launch_bounds__(256) k_zero(unsigned *p, unsigned long long words)
{
    const unsigned long long gs = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gs)
        p[i] = 0;
}

size_t rec_bytes(int d) { return d == 1 ? 4 : (d == 2 ? 8 : 16); }

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

// Device state of csp_solve_dev_noalloc: one array on every GPU the library
// runs on, held until the process ends.  Host code never uses this name as
// an address: each device's copy is reached through the pointer that
// hipGetSymbolAddress returned for it (scratch_dev).
static __device__ __align__(256) uint8_t scratch[CSP_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_DEVICES = 64;
std::mutex scratch_mu;
uint8_t *scratch_dev[SCRATCH_DEVICES] = {};   // per device: address of its copy of scratch
}  // namespace

struct csp_ctx {
    int device = 0;
    uint8_t *scratch = nullptr;     // this device's copy of the static scratch (null: unavailable)
    int num_cu = 0;
    int max_blocks[5] = {0, 0, 0, 0, 0};
    unsigned long long wall_khz = 100000;
    unsigned *lab = nullptr;
    size_t lab_cap = 0;
    // general graphs
    unsigned *gstamp = nullptr, *glists = nullptr;
    size_t gstamp_cap = 0, glists_cap = 0;
    uint4 *gpool = nullptr;
    size_t gpool_cap = 0;
    unsigned long long gpool_seen = 0;
    uint8_t *rec = nullptr;
    size_t rec_cap = 0;
    unsigned *queue = nullptr;
    size_t queue_cap = 0;
    uint2 *pool = nullptr;
    size_t pool_cap = 0;            // flows
    Ctl *ctl = nullptr;
    Ctl *h_ctl = nullptr;           // pinned
    uint8_t *in_buf = nullptr;      // staging for host-pointer solves
    size_t in_cap = 0;
    uint8_t *h_byte = nullptr;      // pinned scratch
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    float last_ms = -1.f;
    unsigned long long last_prof[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    unsigned long long last_psum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    unsigned long long last_pmax[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    long long last_spread_ranges = 0;
    int prof = 0;
    unsigned long long pool_hint = 0;
    int blocks_override = 0;
    int path_override = 0;          // 0 auto, 1 LDS ranges, 2 global labels, 3 LDS pencils
    // autotuned (blocks, path) per lattice shape, used when no override is set
    struct Tuned {
        int d;
        long long N;
        int blocks, path;
        float ms;
        long long dense;            // dense threshold (-1: automatic)
    };
    long long dense_override = -1;  // -1 automatic, else the threshold for later solves
    long long wait_us = -1;         // -1 default (20 s), else the barrier wait limit of later solves
    std::vector<Tuned> tuned;
    long long batch_target = 0;     // batch: vertices per workgroup (0 = fewest workgroups)
    // batch: wheel pool and candidate capacity a problem (same lattice, masks
    // and M at the same addresses) needed in an earlier batch, so a repeated
    // problem starts with them instead of overflowing and running again
    std::map<std::tuple<int, long long, unsigned, const void *, const void *, const void *, const void *>,
             std::pair<unsigned long long, unsigned long long>>
        batch_seen;
    long long *trace = nullptr;     // device [trace_cap][4], or null
    long long trace_cap = 0;
    long long last_trace_rows = 0;
    int last_path = 0;
    size_t lds_limit = 65536;
    unsigned long long *pub = nullptr;   // candidate fills [2][G][NOMAX]
    size_t pub_cap = 0;
    uint2 *cand = nullptr;          // candidates [2][G][NO][cap]
    size_t cand_cap = 0;
    // improvement log (csp_reconstruct_log_dev)
    unsigned *wptr = nullptr, *cptr = nullptr, *cur = nullptr;
    size_t wptr_cap = 0, cptr_cap = 0, cur_cap = 0;
    unsigned long long *winner = nullptr;
    size_t winner_cap = 0;
    uint4 *logbuf = nullptr;
    size_t logbuf_cap = 0;
    unsigned long long log_seen = 0;   // records per range a logged solve needed so far
    long long *walk = nullptr;         // [cap + 1] path from X back, then its length
    size_t walk_cap = 0;
    long long last_xrec = -1;
    unsigned long long cand_seen = 0;
    unsigned long long pool_flows_seen = 0;   // largest pool a solve needed so far
    uint8_t *arena = nullptr;       // batch: per-problem device state
    size_t arena_cap = 0;
    uint8_t *h_stage = nullptr;     // batch: pinned staging for job tables and results
    size_t h_stage_cap = 0;
    char err[256] = {0};
};

namespace {

int fail(csp_ctx *ctx, int code, const char *what, hipError_t e = hipSuccess)
{
    if (ctx) {
        if (e != hipSuccess)
            snprintf(ctx->err, sizeof(ctx->err), "%s: %s", what, hipGetErrorString(e));
        else
            snprintf(ctx->err, sizeof(ctx->err), "%s", what);
    }
    return code;
}

#define HIP_TRY(call, what)                                            \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) return fail(ctx, CSP_EDEVICE, what, e_); \
    } while (0)

template <class T>
int grow(csp_ctx *ctx, T **p, size_t &cap, size_t need, const char *what)
{
    if (need <= cap && *p) return CSP_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    cap = 0;
    hipError_t e = hipMalloc((void **)p, need * sizeof(T));
    if (e != hipSuccess) return fail(ctx, CSP_ENOMEM, what, e);
    cap = need;
    return CSP_OK;
}

const void *lds_kernel(int d, int tile, bool log = false)
{
    if (log) {
        switch (d) {
        case 1: return (const void *)k_ranges<1, false, true>;
        case 2: return (const void *)k_ranges<2, false, true>;
        case 3: return tile ? (const void *)k_ranges<3, true, true> : (const void *)k_ranges<3, false, true>;
        default: return (const void *)k_ranges<4, false, true>;
        }
    }
    switch (d) {
    case 1: return (const void *)k_ranges<1>;
    case 2: return (const void *)k_ranges<2>;
    case 3: return tile ? (const void *)k_ranges<3, true> : (const void *)k_ranges<3>;
    default: return (const void *)k_ranges<4>;
    }
}

const void *batch_kernel(int d)
{
    switch (d) {
    case 1: return (const void *)k_batch<1>;
    case 2: return (const void *)k_batch<2>;
    case 3: return (const void *)k_batch<3>;
    default: return (const void *)k_batch<4>;
    }
}

// Layout of a range-owned solve: G ranges of c vertices, neighbours within K
// ranges, LT-byte LDS labels, dynamic LDS bytes.
struct LdsPlan {
    bool ok = false;
    int G = 1;
    long long c = 0;
    int K = 0;
    int lt = 4;
    int llist = 0;
    int tile = 0;                   // d = 3: x-pencils of n x ty x tz
    int ty = 0, tz = 0, nty = 0;
    size_t lds = 0;
};

// LDS bytes of a range's frontier list (16-bit local indices)
size_t lds_list_bytes(long long c) { return (size_t)(((c * 2) + 3) / 4 * 4); }

// Frontier-list entries a range of c vertices keeps in LDS beside `need`
// bytes (the list is usually far shorter than the range); 16-bit local
// indices need c <= 65536.
long long lds_list_cap(long long c, size_t need, size_t budget)
{
    if (c > 65536 || need >= budget) return 0;
    const long long room = (long long)((budget - need) / 4) * 2;
    return std::min(c, room);
}

size_t lds_bytes_for(long long c, int K, int lt)
{
    (void)K;
    const long long cw = (c + 31) / 32;
    const long long lab_words = (c * lt + 3) / 4;
    return (size_t)(4 * (lab_words + 2 * cw + MAXW));
}

LdsPlan plan_lds(const csp_ctx *ctx, int d, long long n, long long N, uint32_t M, int G_want, int path);

const void *solve_kernel(int d)
{
    switch (d) {
    case 1: return (const void *)k_solve<1>;
    case 2: return (const void *)k_solve<2>;
    case 3: return (const void *)k_solve<3>;
    default: return (const void *)k_solve<4>;
    }
}

int check_shape(csp_ctx *ctx, int d, int64_t n, uint32_t M, long long &N)
{
    if (d < 1 || d > 4) return fail(ctx, CSP_EINVAL, "d must be 1..4");
    if (n < 2) return fail(ctx, CSP_EINVAL, "n must be >= 2");
    long long v = 1;
    for (int k = 0; k < d; ++k) {
        if (v > (1ll << 31) / n) return fail(ctx, CSP_EINVAL, "n^d must be below 2^31");
        v *= n;
    }
    if (v >= (1ll << 31)) return fail(ctx, CSP_EINVAL, "n^d must be below 2^31");
    if (M < 1 || M > CSP_MAX_M) return fail(ctx, CSP_EINVAL, "M out of range");
    N = v;
    return CSP_OK;
}

const csp_ctx::Tuned *tuned_for(const csp_ctx *ctx, int d, long long N)
{
    for (const auto &e : ctx->tuned)
        if (e.d == d && e.N == N) return &e;
    return nullptr;
}

// Kernel path of a solve: the override, else the autotuned one, else
// x-pencil ranges for 3-d lattices of 2^23 vertices or more and the
// automatic choice below that.  Pencils ship candidates only across their
// y and z faces (a quarter or less of the cross-range tests of whole-plane
// ranges); measured on MI355X they win on the 256^3 cubes (sparse 307.3 ->
// 286.6 ms, stress 9.42 -> 8.82 ms) and lose on the 128^3 cubes (+3 %) and
// the paper's 50^3..125^3 cubes (+7 %), whose ranges are smaller.
int path_for(const csp_ctx *ctx, int d, long long N)
{
    if (ctx->path_override) return ctx->path_override;
    const csp_ctx::Tuned *e = tuned_for(ctx, d, N);
    if (e && e->path) return e->path;              // 0 recorded: the automatic choice won
    return d == 3 && N >= (1ll << 23) ? 3 : 0;
}

int blocks_for(csp_ctx *ctx, int d, long long N)
{
    if (ctx->blocks_override > 0) return std::min(ctx->blocks_override, ctx->max_blocks[d]);
    if (const csp_ctx::Tuned *e = tuned_for(ctx, d, N)) return std::min(e->blocks, ctx->max_blocks[d]);
    // Few vertices: one workgroup (its barrier is a workgroup barrier).
    // Otherwise about one workgroup per 8K vertices, up to one per CU.
    long long want = (N + 8191) / 8192;
    if (N <= 32768) want = 1;
    return (int)std::max(1ll, std::min(want, (long long)ctx->max_blocks[d]));
}

LdsPlan plan_lds(const csp_ctx *ctx, int d, long long n, long long N, uint32_t M, int G_want, int path)
{
    LdsPlan pl;
    long long smax = 1;
    for (int k = 1; k < d; ++k) smax *= n;           // largest neighbour offset
    const size_t budget = ctx->lds_limit > 4096 ? ctx->lds_limit - 4096 : 0;   // static LDS margin
    // 3-d lattices on request: x-pencils (every range spans x, so a front
    // moving along x is shared by all ranges, and only the y and z faces of a
    // pencil ship candidates), m x m pencils with m^2 close to G_want.  They
    // ship about a quarter of the candidates of whole-plane ranges but
    // measured slower on MI355X (more spread in per-range departure work),
    // so consecutive-index ranges are the default.
    if (d == 3 && G_want >= 4 && path == 3) {
        int m = 1;
        while ((m + 1) * (m + 1) <= G_want) ++m;
        for (; m >= 2; --m) {
            const long long t = (n + m - 1) / m, mm = (n + t - 1) / t;
            const long long c = n * t * t;
            bool done = false;
            for (int lt : {4, 2}) {
                if (lt == 2 && M > 0xFFFFu) continue;
                const size_t need = lds_bytes_for(c, 0, lt);
                if (c <= 0x1FFFF && need <= budget) {
                    pl.ok = true;
                    pl.G = (int)(mm * mm);
                    pl.c = c;
                    pl.K = 0;
                    pl.lt = lt;
                    pl.tile = 1;
                    pl.ty = pl.tz = (int)t;
                    pl.nty = (int)mm;
                    pl.llist = (int)lds_list_cap(c, need, budget);
                    pl.lds = need + lds_list_bytes(pl.llist);
                    done = true;
                    break;
                }
            }
            if (done) return pl;
        }
    }
    for (int G = std::max(1, G_want); G >= 1; G = (G > 1 ? G / 2 : 0)) {
        const long long c = (N + G - 1) / G;
        if ((long long)(G - 1) * c >= N) continue;    // empty range
        const int K = G == 1 ? 0 : (int)((smax + c - 1) / c);
        if (K > KMAX) continue;
        for (int lt : {4, 2}) {
            if (lt == 2 && M > 0xFFFFu) continue;
            const size_t need = lds_bytes_for(c, K, lt);
            if (need <= budget) {
                pl.ok = true;
                pl.G = G;
                pl.c = c;
                pl.K = K;
                pl.lt = lt;
                pl.llist = (int)lds_list_cap(c, need, budget);
                pl.lds = need + lds_list_bytes(pl.llist);
                return pl;
            }
        }
        if (G == 1) break;
    }
    return pl;
}

// Automatic dense threshold of a range of c vertices: a range of 32,768
// vertices or more builds I_t in dense form in the cycles where more than
// 4,096 flows are delivered to it; smaller ranges keep the append list.  The
// dense form saves the append's dependent LDS round trips on every first
// raise and costs a sweep of the whole bitmap, so it pays only on large
// buckets of large ranges: on the 256^3 cube 4,096 beat 0, 2,048, 8,192 and
// never (253 against 254, 255, 256 and 266 ms); on the 128^3 cubes (8,192
// vertices per range) never and 8,192 were fastest (5.72 against 5.95 ms at
// 4,096).
unsigned dense_default(long long c)
{
    return c >= 32768 ? 4096u : DENSE_NEVER;
}

// Dense threshold of a single solve: the override, else the autotuned one,
// else automatic.
unsigned dense_for(const csp_ctx *ctx, int d, long long N, long long c)
{
    long long v = ctx->dense_override;
    if (v < 0) {
        const csp_ctx::Tuned *e = tuned_for(ctx, d, N);
        v = e ? e->dense : -1;
    }
    if (v < 0) return dense_default(c);
    return v >= (long long)DENSE_NEVER ? DENSE_NEVER : (unsigned)v;
}

// Wall-clock ticks a barrier wait of a single solve may take before the run
// is marked broken: 20 s, or what csp_set_wait_limit set.
unsigned long long solve_wait_ticks(const csp_ctx *ctx)
{
    if (ctx->wait_us < 0) return ctx->wall_khz * 1000ull * 20ull;
    return ctx->wall_khz * (unsigned long long)ctx->wait_us / 1000ull;
}

void fill_job(RJ &p, int d, long long n, long long N, const LdsPlan &plan, const uint8_t *f1, const uint8_t *f2, const uint8_t *A, const uint8_t *B, uint32_t M)
{
    memset(&p, 0, sizeof(p));
    p.n = n;
    p.N = N;
    p.c = plan.c;
    p.d = d;
    p.K = plan.K;
    p.lt = plan.lt;
    p.llist = plan.llist;
    p.dense_thr = dense_default(plan.c);
    p.tile = plan.tile;
    p.ty = plan.ty;
    p.tz = plan.tz;
    p.nty = (unsigned)plan.nty;
    p.g = (unsigned)plan.G;
    p.f1 = f1;
    p.f2 = f2;
    p.A = A;
    p.B = B;
    p.M = M;
}

// Gang layout of one problem run by persistent workers with `budget` bytes
// of dynamic LDS each: 16-bit LDS labels when M allows (larger ranges, fewer
// workgroups), g ranges of c vertices, neighbours within K ranges, a wheel of
// `pool` flows and candidate buffers of `ccap` entries per (sender, offset).
struct GangPlan {
    long long N = 0, c = 0;
    int g = 1, K = 0, lt = 4, llist = 0;
    size_t lds = 0;
    unsigned long long pool = 0, ccap = 1;
};

int plan_gang(csp_ctx *ctx, size_t budget, int gmax, int d, long long n, long long N, uint32_t M, GangPlan &pl,
              int g_want = 0)
{
    pl.N = N;
    pl.lt = M <= 0xFFFFu ? 2 : 4;
    long long cmax = 0;
    {
        long long lo = 1, hi = 1ll << 22;
        while (lo < hi) {
            const long long mid = (lo + hi + 1) / 2;
            if (lds_bytes_for(mid, 0, pl.lt) <= budget) lo = mid;
            else hi = mid - 1;
        }
        cmax = lo;
    }
    // the fewest workgroups whose ranges fit LDS, or more when asked (shorter
    // cycles for a lone problem) while neighbours stay within KMAX ranges
    const long long gcap = std::min(gmax, GMAX);
    const long long gmin = std::min<long long>((N + cmax - 1) / cmax, gcap);
    long long smax = 1;
    for (int k = 1; k < d; ++k) smax *= n;
    long long g = std::max<long long>(gmin, std::min<long long>(g_want, gcap));
    while (g > gmin) {
        const long long c = (N + g - 1) / g;
        if ((g - 1) * c < N && (smax + c - 1) / c <= KMAX) break;
        --g;
    }
    pl.g = (int)g;
    pl.c = (N + pl.g - 1) / pl.g;
    if (pl.c > cmax) return fail(ctx, CSP_EINVAL, "problem too large for one launch");
    pl.K = pl.g == 1 ? 0 : (int)((smax + pl.c - 1) / pl.c);
    if (pl.K > KMAX) return fail(ctx, CSP_EINVAL, "problem ranges too thin");
    // 32-bit labels (one atomicMax per raise) when the range fits with them;
    // 16-bit labels take a compare-and-swap loop
    if (pl.lt == 2 && lds_bytes_for(pl.c, pl.K, 4) <= budget) pl.lt = 4;
    pl.lds = lds_bytes_for(pl.c, pl.K, pl.lt);
    pl.llist = (int)lds_list_cap(pl.c, pl.lds, budget);
    pl.lds += lds_list_bytes(pl.llist);
    pl.pool = ctx->pool_hint ? ctx->pool_hint * 256ull * pl.g : std::max<unsigned long long>(1ull << 15, 6ull * d * N);
    const unsigned long long cmaxc = 2ull * d * (unsigned long long)pl.c;
    pl.ccap = pl.g == 1 ? 1
                        : std::min<unsigned long long>(cmaxc, ctx->pool_hint ? 64ull
                                                                             : std::max<unsigned long long>(
                                                                                   2048, pl.c / 2));
    return CSP_OK;
}

void launch_pack(int d, long long n, long long N, const uint8_t *f1, const uint8_t *f2, void *rec, Ctl *ctl,
                 int num_cu, hipStream_t s)
{
    const int nb = (int)std::max(1ll, std::min((N + 255) / 256, (long long)num_cu * 16));
    switch (d) {
    case 1: hipLaunchKernelGGL(k_pack<1>, dim3(nb), dim3(256), 0, s, n, N, f1, f2, (Rec<1>::T *)rec, ctl); break;
    case 2: hipLaunchKernelGGL(k_pack<2>, dim3(nb), dim3(256), 0, s, n, N, f1, f2, (Rec<2>::T *)rec, ctl); break;
    case 3: hipLaunchKernelGGL(k_pack<3>, dim3(nb), dim3(256), 0, s, n, N, f1, f2, (Rec<3>::T *)rec, ctl); break;
    default: hipLaunchKernelGGL(k_pack<4>, dim3(nb), dim3(256), 0, s, n, N, f1, f2, (Rec<4>::T *)rec, ctl); break;
    }
}

}  // namespace

extern "C" {

int csp_create(int device, csp_ctx **out)
{
    if (!out) return CSP_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CSP_EDEVICE;
    csp_ctx *ctx = new csp_ctx();
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess) { delete ctx; return CSP_EDEVICE; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) { delete ctx; return CSP_EDEVICE; }
    ctx->num_cu = prop.multiProcessorCount;
    ctx->lds_limit = std::max<size_t>(prop.sharedMemPerBlock, prop.sharedMemPerBlockOptin);
    if (device < SCRATCH_DEVICES) {
        // once per device, with the device current: its copy of the static
        // scratch (left null if the runtime cannot give it; only
        // csp_solve_dev_noalloc needs it and then reports the error)
        std::lock_guard<std::mutex> lock(scratch_mu);
        if (!scratch_dev[device]) {
            void *ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess) scratch_dev[device] = (uint8_t *)ptr;
            else (void)hipGetLastError();
        }
        ctx->scratch = scratch_dev[device];
    }
    {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
            ctx->wall_khz = (unsigned long long)khz;
    }
    for (int d = 1; d <= 4; ++d) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, solve_kernel(d), BLOCK, 0) != hipSuccess || nb < 1)
            nb = 1;
        ctx->max_blocks[d] = std::min(GMAX, std::min(nb, 1) * ctx->num_cu);
    }
    if (hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess ||
        hipMalloc((void **)&ctx->ctl, sizeof(Ctl)) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_ctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_byte, 64, hipHostMallocDefault) != hipSuccess) {
        csp_destroy(ctx);
        return CSP_ENOMEM;
    }
    *out = ctx;
    return CSP_OK;
}

void csp_destroy(csp_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    for (void *p : {(void *)ctx->lab, (void *)ctx->rec, (void *)ctx->queue, (void *)ctx->pool,
                    (void *)ctx->ctl, (void *)ctx->in_buf, (void *)ctx->pub, (void *)ctx->cand,
                    (void *)ctx->arena, (void *)ctx->gstamp, (void *)ctx->glists, (void *)ctx->gpool,
                    (void *)ctx->wptr, (void *)ctx->cptr, (void *)ctx->cur, (void *)ctx->winner,
                    (void *)ctx->logbuf, (void *)ctx->walk})
        if (p) (void)hipFree(p);
    if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
    for (void *p : {(void *)ctx->h_ctl, (void *)ctx->h_byte})
        if (p) (void)hipHostFree(p);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    delete ctx;
}

const char *csp_last_error(const csp_ctx *ctx)
{
    return ctx ? ctx->err : "no context";
}

}  // extern "C"

namespace {

int solve_impl(csp_ctx *ctx, int d, int64_t n, const uint8_t *f1, const uint8_t *f2, const uint8_t *A,
               const uint8_t *B, uint32_t M, uint32_t *labels, csp_result *out, csp_counters *cnt,
               int64_t max_cycles, void *stream, bool log)
{
    if (!ctx || !out || !f1 || !f2 || !A || !B) return fail(ctx, CSP_EINVAL, "null argument");
    long long N = 0;
    int rc = check_shape(ctx, d, n, M, N);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");

    rc = grow(ctx, &ctx->lab, ctx->lab_cap, (size_t)N, "labels");
    if (rc) return rc;
    rc = grow(ctx, &ctx->rec, ctx->rec_cap, (size_t)N * rec_bytes(d), "edge records");
    if (rc) return rc;

    long long stride[4] = {1, 1, 1, 1};
    for (int k = 1; k < d; ++k) stride[k] = stride[k - 1] * n;
    long long off[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int dir = 0; dir < 2 * d; ++dir) {
        const bool lower = dir < d;
        const int k = lower ? d - 1 - dir : dir - d;
        off[dir] = lower ? -stride[k] : stride[k];
    }

    // Range-owned kernel when a range fits in LDS, else the global-label kernel.
    int G = blocks_for(ctx, d, N);
    const int path = path_for(ctx, d, N);
    LdsPlan plan;
    if (path != 2) {
        plan = plan_lds(ctx, d, n, N, M, G, path);
        if (plan.ok) {
            const void *kf = lds_kernel(d, plan.tile, log);
            if (hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)plan.lds) != hipSuccess)
                plan.ok = false;
            int nb = 0;
            if (plan.ok && (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kf, BLOCK, plan.lds) != hipSuccess ||
                            nb * ctx->num_cu < plan.G))
                plan.ok = false;
        }
        if (!plan.ok && (ctx->path_override == 1 || ctx->path_override == 3))
            return fail(ctx, CSP_EINVAL, "range does not fit in LDS");
    }
    const bool use_lds = plan.ok;
    if (use_lds) G = plan.G;
    if (ctx->trace && !use_lds) return fail(ctx, CSP_EINVAL, "the cycle trace needs the range-owned kernel");
    if (log && !use_lds) return fail(ctx, CSP_EINVAL, "the improvement log needs the range-owned kernel");
    // log records per range: at least two per vertex, else what a solve needed before
    unsigned long long log_cap = log ? std::max<unsigned long long>(2ull * plan.c, ctx->log_seen) : 0ull;
    // record indices are 32-bit across all G ranges: a size remembered from a
    // solve with fewer ranges may not fit this one
    if (log) log_cap = std::min<unsigned long long>(log_cap, ((1ull << 32) - 1) / (unsigned long long)G);
    ctx->last_path = use_lds ? 1 : 2;

    // wheel capacity: start from the largest a solve has needed, at least
    // 16 flows per directed-edge endpoint; doubled on overflow up to the
    // bound at which no bucket can overflow
    const unsigned long long NO = use_lds ? (unsigned long long)(plan.tile ? 2 * d : 2 * plan.K + 1) : 1ull;
    if (use_lds) {
        rc = grow(ctx, &ctx->rec, ctx->rec_cap, (size_t)(plan.c * G) * rec_bytes(d), "edge records");
        if (rc) return rc;
    }
    unsigned long long pool = ctx->pool_hint ? ctx->pool_hint * 256ull * G
                                             : std::max<unsigned long long>(
                                                   std::max<unsigned long long>(1ull << 20, 16ull * d * N),
                                                   ctx->pool_flows_seen);
    const unsigned long long pool_max = 2ull * d * N * 256ull * G + (1ull << 20);
    unsigned long long qs = std::max<unsigned long long>((N + G - 1) / G, 4096ull);
    // candidates per (sender, offset) and cycle: at most 2d per vertex of the range
    const unsigned long long cand_max = use_lds ? 2ull * d * (unsigned long long)plan.c : 0ull;
    unsigned long long ccap = use_lds ? std::min<unsigned long long>(
                                            cand_max, std::max<unsigned long long>(
                                                          {4096ull, (unsigned long long)plan.c / 2, ctx->cand_seen}))
                                      : 0ull;
    if (use_lds && ctx->pool_hint) ccap = std::min<unsigned long long>(cand_max, 64ull);
    // a pencil face of n t vertices ships at most one candidate per vertex and cycle
    if (use_lds && plan.tile && !ctx->pool_hint) ccap = (unsigned long long)n * plan.ty;

    for (;;) {
        rc = grow(ctx, &ctx->pool, ctx->pool_cap, (size_t)pool, "transit pool");
        if (rc) return rc;
        hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(BLOCK), 0, s, ctx->ctl);
        if (use_lds) {
            rc = grow(ctx, &ctx->queue, ctx->queue_cap, (size_t)(plan.c * G), "frontier");
            if (rc) return rc;
            rc = grow(ctx, &ctx->pub, ctx->pub_cap, (size_t)2 * G * NOMAX, "candidate fills");
            if (rc) return rc;
            rc = grow(ctx, &ctx->cand, ctx->cand_cap, (size_t)(2ull * G * NO * ccap), "candidates");
            if (rc) return rc;
            if (log) {
                rc = grow(ctx, &ctx->wptr, ctx->wptr_cap, (size_t)pool, "log: wheel senders");
                if (!rc) rc = grow(ctx, &ctx->cptr, ctx->cptr_cap, (size_t)(2ull * G * NO * ccap), "log: candidate senders");
                if (!rc) rc = grow(ctx, &ctx->cur, ctx->cur_cap, (size_t)(plan.c * G), "log: latest records");
                if (!rc) rc = grow(ctx, &ctx->winner, ctx->winner_cap, (size_t)(plan.c * G), "log: best deliveries");
                if (!rc) rc = grow(ctx, &ctx->logbuf, ctx->logbuf_cap, (size_t)(log_cap * G), "log: records");
                if (rc) return rc;
            }
            RJ p;
            fill_job(p, d, n, N, plan, f1, f2, A, B, M);
            p.dense_thr = dense_for(ctx, d, N, plan.c);
            p.rec = ctx->rec;
            p.lists = ctx->queue;
            p.pool = ctx->pool;
            p.pool_flows = pool;
            p.cand = ctx->cand;
            p.cand_cap = (unsigned)ccap;
            p.pubc = ctx->pub;
            p.bar = &ctx->ctl->rbar;
            p.out = &ctx->ctl->rout;
            p.labels_out = labels;
            p.max_cycles = max_cycles;
            p.wait_limit = solve_wait_ticks(ctx);
            p.prof = ctx->prof;
            p.trace = ctx->trace;
            p.trace_cap = ctx->trace_cap;
            if (log) {
                p.wptr = ctx->wptr;
                p.cptr = ctx->cptr;
                p.cur = ctx->cur;
                p.winner = ctx->winner;
                p.log = ctx->logbuf;
                p.log_cap = log_cap;
            }
            void *args[] = {&p};
            HIP_TRY(hipEventRecord(ctx->ev0, s), "event");
            HIP_TRY(hipLaunchCooperativeKernel(lds_kernel(d, plan.tile, log), dim3(G), dim3(BLOCK), args,
                                               (unsigned)plan.lds, s),
                    "solve launch");
            HIP_TRY(hipEventRecord(ctx->ev1, s), "event");
        } else {
            launch_pack(d, n, N, f1, f2, ctx->rec, ctx->ctl, ctx->num_cu, s);
            HIP_TRY(hipGetLastError(), "pack launch");
            rc = grow(ctx, &ctx->queue, ctx->queue_cap, (size_t)(qs * G), "frontier");
            if (rc) return rc;
            Params p;
            memset(&p, 0, sizeof(p));
            p.N = N;
            for (int dir = 0; dir < 8; ++dir) p.off[dir] = off[dir];
            p.rec = ctx->rec;
            p.A = A;
            p.B = B;
            p.M = M;
            p.qs = (unsigned)qs;
            p.pool_flows = pool;
            p.lab = ctx->lab;
            p.queue = ctx->queue;
            p.pool = ctx->pool;
            p.ctl = ctx->ctl;
            p.labels_out = labels;
            p.max_cycles = max_cycles;
            p.wait_limit = solve_wait_ticks(ctx);
            p.prof = ctx->prof;
            void *args[] = {&p};
            HIP_TRY(hipEventRecord(ctx->ev0, s), "event");
            HIP_TRY(hipLaunchCooperativeKernel(solve_kernel(d), dim3(G), dim3(BLOCK), args, 0, s), "solve launch");
            HIP_TRY(hipEventRecord(ctx->ev1, s), "event");
        }
        {
            // the results part of the control block: scalars, counters, result, Out
            const size_t lo = offsetof(Ctl, xkey), hi = offsetof(Ctl, rbar);
            HIP_TRY(hipMemcpyAsync(reinterpret_cast<uint8_t *>(ctx->h_ctl) + lo,
                                   reinterpret_cast<const uint8_t *>(ctx->ctl) + lo, hi - lo, hipMemcpyDeviceToHost, s),
                    "ctl copy");
        }
        HIP_TRY(hipStreamSynchronize(s), "solve");
        const Ctl &c = *ctx->h_ctl;
        const int status = use_lds ? c.rout.status : c.status;
        const long long *res = use_lds ? c.rout.res : c.res;
        const unsigned long long *ctr = use_lds ? c.rout.ctr : c.ctr;
        const unsigned long long *prof = use_lds ? c.rout.prof : c.prof;
        if (status == ST_INVAL || (!use_lds && c.bad)) {
            return fail(ctx, CSP_EINVAL, "an edge has f1 or f2 equal to 0, or A and B overlap");
        }
        if (status == ST_OVERFLOW && log && use_lds && c.rout.log_over) {
            // only the log ran out
            log_cap *= 2;
            if (log_cap * (unsigned long long)G >= (1ull << 32))
                return fail(ctx, CSP_EOVERFLOW, "improvement log beyond 2^32 records");
            continue;
        }
        if (status == ST_OVERFLOW) {
            if (pool >= pool_max && ccap >= cand_max)
                return fail(ctx, CSP_EOVERFLOW, "transit pool overflow at the edge bound");
            pool = std::min(pool * 2, pool_max);
            qs = std::min<unsigned long long>(qs * 2, (unsigned long long)N);
            ccap = std::min(ccap * 2, cand_max);
            continue;
        }
        if (status == ST_CANCELED) return fail(ctx, CSP_ECANCELED, "cycle cap reached");
        if (status == ST_BROKEN) return fail(ctx, CSP_EDEVICE, "grid barrier timed out or inconsistent result");
        if (status != ST_DONE) return fail(ctx, CSP_EDEVICE, "solve did not finish");
        if (!ctx->pool_hint) {
            ctx->pool_flows_seen = std::max(ctx->pool_flows_seen, pool);
            ctx->cand_seen = std::max(ctx->cand_seen, ccap);
        }
        HIP_TRY(hipEventElapsedTime(&ctx->last_ms, ctx->ev0, ctx->ev1), "event time");
        for (int i = 0; i < 8; ++i) {
            ctx->last_prof[i] = prof[i];
            ctx->last_psum[i] = use_lds && ctx->prof == 2 ? c.rout.psum[i] : 0;
            ctx->last_pmax[i] = use_lds && ctx->prof == 2 ? c.rout.pmax[i] : 0;
        }
        ctx->last_spread_ranges = use_lds ? G : 0;
        ctx->last_trace_rows = use_lds ? c.rout.trace_rows : 0;
        ctx->last_xrec = log ? c.rout.xrec : -1;
        if (log && !ctx->pool_hint) ctx->log_seen = std::max(ctx->log_seen, log_cap);
        out->T = res[0];
        out->X = res[1];
        out->x = res[2];
        out->Y = res[3];
        out->F2 = res[4];
        if (cnt) {
            cnt->C = (int64_t)ctr[0];
            cnt->U = (int64_t)ctr[1];
            cnt->D = (int64_t)ctr[2];
            cnt->E = (int64_t)ctr[3];
            cnt->R = (int64_t)ctr[4];
            cnt->P = (int64_t)ctr[5];
            cnt->I = (int64_t)ctr[6];
        }
        return CSP_OK;
    }
}

// csp_solve_dev without allocation: the range-owned kernel (the only one the
// scratch serves) with its edge records, frontier lists, candidate fills,
// candidates and wheel carved from this device's copy of the static scratch;
// the barrier and result block stay in the context (allocated when it was
// created).  Nothing in the scratch has to start at zero: every range packs
// its records, clears its own fills before the first barrier and writes
// wheel and candidate entries before anything reads them.  Calls on one GPU
// share the array, so calls that overlap on one GPU race.
int solve_noalloc(csp_ctx *ctx, int d, int64_t n, const uint8_t *f1, const uint8_t *f2, const uint8_t *A,
                  const uint8_t *B, uint32_t M, uint32_t *labels, csp_result *out, csp_counters *cnt,
                  int64_t max_cycles, void *stream)
{
    if (!ctx || !out || !f1 || !f2 || !A || !B) return fail(ctx, CSP_EINVAL, "null argument");
    if (ctx->trace) return fail(ctx, CSP_EINVAL, "the allocation-free solve keeps no cycle trace");
    if (!ctx->scratch) return fail(ctx, CSP_EDEVICE, "no static scratch on this device");
    long long N = 0;
    int rc = check_shape(ctx, d, n, M, N);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");

    const int path = path_for(ctx, d, N);
    if (path == 2) return fail(ctx, CSP_EINVAL, "the allocation-free solve runs only the range-owned kernel");
    LdsPlan plan = plan_lds(ctx, d, n, N, M, blocks_for(ctx, d, N), path);
    const void *kf = plan.ok ? lds_kernel(d, plan.tile, false) : nullptr;
    if (plan.ok && hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)plan.lds) != hipSuccess)
        plan.ok = false;
    int nb = 0;
    if (plan.ok && (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kf, BLOCK, plan.lds) != hipSuccess ||
                    nb * ctx->num_cu < plan.G))
        plan.ok = false;
    if (!plan.ok) return fail(ctx, CSP_EINVAL, "a range of this lattice does not fit in LDS");
    const int G = plan.G;
    ctx->last_path = 1;

    // layout in the scratch: records | lists | fills | candidates | wheel
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const unsigned long long NO = plan.tile ? 2ull * d : 2ull * plan.K + 1;
    const unsigned long long cand_max = 2ull * d * (unsigned long long)plan.c;
    const unsigned long long ccap =
        plan.tile ? (unsigned long long)n * plan.ty
                  : std::min<unsigned long long>(cand_max, std::max<unsigned long long>(4096ull, plan.c / 2));
    const size_t off_lists = up((size_t)(plan.c * G) * rec_bytes(d));
    const size_t off_pub = off_lists + up((size_t)(plan.c * G) * 4);
    const size_t off_cand = off_pub + up((size_t)2 * G * NOMAX * 8);
    const size_t off_pool = off_cand + up((size_t)(2ull * G * NO * ccap * 8));
    // the wheel gets the rest; at least 16 flows per bucket of every range
    if (off_pool + (size_t)G * MAXW * 16 * 8 > (size_t)CSP_SCRATCH_BYTES)
        return fail(ctx, CSP_EINVAL, "lattice too large for the allocation-free solve (CSP_SCRATCH_BYTES)");
    const unsigned long long pool = ((size_t)CSP_SCRATCH_BYTES - off_pool) / 8;

    hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(BLOCK), 0, s, ctx->ctl);
    RJ p;
    fill_job(p, d, n, N, plan, f1, f2, A, B, M);
    p.dense_thr = dense_for(ctx, d, N, plan.c);
    p.rec = ctx->scratch;
    p.lists = reinterpret_cast<unsigned *>(ctx->scratch + off_lists);
    p.pubc = reinterpret_cast<unsigned long long *>(ctx->scratch + off_pub);
    p.cand = reinterpret_cast<uint2 *>(ctx->scratch + off_cand);
    p.cand_cap = (unsigned)ccap;
    p.pool = reinterpret_cast<uint2 *>(ctx->scratch + off_pool);
    p.pool_flows = pool;
    p.bar = &ctx->ctl->rbar;
    p.out = &ctx->ctl->rout;
    p.labels_out = labels;
    p.max_cycles = max_cycles;
    p.wait_limit = solve_wait_ticks(ctx);
    p.prof = ctx->prof;
    void *args[] = {&p};
    HIP_TRY(hipEventRecord(ctx->ev0, s), "event");
    HIP_TRY(hipLaunchCooperativeKernel(kf, dim3(G), dim3(BLOCK), args, (unsigned)plan.lds, s), "solve launch");
    HIP_TRY(hipEventRecord(ctx->ev1, s), "event");
    {
        const size_t lo = offsetof(Ctl, xkey), hi = offsetof(Ctl, rbar);
        HIP_TRY(hipMemcpyAsync(reinterpret_cast<uint8_t *>(ctx->h_ctl) + lo,
                               reinterpret_cast<const uint8_t *>(ctx->ctl) + lo, hi - lo, hipMemcpyDeviceToHost, s),
                "ctl copy");
    }
    HIP_TRY(hipStreamSynchronize(s), "solve");
    const Out &o = ctx->h_ctl->rout;
    if (o.status == ST_INVAL) return fail(ctx, CSP_EINVAL, "an edge has f1 or f2 equal to 0, or A and B overlap");
    if (o.status == ST_OVERFLOW)
        return fail(ctx, CSP_EOVERFLOW, "flows in transit overflow the allocation-free solve's wheel");
    if (o.status == ST_CANCELED) return fail(ctx, CSP_ECANCELED, "cycle cap reached");
    if (o.status == ST_BROKEN) return fail(ctx, CSP_EDEVICE, "grid barrier timed out or inconsistent result");
    if (o.status != ST_DONE) return fail(ctx, CSP_EDEVICE, "solve did not finish");
    HIP_TRY(hipEventElapsedTime(&ctx->last_ms, ctx->ev0, ctx->ev1), "event time");
    for (int i = 0; i < 8; ++i) {
        ctx->last_prof[i] = o.prof[i];
        ctx->last_psum[i] = ctx->prof == 2 ? o.psum[i] : 0;
        ctx->last_pmax[i] = ctx->prof == 2 ? o.pmax[i] : 0;
    }
    ctx->last_spread_ranges = G;
    ctx->last_trace_rows = 0;
    ctx->last_xrec = -1;
    out->T = o.res[0];
    out->X = o.res[1];
    out->x = o.res[2];
    out->Y = o.res[3];
    out->F2 = o.res[4];
    if (cnt) {
        cnt->C = (int64_t)o.ctr[0];
        cnt->U = (int64_t)o.ctr[1];
        cnt->D = (int64_t)o.ctr[2];
        cnt->E = (int64_t)o.ctr[3];
        cnt->R = (int64_t)o.ctr[4];
        cnt->P = (int64_t)o.ctr[5];
        cnt->I = (int64_t)o.ctr[6];
    }
    return CSP_OK;
}

}  // namespace

extern "C" {

int csp_solve_dev(csp_ctx *ctx, int d, int64_t n, const uint8_t *f1, const uint8_t *f2,
                  const uint8_t *A, const uint8_t *B, uint32_t M, uint32_t *labels,
                  csp_result *out, csp_counters *cnt, int64_t max_cycles, void *stream)
{
    return solve_impl(ctx, d, n, f1, f2, A, B, M, labels, out, cnt, max_cycles, stream, false);
}

int csp_solve_dev_noalloc(csp_ctx *ctx, int d, int64_t n, const uint8_t *f1, const uint8_t *f2,
                          const uint8_t *A, const uint8_t *B, uint32_t M, uint32_t *labels,
                          csp_result *out, csp_counters *cnt, int64_t max_cycles, void *stream)
{
    return solve_noalloc(ctx, d, n, f1, f2, A, B, M, labels, out, cnt, max_cycles, stream);
}

int csp_solve_graph_dev(csp_ctx *ctx, int64_t nv, const int64_t *off, const int32_t *nbr, const uint8_t *f1,
                        const uint8_t *f2, const int64_t *eid, const uint8_t *A, const uint8_t *B, uint32_t M,
                        uint32_t *labels, csp_result *out, csp_counters *cnt, int64_t max_cycles, void *stream)
{
    if (!ctx || !out || !off || !nbr || !f1 || !f2 || !eid || !A || !B) return fail(ctx, CSP_EINVAL, "null argument");
    if (nv < 1 || nv >= (1ll << 31)) return fail(ctx, CSP_EINVAL, "vertex count out of range");
    if (M < 1 || M > CSP_MAX_M) return fail(ctx, CSP_EINVAL, "M out of range");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    long long m = 0;
    HIP_TRY(hipMemcpyAsync(&m, off + nv, sizeof(m), hipMemcpyDeviceToHost, s), "edge count");
    HIP_TRY(hipStreamSynchronize(s), "edge count");
    if (m < 0 || m >= (1ll << 31)) return fail(ctx, CSP_EINVAL, "adjacency entries out of range");
    const void *kf = (const void *)k_graph;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kf, BLOCK, 0) != hipSuccess || nb < 1)
        return fail(ctx, CSP_EDEVICE, "graph kernel occupancy");
    const long long gmax = std::min<long long>(GMAX, (long long)nb * ctx->num_cu);
    long long G = ctx->blocks_override > 0 ? ctx->blocks_override : (nv + 8191) / 8192;
    if (nv <= 32768 && ctx->blocks_override <= 0) G = 1;
    G = std::max(1ll, std::min(G, gmax));
    int rc = grow(ctx, &ctx->lab, ctx->lab_cap, (size_t)nv, "labels");
    if (!rc) rc = grow(ctx, &ctx->gstamp, ctx->gstamp_cap, (size_t)nv, "graph stamps");
    if (rc) return rc;
    // each workgroup lists only its own chunk of vertices
    unsigned long long qcap = (unsigned long long)((nv + G - 1) / G);
    unsigned long long pool = ctx->pool_hint ? ctx->pool_hint * 256ull * G
                                             : std::max<unsigned long long>({1ull << 20, 8ull * (unsigned long long)m,
                                                                             ctx->gpool_seen});
    const unsigned long long pool_max = 256ull * G * ((unsigned long long)m + 1) + (1ull << 20);
    for (;;) {
        rc = grow(ctx, &ctx->glists, ctx->glists_cap, (size_t)(G * qcap), "graph frontier lists");
        if (!rc) rc = grow(ctx, &ctx->gpool, ctx->gpool_cap, (size_t)pool, "graph transit pool");
        if (rc) return rc;
        hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(BLOCK), 0, s, ctx->ctl);
        GJ p;
        memset(&p, 0, sizeof(p));
        p.nv = nv;
        p.m = m;
        p.off = reinterpret_cast<const long long *>(off);
        p.nbr = nbr;
        p.f1 = f1;
        p.f2 = f2;
        p.eid = reinterpret_cast<const long long *>(eid);
        p.A = A;
        p.B = B;
        p.M = M;
        p.lab = ctx->lab;
        p.stamp = ctx->gstamp;
        p.lists = ctx->glists;
        p.qcap = qcap;
        p.pool = ctx->gpool;
        p.pool_flows = pool;
        p.bar = &ctx->ctl->rbar;
        p.out = &ctx->ctl->rout;
        p.xsel = &ctx->ctl->xkey;
        p.labels_out = labels;
        p.max_cycles = max_cycles;
        p.wait_limit = solve_wait_ticks(ctx);
        p.prof = ctx->prof;
        void *args[] = {&p};
        HIP_TRY(hipEventRecord(ctx->ev0, s), "event");
        HIP_TRY(hipLaunchCooperativeKernel(kf, dim3((unsigned)G), dim3(BLOCK), args, 0, s), "graph launch");
        HIP_TRY(hipEventRecord(ctx->ev1, s), "event");
        {
            const size_t lo = offsetof(Ctl, xkey), hi = offsetof(Ctl, rbar);
            HIP_TRY(hipMemcpyAsync(reinterpret_cast<uint8_t *>(ctx->h_ctl) + lo,
                                   reinterpret_cast<const uint8_t *>(ctx->ctl) + lo, hi - lo, hipMemcpyDeviceToHost, s),
                    "ctl copy");
        }
        HIP_TRY(hipStreamSynchronize(s), "graph solve");
        const Out &o = ctx->h_ctl->rout;
        if (o.status == ST_INVAL)
            return fail(ctx, CSP_EINVAL,
                        "an edge has f1 or f2 equal to 0, A and B overlap, or off / nbr are out of range");
        if (o.status == ST_OVERFLOW) {
            if (pool >= pool_max)
                return fail(ctx, CSP_EOVERFLOW, "graph transit pool overflow at the edge bound");
            pool = std::min(pool * 2, pool_max);
            continue;
        }
        if (o.status == ST_CANCELED) return fail(ctx, CSP_ECANCELED, "cycle cap reached");
        if (o.status == ST_BROKEN) return fail(ctx, CSP_EDEVICE, "grid barrier timed out or inconsistent result");
        if (o.status != ST_DONE) return fail(ctx, CSP_EDEVICE, "graph solve did not finish");
        if (!ctx->pool_hint) ctx->gpool_seen = std::max(ctx->gpool_seen, pool);
        HIP_TRY(hipEventElapsedTime(&ctx->last_ms, ctx->ev0, ctx->ev1), "event time");
        for (int i = 0; i < 8; ++i) ctx->last_prof[i] = o.prof[i];
        ctx->last_path = 2;
        out->T = o.res[0];
        out->X = o.res[1];
        out->x = o.res[2];
        out->Y = o.res[3];
        out->F2 = o.res[4];
        if (cnt) {
            cnt->C = (int64_t)o.ctr[0];
            cnt->U = (int64_t)o.ctr[1];
            cnt->D = (int64_t)o.ctr[2];
            cnt->E = (int64_t)o.ctr[3];
            cnt->R = (int64_t)o.ctr[4];
            cnt->P = (int64_t)o.ctr[5];
            cnt->I = (int64_t)o.ctr[6];
        }
        return CSP_OK;
    }
}

int csp_reconstruct_log_dev(csp_ctx *ctx, int d, int64_t n, const uint8_t *f1, const uint8_t *f2,
                            const uint8_t *A, const uint8_t *B, uint32_t M, int64_t *path, int64_t cap,
                            int64_t *len, csp_result *out, csp_counters *cnt, void *stream)
{
    if (!ctx || !path || !len || !out) return fail(ctx, CSP_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    *len = 0;
    int rc = solve_impl(ctx, d, n, f1, f2, A, B, M, nullptr, out, cnt, 0, stream, true);
    if (rc) return rc;
    if (out->T < 0) return CSP_OK;
    long long N = 1;
    for (int k = 0; k < d; ++k) N *= n;
    // a path has at most min(M, N) vertices
    const long long wcap = std::min<long long>((long long)M, N);
    rc = grow(ctx, &ctx->walk, ctx->walk_cap, (size_t)wcap + 1, "path walk");
    if (rc) return rc;
    if (ctx->last_xrec < 0 || (size_t)ctx->last_xrec >= ctx->logbuf_cap)
        return fail(ctx, CSP_EDEVICE, "no improvement record for X");
    hipLaunchKernelGGL(k_walk, dim3(1), dim3(64), 0, s, (const uint4 *)ctx->logbuf,
                       (unsigned long long)ctx->logbuf_cap, ctx->last_xrec, ctx->walk, wcap, ctx->walk + wcap);
    HIP_TRY(hipGetLastError(), "walk launch");
    long long L = 0;
    HIP_TRY(hipMemcpyAsync(&L, ctx->walk + wcap, sizeof(L), hipMemcpyDeviceToHost, s), "walk length");
    HIP_TRY(hipStreamSynchronize(s), "walk");
    if (L < 2) return fail(ctx, CSP_EDEVICE, "improvement log did not lead back to A");
    *len = L;
    if (L > cap) return fail(ctx, CSP_EINVAL, "path buffer too small");
    HIP_TRY(hipMemcpyAsync(path, ctx->walk, (size_t)L * sizeof(long long), hipMemcpyDeviceToHost, s), "walk copy");
    HIP_TRY(hipStreamSynchronize(s), "walk copy");
    std::reverse(path, path + L);
    if (path[L - 1] != out->X || path[L - 2] != out->Y) return fail(ctx, CSP_EDEVICE, "logged path disagrees with x");
    return CSP_OK;
}

int csp_solve(csp_ctx *ctx, int d, int64_t n, const uint8_t *f1, const uint8_t *f2,
              const uint8_t *A, const uint8_t *B, uint32_t M, uint32_t *labels,
              csp_result *out, csp_counters *cnt)
{
    if (!ctx || !out || !f1 || !f2 || !A || !B) return fail(ctx, CSP_EINVAL, "null argument");
    long long N = 0;
    int rc = check_shape(ctx, d, n, M, N);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    // staging: f1 | f2 | A | B | labels, each region 256-byte aligned
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t fbytes = (size_t)d * N;
    const size_t o_f2 = up(fbytes), o_A = o_f2 + up(fbytes), o_B = o_A + up(N), o_L = o_B + up(N);
    const size_t need = o_L + (size_t)N * 4;
    rc = grow(ctx, &ctx->in_buf, ctx->in_cap, need, "input staging");
    if (rc) return rc;
    uint8_t *df1 = ctx->in_buf, *df2 = ctx->in_buf + o_f2, *dA = ctx->in_buf + o_A, *dB = ctx->in_buf + o_B;
    uint32_t *dl = reinterpret_cast<uint32_t *>(ctx->in_buf + o_L);
    HIP_TRY(hipMemcpy(df1, f1, fbytes, hipMemcpyHostToDevice), "upload f1");
    HIP_TRY(hipMemcpy(df2, f2, fbytes, hipMemcpyHostToDevice), "upload f2");
    HIP_TRY(hipMemcpy(dA, A, N, hipMemcpyHostToDevice), "upload A");
    HIP_TRY(hipMemcpy(dB, B, N, hipMemcpyHostToDevice), "upload B");
    rc = csp_solve_dev(ctx, d, n, df1, df2, dA, dB, M, labels ? dl : nullptr, out, cnt, 0, nullptr);
    if (rc) return rc;
    if (labels) HIP_TRY(hipMemcpy(labels, dl, (size_t)N * 4, hipMemcpyDeviceToHost), "download labels");
    return CSP_OK;
}

int csp_reconstruct(csp_ctx *ctx, int d, int64_t n, const uint8_t *f1, const uint8_t *f2, const uint8_t *A,
                    const uint8_t *B, uint32_t M, int64_t *path, int64_t cap, int64_t *len, csp_result *out)
{
    if (!ctx || !out || !f1 || !f2 || !A || !B || !path || !len) return fail(ctx, CSP_EINVAL, "null argument");
    long long N = 0;
    int rc = check_shape(ctx, d, n, M, N);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    // staging: f1 | f2 | A | B | the B' mask of the re-solves, each region 256-byte aligned
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t fbytes = (size_t)d * N;
    const size_t o_f2 = up(fbytes), o_A = o_f2 + up(fbytes), o_B = o_A + up(N), o_S = o_B + up(N);
    const size_t need = o_S + up(N);
    rc = grow(ctx, &ctx->in_buf, ctx->in_cap, need, "input staging");
    if (rc) return rc;
    uint8_t *df1 = ctx->in_buf, *df2 = ctx->in_buf + o_f2, *dA = ctx->in_buf + o_A, *dB = ctx->in_buf + o_B;
    uint8_t *dS = ctx->in_buf + o_S;
    HIP_TRY(hipMemcpy(df1, f1, fbytes, hipMemcpyHostToDevice), "upload f1");
    HIP_TRY(hipMemcpy(df2, f2, fbytes, hipMemcpyHostToDevice), "upload f2");
    HIP_TRY(hipMemcpy(dA, A, N, hipMemcpyHostToDevice), "upload A");
    HIP_TRY(hipMemcpy(dB, B, N, hipMemcpyHostToDevice), "upload B");
    const unsigned long long words = up(N) / 4;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)std::min<unsigned long long>((words + 255) / 256, 1024ull)), dim3(256),
                       0, (hipStream_t) nullptr, reinterpret_cast<unsigned *>(dS), words);
    HIP_TRY(hipGetLastError(), "clear mask");
    return csp_reconstruct_dev(ctx, d, n, df1, df2, dA, dB, M, dS, path, cap, len, out, nullptr);
}

int csp_reconstruct_dev(csp_ctx *ctx, int d, int64_t n, const uint8_t *f1, const uint8_t *f2,
                        const uint8_t *A, const uint8_t *B, uint32_t M, uint8_t *scratch_mask,
                        int64_t *path, int64_t cap, int64_t *len, csp_result *out, void *stream)
{
    if (!ctx || !path || !len || !out || !scratch_mask) return fail(ctx, CSP_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    *len = 0;
    csp_result cur;
    int rc = csp_solve_dev(ctx, d, n, f1, f2, A, B, M, nullptr, &cur, nullptr, 0, stream);
    if (rc) return rc;
    *out = cur;
    if (cur.T < 0) return CSP_OK;
    long long N = 1;
    for (int k = 0; k < d; ++k) N *= n;
    // vertices collected from X backwards, then reversed into path
    int64_t count = 0;
    auto put = [&](int64_t v) {
        if (count < cap) path[count] = v;
        ++count;
    };
    put(cur.X);
    for (;;) {
        put(cur.Y);
        HIP_TRY(hipMemcpyAsync(ctx->h_byte, A + cur.Y, 1, hipMemcpyDeviceToHost, s), "read A");
        HIP_TRY(hipMemcpyAsync(ctx->h_byte + 1, f2 + cur.x, 1, hipMemcpyDeviceToHost, s), "read f2");
        HIP_TRY(hipStreamSynchronize(s), "reconstruct");
        if (ctx->h_byte[0]) break;
        if (count > N) return fail(ctx, CSP_EDEVICE, "reconstruction did not reach A");
        const uint32_t Mn = (uint32_t)(cur.F2 - (int64_t)ctx->h_byte[1] + 1);
        const int64_t Yv = cur.Y;
        hipLaunchKernelGGL(k_set_byte, dim3(1), dim3(1), 0, s, scratch_mask, (long long)Yv, (uint8_t)1);
        csp_result nxt;
        rc = csp_solve_dev(ctx, d, n, f1, f2, A, scratch_mask, Mn, nullptr, &nxt, nullptr, 0, stream);
        hipLaunchKernelGGL(k_set_byte, dim3(1), dim3(1), 0, s, scratch_mask, (long long)Yv, (uint8_t)0);
        if (rc) return rc;
        if (nxt.T < 0 || nxt.X != Yv) return fail(ctx, CSP_EDEVICE, "re-solve did not end at Y");
        cur = nxt;
    }
    HIP_TRY(hipStreamSynchronize(s), "reconstruct");
    *len = count;
    if (count > cap) return fail(ctx, CSP_EINVAL, "path buffer too small");
    std::reverse(path, path + count);
    return CSP_OK;
}

int csp_last_kernel_ms(const csp_ctx *ctx, float *ms)
{
    if (!ctx || !ms) return CSP_EINVAL;
    *ms = ctx->last_ms;
    return ctx->last_ms < 0 ? CSP_EINVAL : CSP_OK;
}

int csp_microbench(csp_ctx *ctx, int kind, int64_t p0, int64_t p1, int64_t p2, double *r, void *stream)
{
    if (!ctx || !r) return fail(ctx, CSP_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    float ms = 0.f;
    auto timed = [&](auto launch) -> int {
        HIP_TRY(hipEventRecord(ctx->ev0, s), "event");
        launch();
        HIP_TRY(hipGetLastError(), "microbenchmark launch");
        HIP_TRY(hipEventRecord(ctx->ev1, s), "event");
        HIP_TRY(hipEventSynchronize(ctx->ev1), "microbenchmark");
        HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1), "event time");
        return CSP_OK;
    };
    const unsigned nb = (unsigned)ctx->num_cu * 8;
    int rc = CSP_OK;
    if (kind == 0) {
        // copy p0 bytes (a multiple of 16), p1 times; bytes read plus written per second
        if (p0 < 16 || p0 % 16 || p1 < 1) return fail(ctx, CSP_EINVAL, "copy size");
        rc = grow(ctx, &ctx->arena, ctx->arena_cap, (size_t)p0 * 2, "microbenchmark buffer");
        if (rc) return rc;
        uint4 *a = reinterpret_cast<uint4 *>(ctx->arena), *b = a + p0 / 16;
        hipLaunchKernelGGL(k_mb_copy, dim3(nb), dim3(256), 0, s, (const uint4 *)b, a, (unsigned long long)(p0 / 16));
        rc = timed([&] {
            for (int64_t k = 0; k < p1; ++k)
                hipLaunchKernelGGL(k_mb_copy, dim3(nb), dim3(256), 0, s, (const uint4 *)a, b, (unsigned long long)(p0 / 16));
        });
        if (rc) return rc;
        r[0] = 2.0 * (double)p0 * (double)p1 / (ms * 1e-3) / 1e9;
    } else if (kind == 1) {
        // p0 atomic maxima over p1 words (a power of two)
        if (p0 < 1 || p1 < 1 || (p1 & (p1 - 1))) return fail(ctx, CSP_EINVAL, "atomic counts");
        rc = grow(ctx, &ctx->arena, ctx->arena_cap, (size_t)p1 * 4, "microbenchmark buffer");
        if (rc) return rc;
        unsigned *a = reinterpret_cast<unsigned *>(ctx->arena);
        hipLaunchKernelGGL(k_mb_atomic, dim3(nb), dim3(256), 0, s, a, (unsigned long long)p1, (unsigned long long)p1);
        rc = timed([&] {
            hipLaunchKernelGGL(k_mb_atomic, dim3(nb), dim3(256), 0, s, a, (unsigned long long)p1, (unsigned long long)p0);
        });
        if (rc) return rc;
        r[0] = (double)p0 / (ms * 1e-3) / 1e9;
    } else if (kind == 2) {
        // one workgroup per CU, p0 scattered 16-byte loads each per round
        // in a slab of 2^p2 records, p1 rounds
        const int lg = p2 == 0 ? 16 : (int)p2;
        if (p0 < 1 || p1 < 1 || lg < 10 || lg > 18) return fail(ctx, CSP_EINVAL, "load counts or slab size");
        const size_t slabs = (size_t)ctx->num_cu * ((size_t)16 << lg);
        const size_t words = slabs + 64;
        rc = grow(ctx, &ctx->arena, ctx->arena_cap, words, "microbenchmark buffer");
        if (rc) return rc;
        HIP_TRY(hipMemsetAsync(ctx->arena, 1, words, s), "fill");
        const uint4 *rec = reinterpret_cast<const uint4 *>(ctx->arena);
        unsigned *sink = reinterpret_cast<unsigned *>(ctx->arena + slabs);
        rc = timed([&] {
            hipLaunchKernelGGL(k_mb_loads, dim3((unsigned)ctx->num_cu), dim3(BLOCK), 0, s, rec, (int)p0, (int)p1, lg,
                               sink);
        });
        if (rc) return rc;
        r[0] = (double)ctx->num_cu * (double)p0 * (double)p1 / (ms * 1e-3) / 1e9;
        r[1] = 1000.0 * ms / (double)p1;
    } else if (kind == 3) {
        // p0 barriers among p1 workgroups: the cycle loop's, then the fully
        // fenced one with p2 KiB of dirty lines per member
        if (p0 < 1 || p1 < 2 || p1 > ctx->num_cu || p2 < 0) return fail(ctx, CSP_EINVAL, "barrier counts");
        const unsigned G = (unsigned)p1;
        const size_t bar = (bar_bytes(G) + 255) & ~(size_t)255;
        const unsigned long long dw = (unsigned long long)p2 * 256;
        rc = grow(ctx, &ctx->arena, ctx->arena_cap, bar + (size_t)G * dw * 4 + 256, "microbenchmark buffer");
        if (rc) return rc;
        BarHdr *bh = reinterpret_cast<BarHdr *>(ctx->arena);
        unsigned *dirty = reinterpret_cast<unsigned *>(ctx->arena + bar);
        const unsigned long long limit = ctx->wall_khz * 1000ull * 10ull;
        for (int kd = 0; kd < 2; ++kd) {
            hipLaunchKernelGGL(k_zero, dim3(64), dim3(256), 0, s, reinterpret_cast<unsigned *>(bh),
                               (unsigned long long)(bar / 4));
            int kdv = kd, it = (int)p0;
            void *args[] = {&bh, &kdv, &it, &dirty, const_cast<unsigned long long *>(&dw),
                            const_cast<unsigned long long *>(&limit)};
            rc = timed([&] {
                (void)hipLaunchCooperativeKernel((const void *)k_mb_barrier, dim3(G), dim3(BLOCK), args, 0, s);
            });
            if (rc) return rc;
            int broken = 0;
            HIP_TRY(hipMemcpy(&broken, &bh->broken, sizeof(int), hipMemcpyDeviceToHost), "barrier check");
            if (broken) return fail(ctx, CSP_EDEVICE, "barrier microbenchmark: wrong combine or timeout");
            r[kd] = 1000.0 * ms / (double)p0;
        }
    } else {
        return fail(ctx, CSP_EINVAL, "unknown microbenchmark");
    }
    return CSP_OK;
}

int csp_set_pool_hint(csp_ctx *ctx, uint64_t flows_per_bucket)
{
    if (!ctx) return CSP_EINVAL;
    ctx->pool_hint = flows_per_bucket;
    return CSP_OK;
}

int csp_set_phase_timing(csp_ctx *ctx, int on)
{
    if (!ctx || on < 0 || on > 2) return CSP_EINVAL;
    ctx->prof = on;
    return CSP_OK;
}

int csp_last_phase_spread(const csp_ctx *ctx, double *mean, double *mx)
{
    if (!ctx || !mean || !mx) return CSP_EINVAL;
    const double G = ctx->last_spread_ranges > 0 ? (double)ctx->last_spread_ranges : 1.0;
    for (int i = 0; i < 6; ++i) {
        mean[i] = (double)ctx->last_psum[i] * 1000.0 / (double)ctx->wall_khz / G;
        mx[i] = (double)ctx->last_pmax[i] * 1000.0 / (double)ctx->wall_khz;
    }
    return CSP_OK;
}

int csp_last_phase_us(const csp_ctx *ctx, double *us)
{
    if (!ctx || !us) return CSP_EINVAL;
    for (int i = 0; i < 6; ++i) us[i] = (double)ctx->last_prof[i] * 1000.0 / (double)ctx->wall_khz;
    return CSP_OK;
}

int csp_solve_batch(csp_ctx *ctx, int count, const csp_problem *probs, csp_result *out, csp_counters *cnt,
                    void *stream)
{
    if (!ctx || count < 0 || (count > 0 && (!probs || !out))) return fail(ctx, CSP_EINVAL, "null argument");
    if (count == 0) return CSP_OK;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    const size_t budget = ctx->lds_limit > 4096 ? ctx->lds_limit - 4096 : 0;

    struct Plan {
        long long N, c;
        int g, K, lt, llist;
        size_t lds;
        unsigned long long pool, ccap;
        size_t off_rec, off_lists, off_pool, off_cand, off_pubc, off_bar, off_out, end;
        long long off[8];
    };
    std::vector<Plan> plan(count);
    std::vector<int> todo(count);
    for (int i = 0; i < count; ++i) {
        const csp_problem &q = probs[i];
        if (!q.f1 || !q.f2 || !q.A || !q.B) return fail(ctx, CSP_EINVAL, "null argument in batch");
        long long N = 0;
        int rc = check_shape(ctx, q.d, q.n, q.M, N);
        if (rc) return rc;
        Plan &pl = plan[i];
        pl.N = N;
        long long stride[4] = {1, 1, 1, 1};
        for (int k = 1; k < q.d; ++k) stride[k] = stride[k - 1] * q.n;
        for (int dir = 0; dir < 8; ++dir) pl.off[dir] = 0;
        for (int dir = 0; dir < 2 * q.d; ++dir) {
            const bool lower = dir < q.d;
            const int k = lower ? q.d - 1 - dir : dir - q.d;
            pl.off[dir] = lower ? -stride[k] : stride[k];
        }
        GangPlan gp;
        const long long gw = ctx->batch_target > 0 ? (N + ctx->batch_target - 1) / ctx->batch_target : 0;
        rc = plan_gang(ctx, budget, ctx->num_cu, q.d, q.n, N, q.M, gp, (int)std::min<long long>(gw, GMAX));
        if (rc) return rc;
        pl.c = gp.c;
        pl.g = gp.g;
        pl.K = gp.K;
        pl.lt = gp.lt;
        pl.llist = gp.llist;
        pl.lds = gp.lds;
        pl.pool = gp.pool;
        pl.ccap = gp.ccap;
        if (!ctx->pool_hint) {
            const auto it = ctx->batch_seen.find(std::make_tuple(q.d, (long long)q.n, q.M, (const void *)q.f1,
                                                                 (const void *)q.f2, (const void *)q.A,
                                                                 (const void *)q.B));
            if (it != ctx->batch_seen.end()) {
                pl.pool = std::max(pl.pool, it->second.first);
                pl.ccap = std::max(pl.ccap, it->second.second);
            }
        }
        todo[i] = i;
    }

    float total_ms = 0.f;
    int rounds = 0;
    while (!todo.empty()) {
        if (++rounds > 24) return fail(ctx, CSP_EOVERFLOW, "batch did not converge");
        // arena layout for the problems of this round
        auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
        size_t at = 0;
        for (int i : todo) {
            Plan &pl = plan[i];
            const int d = probs[i].d;
            const long long NO = 2 * pl.K + 1;
            pl.off_rec = at;
            at = up(at + (size_t)pl.N * rec_bytes(d));
            pl.off_lists = at;
            at = up(at + (size_t)pl.g * pl.c * 4);
            pl.off_pool = at;
            at = up(at + (size_t)pl.pool * 8);
            pl.off_cand = at;
            at = up(at + (size_t)(2ull * pl.g * NO * pl.ccap * 8));
            pl.off_pubc = at;
            at = up(at + (size_t)2 * pl.g * NOMAX * 8);
            pl.off_bar = at;
            at = up(at + bar_bytes((unsigned)pl.g));
            pl.off_out = at;
            at = up(at + sizeof(Out));
            pl.end = at;
        }
        const size_t n_todo = todo.size();
        const size_t jobs_off = up(at), slots_off = up(jobs_off + n_todo * sizeof(RJ));
        size_t nslots = 0;
        for (int i : todo) nslots += (size_t)plan[i].g;
        const size_t next_off = up(slots_off + 2 * nslots * 4);
        const size_t total = next_off + 256;
        int rc = grow(ctx, &ctx->arena, ctx->arena_cap, total, "batch arena");
        if (rc) return rc;
        const size_t stage = std::max(total - jobs_off, n_todo * sizeof(Out));
        if (stage > ctx->h_stage_cap) {
            if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
            ctx->h_stage = nullptr;
            ctx->h_stage_cap = 0;
            if (hipHostMalloc((void **)&ctx->h_stage, stage, hipHostMallocDefault) != hipSuccess)
                return fail(ctx, CSP_ENOMEM, "batch staging");
            ctx->h_stage_cap = stage;
        }
        // per-dimension groups, largest gangs first
        std::vector<int> order(todo.begin(), todo.end());
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            if (probs[a].d != probs[b].d) return probs[a].d < probs[b].d;
            if (plan[a].g != plan[b].g) return plan[a].g > plan[b].g;
            return plan[a].N > plan[b].N;
        });
        uint8_t *h = ctx->h_stage;
        RJ *hjobs = reinterpret_cast<RJ *>(h);
        unsigned *hslot = reinterpret_cast<unsigned *>(h + (slots_off - jobs_off));
        std::vector<size_t> job_of(count);
        for (size_t j = 0; j < n_todo; ++j) {
            const int i = order[j];
            const csp_problem &q = probs[i];
            const Plan &pl = plan[i];
            LdsPlan lp;
            lp.ok = true;
            lp.G = pl.g;
            lp.c = pl.c;
            lp.K = pl.K;
            lp.lt = pl.lt;
            lp.llist = pl.llist;
            lp.lds = pl.lds;
            RJ &p = hjobs[j];
            fill_job(p, q.d, q.n, pl.N, lp, q.f1, q.f2, q.A, q.B, q.M);
            p.rec = ctx->arena + pl.off_rec;
            p.lists = reinterpret_cast<unsigned *>(ctx->arena + pl.off_lists);
            p.pool = reinterpret_cast<uint2 *>(ctx->arena + pl.off_pool);
            p.pool_flows = pl.pool;
            p.cand = reinterpret_cast<uint2 *>(ctx->arena + pl.off_cand);
            p.cand_cap = (unsigned)pl.ccap;
            p.pubc = reinterpret_cast<unsigned long long *>(ctx->arena + pl.off_pubc);
            p.bar = reinterpret_cast<BarHdr *>(ctx->arena + pl.off_bar);
            p.out = reinterpret_cast<Out *>(ctx->arena + pl.off_out);
            p.labels_out = q.labels;
            p.max_cycles = 0;
            p.wait_limit = ctx->wall_khz * 1000ull * 60ull;   // 60 s
            p.prof = 0;
            job_of[i] = j;
        }
        // slot lists (job, range), grouped by dimension
        std::vector<std::pair<int, std::pair<size_t, size_t>>> groups;   // d, [slot begin, end)
        size_t sl = 0;
        for (size_t j = 0; j < n_todo;) {
            const int d = probs[order[j]].d;
            const size_t b0 = sl;
            while (j < n_todo && probs[order[j]].d == d) {
                for (int m = 0; m < plan[order[j]].g; ++m) {
                    hslot[sl] = (unsigned)j;
                    hslot[nslots + sl] = (unsigned)m;
                    ++sl;
                }
                ++j;
            }
            groups.push_back({d, {b0, sl}});
        }
        // zero barrier headers/lines and outputs, then upload the tables
        for (int i : todo) {
            const Plan &pl = plan[i];
            const unsigned long long words = (pl.end - pl.off_bar) / 4;
            const int nb = (int)std::max(1ull, std::min((words + 255) / 256, 1024ull));
            hipLaunchKernelGGL(k_zero, dim3(nb), dim3(256), 0, s,
                               reinterpret_cast<unsigned *>(ctx->arena + pl.off_bar), words);
        }
        hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, reinterpret_cast<unsigned *>(ctx->arena + next_off),
                           64ull);
        HIP_TRY(hipGetLastError(), "batch zero");
        HIP_TRY(hipMemcpyAsync(ctx->arena + jobs_off, h, next_off - jobs_off, hipMemcpyHostToDevice, s),
                "batch tables");
        HIP_TRY(hipEventRecord(ctx->ev0, s), "event");
        unsigned gi = 0;
        for (auto &gr : groups) {
            const int d = gr.first;
            size_t lds = 0;
            for (size_t q = gr.second.first; q < gr.second.second; ++q)
                lds = std::max(lds, plan[order[hslot[q]]].lds);
            const void *kf = batch_kernel(d);
            if (hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
                return fail(ctx, CSP_EDEVICE, "batch LDS attribute");
            int nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kf, BLOCK, lds) != hipSuccess || nb < 1)
                return fail(ctx, CSP_EDEVICE, "batch occupancy");
            BatchArgs a;
            a.jobs = reinterpret_cast<const RJ *>(ctx->arena + jobs_off);
            a.slot_job = reinterpret_cast<const unsigned *>(ctx->arena + slots_off) + gr.second.first;
            a.slot_range = reinterpret_cast<const unsigned *>(ctx->arena + slots_off) + nslots + gr.second.first;
            a.nslots = (unsigned)(gr.second.second - gr.second.first);
            a.next = reinterpret_cast<unsigned *>(ctx->arena + next_off) + gi++;
            const int grid = std::min<int>(nb * ctx->num_cu, (int)a.nslots);
            void *args[] = {&a};
            HIP_TRY(hipLaunchCooperativeKernel(kf, dim3(grid), dim3(BLOCK), args, (unsigned)lds, s), "batch launch");
        }
        HIP_TRY(hipEventRecord(ctx->ev1, s), "event");
        // gather outputs
        Out *hout = reinterpret_cast<Out *>(h);
        for (size_t j = 0; j < n_todo; ++j)
            HIP_TRY(hipMemcpyAsync(&hout[j], ctx->arena + plan[order[j]].off_out, sizeof(Out), hipMemcpyDeviceToHost,
                                   s),
                    "batch results");
        HIP_TRY(hipStreamSynchronize(s), "batch");
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1), "event time");
        total_ms += ms;
        std::vector<int> again;
        for (size_t j = 0; j < n_todo; ++j) {
            const int i = order[j];
            const Out &o = hout[j];
            if (o.status == ST_OVERFLOW) {
                plan[i].pool *= 2;
                plan[i].ccap = std::min<unsigned long long>(plan[i].ccap * 2, 2ull * probs[i].d * plan[i].c);
                again.push_back(i);
                continue;
            }
            if (o.status == ST_INVAL) return fail(ctx, CSP_EINVAL, "batch problem has a zero edge or A and B overlap");
            if (o.status != ST_DONE) return fail(ctx, CSP_EDEVICE, "batch problem did not finish");
            if (rounds > 1 && !ctx->pool_hint) {
                // this problem overflowed at the starting sizes: remember what it needed
                if (ctx->batch_seen.size() >= 65536) ctx->batch_seen.clear();
                const csp_problem &q = probs[i];
                ctx->batch_seen[std::make_tuple(q.d, (long long)q.n, q.M, (const void *)q.f1, (const void *)q.f2,
                                                (const void *)q.A, (const void *)q.B)] = {plan[i].pool, plan[i].ccap};
            }
            out[i].T = o.res[0];
            out[i].X = o.res[1];
            out[i].x = o.res[2];
            out[i].Y = o.res[3];
            out[i].F2 = o.res[4];
            if (cnt) {
                cnt[i].C = (int64_t)o.ctr[0];
                cnt[i].U = (int64_t)o.ctr[1];
                cnt[i].D = (int64_t)o.ctr[2];
                cnt[i].E = (int64_t)o.ctr[3];
                cnt[i].R = (int64_t)o.ctr[4];
                cnt[i].P = (int64_t)o.ctr[5];
                cnt[i].I = (int64_t)o.ctr[6];
            }
        }
        todo.swap(again);
    }
    ctx->last_ms = total_ms;
    return CSP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// serving host side
// ---------------------------------------------------------------------------

namespace {

// First-fit allocator over [0, cap) with coalescing, 256-byte granules.
struct RangeAlloc {
    std::map<size_t, size_t> free_;     // offset -> length
    size_t cap = 0;
    void reset(size_t c)
    {
        free_.clear();
        cap = c;
        if (c) free_[0] = c;
    }
    bool take(size_t len, size_t &off)
    {
        len = (len + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= len) {
                off = it->first;
                const size_t rest = it->second - len;
                free_.erase(it);
                if (rest) free_[off + len] = rest;
                return true;
            }
        }
        return false;
    }
    void give(size_t off, size_t len)
    {
        len = (len + 255) & ~(size_t)255;
        auto it = free_.emplace(off, len).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct SrvReq {
    csp_request q;
    long long N = 0;
    GangPlan plan;
    int attempts = 0;
};

struct SrvAct {
    SrvReq rq;
    unsigned long long seq = 0;
    size_t dev_off = 0, dev_len = 0, path_off = 0, path_len = 0;
    bool live = false;
};

struct SrvDone {
    csp_completion c;
    std::vector<int64_t> path;
};

}  // namespace

struct csp_server {
    csp_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    hipStream_t aux = nullptr;          // clears a broken job's barrier while the workers run
    hipEvent_t ev_done = nullptr;
    bool running = false;
    bool stop_sent = false;
    // host-coherent memory shared with the kernel
    SrvCtl *hctl = nullptr;
    SJ *hjobs = nullptr;
    unsigned *hslots = nullptr;
    Done *hdone = nullptr;
    long long *hpath = nullptr;
    size_t path_words = 0;
    // device memory
    uint8_t *arena = nullptr;
    size_t arena_bytes = 0;
    uint8_t *fixed = nullptr;
    size_t fixed_bytes = 0;
    size_t off_state = 0, off_dtail = 0, off_watch = 0, off_out = 0, off_cnt = 0, off_bar = 0, bar_stride = 0;
    int max_jobs = 0;
    unsigned ring = 0;
    int workers = 0;
    size_t lds = 0;
    unsigned long long tail = 0, seq = 0, hb = 0;
    int busy = 0;                       // workgroups the admitted jobs need
    int active = 0;
    RangeAlloc dev_alloc, path_alloc;
    std::deque<SrvReq> pending;
    std::vector<SrvAct> act;
    std::vector<int> free_jobs;
    std::deque<SrvDone> ready;
    std::vector<SrvDone> handed;        // completions returned by the last poll
};

namespace {

int srv_fail(csp_server *s, int code, const char *what, hipError_t e = hipSuccess)
{
    return fail(s ? s->ctx : nullptr, code, what, e);
}

size_t srv_footprint(const SrvReq &r)
{
    const GangPlan &pl = r.plan;
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t NO = 2 * pl.K + 1;
    return up((size_t)pl.N * rec_bytes(r.q.d)) + up((size_t)pl.g * pl.c * 4) + up((size_t)pl.pool * 8) +
           up(2ull * pl.g * NO * pl.ccap * 8) + up((size_t)2 * pl.g * NOMAX * 8) +
           up((size_t)pl.g * ((pl.c + 31) / 32) * 4);
}

size_t srv_path_words(const SrvReq &r)
{
    return r.q.reconstruct ? (size_t)std::min<long long>((long long)r.q.M, r.N) : 1;
}

// Launch the workers if jobs wait and none run (first use, or after the
// workers left on stop or a stale heartbeat).
int srv_ensure_running(csp_server *s)
{
    csp_ctx *ctx = s->ctx;
    if (s->running) {
        const hipError_t q = hipEventQuery(s->ev_done);
        if (q == hipSuccess) s->running = false;
        else if (q != hipErrorNotReady) return srv_fail(s, CSP_EDEVICE, "serving kernel", q);
    }
    if (s->running || s->active == 0) return CSP_OK;
    __atomic_store_n(&s->hctl->stop, 0u, __ATOMIC_RELEASE);
    s->stop_sent = false;
    hipLaunchKernelGGL(k_serve_reset, dim3(1), dim3(1), 0, s->stream,
                       reinterpret_cast<unsigned long long *>(s->fixed + s->off_state),
                       reinterpret_cast<unsigned *>(s->fixed + s->off_watch));
    ServeArgs a;
    a.jobs = s->hjobs;
    a.slots = s->hslots;
    a.ring = s->ring;
    a.ctl = s->hctl;
    a.state = reinterpret_cast<unsigned long long *>(s->fixed + s->off_state);
    a.dtail = reinterpret_cast<unsigned long long *>(s->fixed + s->off_dtail);
    a.watch = reinterpret_cast<unsigned *>(s->fixed + s->off_watch);
    a.stale = ctx->wall_khz * 2000ull;   // 2 s without a heartbeat
    a.max_jobs = (unsigned)s->max_jobs;
    // cooperative: every worker is resident before any runs, so a gang of
    // workers waiting for each other at its barrier is never left short
    void *args[] = {&a};
    HIP_TRY(hipLaunchCooperativeKernel((const void *)k_serve, dim3(s->workers), dim3(BLOCK), args, (unsigned)s->lds,
                                       s->stream),
            "serving launch");
    HIP_TRY(hipEventRecord(s->ev_done, s->stream), "event");
    s->running = true;
    return CSP_OK;
}

// Admit waiting requests in arrival order while job slots, workers and
// memory allow.
int srv_admit(csp_server *s)
{
    csp_ctx *ctx = s->ctx;
    while (!s->pending.empty() && !s->free_jobs.empty()) {
        SrvReq &r = s->pending.front();
        if (s->busy + r.plan.g > s->workers) break;
        const size_t fp = srv_footprint(r), pw = srv_path_words(r);
        size_t doff = 0, poff = 0;
        if (!s->dev_alloc.take(fp, doff)) break;
        if (!s->path_alloc.take(pw * 8, poff)) {
            s->dev_alloc.give(doff, fp);
            break;
        }
        const int j = s->free_jobs.back();
        s->free_jobs.pop_back();
        SJ &sj = s->hjobs[j];
        SJ w;
        memset(&w, 0, sizeof(w));
        LdsPlan lp;
        lp.ok = true;
        lp.G = r.plan.g;
        lp.c = r.plan.c;
        lp.K = r.plan.K;
        lp.lt = r.plan.lt;
        lp.llist = r.plan.llist;
        lp.lds = r.plan.lds;
        fill_job(w.rj, r.q.d, r.q.n, r.N, lp, r.q.f1, r.q.f2, r.q.A, r.q.B, r.q.M);
        auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
        const GangPlan &pl = r.plan;
        size_t at = doff;
        w.rj.rec = s->arena + at;
        at += up((size_t)pl.N * rec_bytes(r.q.d));
        w.rj.lists = reinterpret_cast<unsigned *>(s->arena + at);
        at += up((size_t)pl.g * pl.c * 4);
        w.rj.pool = reinterpret_cast<uint2 *>(s->arena + at);
        w.rj.pool_flows = pl.pool;
        at += up((size_t)pl.pool * 8);
        w.rj.cand = reinterpret_cast<uint2 *>(s->arena + at);
        w.rj.cand_cap = (unsigned)pl.ccap;
        at += up(2ull * pl.g * (2 * pl.K + 1) * pl.ccap * 8);
        w.rj.pubc = reinterpret_cast<unsigned long long *>(s->arena + at);
        at += up((size_t)2 * pl.g * NOMAX * 8);
        w.abits = reinterpret_cast<unsigned *>(s->arena + at);
        w.rj.bar = reinterpret_cast<BarHdr *>(s->fixed + s->off_bar + (size_t)j * s->bar_stride);
        w.rj.out = nullptr;
        w.rj.labels_out = nullptr;
        w.rj.max_cycles = 0;
        w.rj.wait_limit = ctx->wall_khz * 1000ull * 60ull;   // 60 s
        w.rj.prof = 0;
        w.out0 = reinterpret_cast<Out *>(s->fixed + s->off_out) + 2 * j;
        w.outc = w.out0 + 1;
        w.done_cnt = reinterpret_cast<unsigned *>(s->fixed + s->off_cnt + (size_t)j * 256);
        w.path = s->hpath + poff / 8;
        w.path_cap = (long long)pw;
        w.done = s->hdone + j;
        w.seq = ++s->seq;
        w.recon = r.q.reconstruct ? 1 : 0;
        memcpy(&sj, &w, sizeof(SJ));
        for (int m = 0; m < pl.g; ++m) {
            const size_t k = (size_t)((s->tail + (unsigned long long)m) & (s->ring - 1));
            s->hslots[2 * k] = (unsigned)j;
            s->hslots[2 * k + 1] = (unsigned)m;
        }
        s->tail += (unsigned long long)pl.g;
        __atomic_store_n(&s->hctl->tail, s->tail, __ATOMIC_RELEASE);
        SrvAct &a = s->act[j];
        a.rq = r;
        a.seq = w.seq;
        a.dev_off = doff;
        a.dev_len = fp;
        a.path_off = poff;
        a.path_len = pw * 8;
        a.live = true;
        s->busy += pl.g;
        s->active += 1;
        s->pending.pop_front();
    }
    // A request that does not fit even an idle server can never run.
    if (!s->pending.empty() && s->active == 0) {
        SrvReq r = s->pending.front();
        s->pending.pop_front();
        SrvDone d;
        memset(&d.c, 0, sizeof(d.c));
        d.c.tag = r.q.tag;
        d.c.status = CSP_ENOMEM;
        d.c.res = csp_result{-1, -1, -1, -1, -1};
        s->ready.push_back(std::move(d));
    }
    return CSP_OK;
}

void srv_counters(csp_counters &c, const unsigned long long *v)
{
    c.C = (int64_t)v[0];
    c.U = (int64_t)v[1];
    c.D = (int64_t)v[2];
    c.E = (int64_t)v[3];
    c.R = (int64_t)v[4];
    c.P = (int64_t)v[5];
    c.I = (int64_t)v[6];
}

// Collect finished jobs; re-queue those whose wheel overflowed.
void srv_reap(csp_server *s)
{
    std::vector<SrvReq> again;
    for (int j = 0; j < s->max_jobs; ++j) {
        SrvAct &a = s->act[j];
        if (!a.live) continue;
        if (__atomic_load_n(&s->hdone[j].seq, __ATOMIC_ACQUIRE) != a.seq) continue;
        const Done &dn = s->hdone[j];
        const int st = __atomic_load_n(&dn.status, __ATOMIC_ACQUIRE);
        a.live = false;
        s->busy -= a.rq.plan.g;
        s->active -= 1;
        s->dev_alloc.give(a.dev_off, a.dev_len);
        if (st == ST_OVERFLOW && a.rq.attempts < 16) {
            SrvReq r = a.rq;
            r.attempts += 1;
            r.plan.pool *= 2;
            r.plan.ccap = std::min<unsigned long long>(r.plan.ccap * 2, 2ull * r.q.d * r.plan.c);
            s->path_alloc.give(a.path_off, a.path_len);
            s->free_jobs.push_back(j);
            again.push_back(r);
            continue;
        }
        SrvDone d;
        memset(&d.c, 0, sizeof(d.c));
        d.c.tag = a.rq.q.tag;
        d.c.status = st == ST_DONE ? CSP_OK
                     : st == ST_INVAL ? CSP_EINVAL
                     : st == ST_OVERFLOW ? CSP_EOVERFLOW
                     : st == ST_CANCELED ? CSP_ECANCELED
                                         : CSP_EDEVICE;
        d.c.res.T = dn.res[0];
        d.c.res.X = dn.res[1];
        d.c.res.x = dn.res[2];
        d.c.res.Y = dn.res[3];
        d.c.res.F2 = dn.res[4];
        srv_counters(d.c.cnt, dn.ctr);
        srv_counters(d.c.cnt_chain, dn.ctr_chain);
        d.c.solves = dn.solves;
        if (d.c.status == CSP_OK && a.rq.q.reconstruct && dn.path_len > 0) {
            const long long *pp = s->hpath + a.path_off / 8;
            d.path.resize((size_t)dn.path_len);
            for (long long i = 0; i < dn.path_len; ++i) d.path[(size_t)i] = pp[dn.path_len - 1 - i];
        }
        d.c.path_len = (int64_t)d.path.size();
        s->path_alloc.give(a.path_off, a.path_len);
        // a gang whose barrier broke leaves its barrier lines dirty (and the
        // broken flag set): every member has left the job, so clear them on
        // the side stream before the slot is used again; retire the slot
        // only if that fails
        bool reuse = true;
        if (st == ST_BROKEN) {
            unsigned *bw = reinterpret_cast<unsigned *>(s->fixed + s->off_bar + (size_t)j * s->bar_stride);
            const unsigned long long words = s->bar_stride / 4;
            hipLaunchKernelGGL(k_zero, dim3((unsigned)std::min<unsigned long long>((words + 255) / 256, 1024ull)),
                               dim3(256), 0, s->aux, bw, words);
            reuse = hipGetLastError() == hipSuccess && hipStreamSynchronize(s->aux) == hipSuccess;
        }
        if (reuse) s->free_jobs.push_back(j);
        s->ready.push_back(std::move(d));
    }
    // overflowed requests go back to the front, in their original order
    for (auto it = again.rbegin(); it != again.rend(); ++it) s->pending.push_front(*it);
}

}  // namespace

extern "C" {

int csp_serve_open(csp_ctx *ctx, uint64_t arena_bytes, int max_jobs, csp_server **out)
{
    if (!ctx || !out || max_jobs < 1 || max_jobs > 4096 || arena_bytes < (1u << 20))
        return fail(ctx, CSP_EINVAL, "serve_open arguments");
    *out = nullptr;
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    csp_server *s = new csp_server;
    s->ctx = ctx;
    auto bail = [&](int code, const char *what, hipError_t e) {
        (void)csp_serve_close(s);
        return fail(ctx, code, what, e);
    };
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking)) != hipSuccess)
        return bail(CSP_EDEVICE, "serve stream", e);
    if ((e = hipStreamCreateWithFlags(&s->aux, hipStreamNonBlocking)) != hipSuccess)
        return bail(CSP_EDEVICE, "serve side stream", e);
    if ((e = hipEventCreateWithFlags(&s->ev_done, hipEventDisableTiming)) != hipSuccess)
        return bail(CSP_EDEVICE, "serve event", e);
    const void *kf = (const void *)k_serve;
    s->lds = ctx->lds_limit > 4096 ? ctx->lds_limit - 4096 : 0;
    if ((e = hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)s->lds)) != hipSuccess)
        return bail(CSP_EDEVICE, "serve LDS attribute", e);
    int nb = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kf, BLOCK, s->lds)) != hipSuccess || nb < 1)
        return bail(CSP_EDEVICE, "serve occupancy", e);
    s->workers = std::min(nb * ctx->num_cu, GMAX);
    s->max_jobs = max_jobs;
    s->ring = 1;
    while (s->ring < 2u * (unsigned)s->workers) s->ring <<= 1;
    // host-coherent tables
    const unsigned fl = hipHostMallocCoherent | hipHostMallocMapped;
    s->path_words = std::max<size_t>(1u << 16, (size_t)max_jobs * 8192);
    if ((e = hipHostMalloc((void **)&s->hctl, sizeof(SrvCtl), fl)) != hipSuccess) return bail(CSP_ENOMEM, "serve control", e);
    if ((e = hipHostMalloc((void **)&s->hjobs, sizeof(SJ) * max_jobs, fl)) != hipSuccess) return bail(CSP_ENOMEM, "serve jobs", e);
    if ((e = hipHostMalloc((void **)&s->hslots, 8ull * s->ring, fl)) != hipSuccess) return bail(CSP_ENOMEM, "serve slots", e);
    if ((e = hipHostMalloc((void **)&s->hdone, sizeof(Done) * max_jobs, fl)) != hipSuccess) return bail(CSP_ENOMEM, "serve results", e);
    if ((e = hipHostMalloc((void **)&s->hpath, 8ull * s->path_words, fl)) != hipSuccess) return bail(CSP_ENOMEM, "serve paths", e);
    memset(s->hctl, 0, sizeof(SrvCtl));
    memset(s->hjobs, 0, sizeof(SJ) * max_jobs);
    memset(s->hslots, 0, 8ull * s->ring);
    memset(s->hdone, 0, sizeof(Done) * max_jobs);
    // device: control words, per-job outputs, finish counters and barriers
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t at = 0;
    s->off_state = at;
    at += 256;
    s->off_dtail = at;
    at += 256;
    s->off_watch = at;
    at += 256;
    s->off_out = at;
    at = up(at + 2 * sizeof(Out) * max_jobs);
    s->off_cnt = at;
    at = up(at + 256ull * max_jobs);
    s->bar_stride = up(bar_bytes(GMAX));
    s->off_bar = at;
    at += s->bar_stride * max_jobs;
    s->fixed_bytes = at;
    if ((e = hipMalloc((void **)&s->fixed, s->fixed_bytes)) != hipSuccess) return bail(CSP_ENOMEM, "serve tables", e);
    if ((e = hipMalloc((void **)&s->arena, arena_bytes)) != hipSuccess) return bail(CSP_ENOMEM, "serve arena", e);
    s->arena_bytes = arena_bytes;
    {
        const unsigned long long words = s->fixed_bytes / 4;
        const int nbz = (int)std::max(1ull, std::min((words + 255) / 256, 4096ull));
        hipLaunchKernelGGL(k_zero, dim3(nbz), dim3(256), 0, s->stream, reinterpret_cast<unsigned *>(s->fixed), words);
        if ((e = hipGetLastError()) != hipSuccess) return bail(CSP_EDEVICE, "serve zero", e);
        if ((e = hipStreamSynchronize(s->stream)) != hipSuccess) return bail(CSP_EDEVICE, "serve zero", e);
    }
    s->dev_alloc.reset(arena_bytes & ~(size_t)255);
    s->path_alloc.reset(8ull * s->path_words);
    s->act.resize(max_jobs);
    for (int j = max_jobs - 1; j >= 0; --j) s->free_jobs.push_back(j);
    *out = s;
    return CSP_OK;
}

int csp_serve_submit(csp_server *s, const csp_request *req)
{
    if (!s || !req) return CSP_EINVAL;
    csp_ctx *ctx = s->ctx;
    const csp_request &q = *req;
    if (!q.f1 || !q.f2 || !q.A || !q.B) return fail(ctx, CSP_EINVAL, "null argument in request");
    SrvReq r;
    r.q = q;
    r.q.reconstruct = q.reconstruct ? 1 : 0;
    int rc = check_shape(ctx, q.d, q.n, q.M, r.N);
    if (rc) return rc;
    // a served request gets about one workgroup per 8K vertices (up to half
    // the workers): its reconstruction chain is a long run of short cycles
    const int g_want = (int)std::min<long long>((r.N + 8191) / 8192, std::max(1, s->workers / 2));
    rc = plan_gang(ctx, s->lds, s->workers, q.d, q.n, r.N, q.M, r.plan, r.N <= 32768 ? 1 : g_want);
    if (rc) return rc;
    if (srv_footprint(r) > s->dev_alloc.cap) return fail(ctx, CSP_ENOMEM, "request larger than the serving arena");
    if (srv_path_words(r) * 8 > s->path_alloc.cap) return fail(ctx, CSP_ENOMEM, "path longer than the path pool");
    if (s->stop_sent) {
        // the workers were told to leave when idle; keep them
        __atomic_store_n(&s->hctl->stop, 0u, __ATOMIC_RELEASE);
        s->stop_sent = false;
    }
    s->pending.push_back(r);
    rc = srv_admit(s);
    if (rc) return rc;
    return srv_ensure_running(s);
}

int csp_serve_poll(csp_server *s, csp_completion *out, int cap, int *count)
{
    if (!s || !count || cap < 0 || (cap > 0 && !out)) return CSP_EINVAL;
    *count = 0;
    s->handed.clear();
    __atomic_store_n(&s->hctl->heartbeat, ++s->hb, __ATOMIC_RELEASE);
    srv_reap(s);
    int rc = srv_admit(s);
    if (rc) return rc;
    rc = srv_ensure_running(s);
    if (rc) return rc;
    if (s->running && s->active == 0 && s->pending.empty() && !s->stop_sent) {
        // idle: let the workers leave so the GPU is free for other work
        __atomic_store_n(&s->hctl->stop, 1u, __ATOMIC_RELEASE);
        s->stop_sent = true;
    }
    while (*count < cap && !s->ready.empty()) {
        s->handed.push_back(std::move(s->ready.front()));
        s->ready.pop_front();
        SrvDone &d = s->handed.back();
        d.c.path = d.path.empty() ? nullptr : d.path.data();
        out[(*count)++] = d.c;
    }
    return CSP_OK;
}

int csp_serve_pending(const csp_server *s, int *queued, int *running)
{
    if (!s) return CSP_EINVAL;
    if (queued) *queued = (int)s->pending.size() + (int)s->ready.size();
    if (running) *running = s->active;
    return CSP_OK;
}

int csp_serve_close(csp_server *s)
{
    if (!s) return CSP_OK;
    int rc = CSP_OK;
    if (s->hctl && s->ev_done && s->stream) {
        // finish admitted work (requests not yet admitted are dropped), then
        // let the workers leave
        s->pending.clear();
        while (s->active > 0) {
            __atomic_store_n(&s->hctl->heartbeat, ++s->hb, __ATOMIC_RELEASE);
            srv_reap(s);
            if (srv_ensure_running(s) != CSP_OK) {
                rc = CSP_EDEVICE;
                break;
            }
        }
        __atomic_store_n(&s->hctl->stop, 1u, __ATOMIC_RELEASE);
        if (s->running && hipEventSynchronize(s->ev_done) != hipSuccess) rc = CSP_EDEVICE;
        s->running = false;
    }
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->ev_done) (void)hipEventDestroy(s->ev_done);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->aux) (void)hipStreamDestroy(s->aux);
    if (s->arena) (void)hipFree(s->arena);
    if (s->fixed) (void)hipFree(s->fixed);
    if (s->hctl) (void)hipHostFree(s->hctl);
    if (s->hjobs) (void)hipHostFree(s->hjobs);
    if (s->hslots) (void)hipHostFree(s->hslots);
    if (s->hdone) (void)hipHostFree(s->hdone);
    if (s->hpath) (void)hipHostFree(s->hpath);
    delete s;
    return rc;
}

int csp_set_trace(csp_ctx *ctx, int64_t *trace, int64_t cap)
{
    if (!ctx || cap < 0 || (cap > 0 && !trace)) return CSP_EINVAL;
    ctx->trace = cap > 0 ? reinterpret_cast<long long *>(trace) : nullptr;
    ctx->trace_cap = cap;
    return CSP_OK;
}

int csp_last_trace_rows(const csp_ctx *ctx, int64_t *rows)
{
    if (!ctx || !rows) return CSP_EINVAL;
    *rows = ctx->last_trace_rows;
    return CSP_OK;
}

int csp_set_path(csp_ctx *ctx, int path)
{
    if (!ctx || path < 0 || path > 3) return CSP_EINVAL;
    ctx->path_override = path;
    return CSP_OK;
}

int csp_last_path(const csp_ctx *ctx)
{
    return ctx ? ctx->last_path : CSP_EINVAL;
}

int csp_set_blocks(csp_ctx *ctx, int blocks)
{
    if (!ctx || blocks < 0) return CSP_EINVAL;
    ctx->blocks_override = blocks;
    return CSP_OK;
}

int csp_autotune(csp_ctx *ctx, int d, int64_t n, const uint8_t *f1, const uint8_t *f2, const uint8_t *A,
                 const uint8_t *B, uint32_t M, int *blocks, int *path, float *ms, void *stream)
{
    if (!ctx || !f1 || !f2 || !A || !B) return fail(ctx, CSP_EINVAL, "null argument");
    long long N = 0;
    int rc = check_shape(ctx, d, n, M, N);
    if (rc) return rc;
    const int save_b = ctx->blocks_override, save_p = ctx->path_override;
    auto forget = [&]() {
        ctx->tuned.erase(std::remove_if(ctx->tuned.begin(), ctx->tuned.end(),
                                        [&](const csp_ctx::Tuned &e) { return e.d == d && e.N == N; }),
                         ctx->tuned.end());
    };
    forget();
    ctx->blocks_override = 0;
    ctx->path_override = 0;
    // candidates: workgroup counts around the automatic choice; for d = 3
    // both range shapes explicitly (contiguous ranges, path 1, and x-pencils,
    // path 3), whichever the automatic choice would be, and the global-label
    // kernel; else path 0 (the automatic kernel choice)
    const int b0 = blocks_for(ctx, d, N);
    std::vector<int> bs;
    for (int b : {b0, b0 / 2, b0 / 4, 2 * b0})
        if (b >= 1 && b <= ctx->max_blocks[d] && std::find(bs.begin(), bs.end(), b) == bs.end()) bs.push_back(b);
    std::vector<int> ps = {0};
    if (d == 3) ps = {1, 3, 2};                   // 2 (global labels) always fits
    // the configuration the automatic choice would run (path_for without a
    // tuned entry): the baseline the 3 % rule compares with
    const int auto_p = d == 3 ? (N >= (1ll << 23) ? 3 : 1) : 0;
    bool have_base = false;
    csp_result r0, r1;
    csp_counters c0, c1;
    bool have = false;
    csp_ctx::Tuned best{d, N, b0, 0, 0.f, -1}, base = best;
    const long long save_dense = ctx->dense_override;
    ctx->dense_override = -1;
    for (int pth : ps) {
        for (int b : bs) {
            ctx->blocks_override = b;
            ctx->path_override = pth;
            float t = -1.f;
            for (int rep = 0; rep < 2 && rc == CSP_OK; ++rep) {
                rc = solve_impl(ctx, d, n, f1, f2, A, B, M, nullptr, &r1, &c1, 0, stream, false);
                if (rc == CSP_OK && (t < 0.f || ctx->last_ms < t)) t = ctx->last_ms;
            }
            if (rc == CSP_EINVAL && pth != 0) {         // this range shape does not fit: not a candidate
                rc = CSP_OK;
                continue;
            }
            if (rc) {
                ctx->blocks_override = save_b;
                ctx->path_override = save_p;
                ctx->dense_override = save_dense;
                return rc;
            }
            if (!have_base && (!have || (pth == auto_p && b == b0))) {
                base = csp_ctx::Tuned{d, N, b, pth, t, -1};  // the automatic configuration
                have_base = pth == auto_p && b == b0;
            }
            if (!have) {
                r0 = r1;
                c0 = c1;
                have = true;
            } else if (memcmp(&r0, &r1, sizeof(r0)) != 0 || memcmp(&c0, &c1, sizeof(c0)) != 0) {
                ctx->blocks_override = save_b;
                ctx->path_override = save_p;
                ctx->dense_override = save_dense;
                return fail(ctx, CSP_EDEVICE, "autotune: two configurations gave different results");
            }
            if (best.ms <= 0.f || t < best.ms) best = csp_ctx::Tuned{d, N, b, pth, t, -1};
        }
    }
    // another configuration replaces the automatic one only when it is at
    // least 3 % faster, so that timing noise does not pick it
    if (best.ms > 0.97f * base.ms) best = base;
    // then the dense threshold on the chosen shape: flows delivered to a
    // range in a cycle above which I_t is built by a bitmap sweep (never,
    // always, and between)
    {
        ctx->blocks_override = best.blocks;
        ctx->path_override = best.path;
        const csp_ctx::Tuned shape = best;
        for (long long thr : {(long long)DENSE_NEVER, 0ll, 2048ll, 4096ll, 8192ll, 16384ll}) {
            ctx->dense_override = thr;
            float t = -1.f;
            for (int rep = 0; rep < 2 && rc == CSP_OK; ++rep) {
                rc = solve_impl(ctx, d, n, f1, f2, A, B, M, nullptr, &r1, &c1, 0, stream, false);
                if (rc == CSP_OK && (t < 0.f || ctx->last_ms < t)) t = ctx->last_ms;
            }
            if (rc == CSP_OK && (memcmp(&r0, &r1, sizeof(r0)) != 0 || memcmp(&c0, &c1, sizeof(c0)) != 0))
                rc = fail(ctx, CSP_EDEVICE, "autotune: two dense thresholds gave different results");
            if (rc) {
                ctx->blocks_override = save_b;
                ctx->path_override = save_p;
                ctx->dense_override = save_dense;
                return rc;
            }
            if (ctx->last_path != 1) break;         // global-label kernel: no ranges to sweep
            if (t < 0.97f * best.ms) {
                best = shape;
                best.dense = thr;
                best.ms = t;
            }
        }
    }
    ctx->blocks_override = save_b;
    ctx->path_override = save_p;
    ctx->dense_override = save_dense;
    ctx->tuned.push_back(best);
    if (blocks) *blocks = best.blocks;
    if (path) *path = best.path;
    if (ms) *ms = best.ms;
    return CSP_OK;
}

int csp_set_wait_limit(csp_ctx *ctx, int64_t microseconds)
{
    if (!ctx) return CSP_EINVAL;
    ctx->wait_us = microseconds < 0 ? -1 : microseconds;
    return CSP_OK;
}

int csp_set_dense_threshold(csp_ctx *ctx, int64_t flows)
{
    if (!ctx) return CSP_EINVAL;
    ctx->dense_override = flows < 0 ? -1 : flows;
    return CSP_OK;
}

int csp_tuned_dense_threshold(const csp_ctx *ctx, int d, int64_t n, int64_t *flows)
{
    if (!ctx || !flows || d < 1 || d > 4 || n < 2) return CSP_EINVAL;
    long long N = 1;
    for (int k = 0; k < d; ++k) N *= n;
    const csp_ctx::Tuned *e = tuned_for(ctx, d, N);
    *flows = e ? e->dense : -1;
    return CSP_OK;
}

int csp_autotune_clear(csp_ctx *ctx)
{
    if (!ctx) return CSP_EINVAL;
    ctx->tuned.clear();
    ctx->batch_target = 0;
    ctx->batch_seen.clear();
    return CSP_OK;
}

int csp_set_batch_target(csp_ctx *ctx, int64_t vertices_per_workgroup)
{
    if (!ctx || vertices_per_workgroup < 0) return CSP_EINVAL;
    ctx->batch_target = vertices_per_workgroup;
    return CSP_OK;
}

int csp_autotune_batch(csp_ctx *ctx, int count, const csp_problem *probs, int64_t *target, float *ms,
                       void *stream)
{
    if (!ctx || count < 1 || !probs) return fail(ctx, CSP_EINVAL, "null argument");
    const long long save = ctx->batch_target;
    std::vector<csp_result> r0((size_t)count), r1((size_t)count);
    std::vector<csp_counters> c0((size_t)count), c1((size_t)count);
    long long best_t = 0;
    float best_ms = -1.f, base_ms = -1.f;
    bool have = false;
    for (long long tgt : {0ll, 65536ll, 32768ll, 16384ll, 8192ll}) {
        ctx->batch_target = tgt;
        float t = -1.f;
        int rc = CSP_OK;
        for (int rep = 0; rep < (have ? 1 : 2) && rc == CSP_OK; ++rep) {   // the first run also warms the arena
            rc = csp_solve_batch(ctx, count, probs, r1.data(), c1.data(), stream);
            if (rc == CSP_OK) t = ctx->last_ms;
        }
        if (rc) {
            ctx->batch_target = save;
            return rc;
        }
        if (!have) {
            r0 = r1;
            c0 = c1;
            have = true;
            base_ms = t;
        } else {
            for (int i = 0; i < count; ++i) {
                if (memcmp(&r0[i], &r1[i], sizeof(csp_result)) == 0 && memcmp(&c0[i], &c1[i], sizeof(csp_counters)) == 0)
                    continue;
                char msg[200];
                snprintf(msg, sizeof(msg),
                         "autotune: batch problem %d differs at %lld vertices per workgroup "
                         "(T %lld/%lld, U %lld/%lld, P %lld/%lld, I %lld/%lld)",
                         i, tgt, (long long)r0[i].T, (long long)r1[i].T, (long long)c0[i].U, (long long)c1[i].U,
                         (long long)c0[i].P, (long long)c1[i].P, (long long)c0[i].I, (long long)c1[i].I);
                ctx->batch_target = save;
                return fail(ctx, CSP_EDEVICE, msg);
            }
        }
        if (best_ms < 0.f || t < best_ms) {
            best_ms = t;
            best_t = tgt;
        }
    }
    if (best_ms > 0.97f * base_ms) {        // keep the fewest-workgroup plan unless clearly slower
        best_ms = base_ms;
        best_t = 0;
    }
    ctx->batch_target = best_t;
    if (target) *target = best_t;
    if (ms) *ms = best_ms;
    return CSP_OK;
}

}  // extern "C"
