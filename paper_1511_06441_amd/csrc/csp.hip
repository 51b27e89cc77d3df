// csp.hip -- libcsp: the water-flow constrained-shortest-path cycle on
// lattice cubes in Z^d, written for MI355X (gfx950, CDNA4, wave64).
//
// Method: I. Matic, "A parallel algorithm for the constrained shortest path
// problem on lattice graphs" (arXiv:1511.06441), sections 4-6,
// Algorithms 1-11.  The paper keeps per-edge records (time remaining,
// source, state) plus a separate phantom list and runs nine barrier-separated
// steps per time unit.  Here every unit of water in transit is a flow record
// (destination, quality, arriving direction) filed in a timing wheel by its
// arrival time, so regular and phantom edges are the same thing and a cycle
// is two phases:
//
//   arrival   (Steps 1-3, 8): deliver the bucket of time t; atomicMax the
//             quality into the destination's label; the first thread that
//             raises a label this cycle appends the vertex to the improved
//             set I_t.  A vertex of B in I_t ends the run (Step 6).
//   departure (Steps 4-5): every Q in I_t tests its 2d lattice neighbours;
//             if Label(Q) - f2 > Label(P), a flow (P, Label(Q) - f2) is filed
//             in bucket (t + f1) mod W.  Delivered flows simply leave their
//             bucket (Steps 7, 9).
//
// Step 1's time skip is the first non-empty bucket after t.  Both phases run
// inside one persistent cooperative kernel separated by a grid barrier.
//
// Label words pack (label << 1) | idle: idle = 1 means "not yet appended to
// this cycle's improved set".  A delivery does atomicMax(word, q << 1), which
// raises the label and clears the idle bit in one operation; the returned
// old word tells the thread whether it raised the label and whether it was
// the first to do so this cycle.  Departure sets the idle bit again.
//
// All arithmetic is integer; results are bit-identical to the CPU oracle.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "csp.h"

namespace {

constexpr int BLOCK = 256;
constexpr int MAXW = 256;          // f1 <= 255, so 256 buckets always suffice
constexpr unsigned IDLE = 1u;

// Control block in device memory: bucket fill counts, queue sizes, barrier
// state, termination reductions and counters.
struct Ctl {
    unsigned cnt[MAXW];
    unsigned qcount[2];
    unsigned bar_count;
    unsigned bar_gen;
    unsigned bhit;
    unsigned ydir;
    unsigned long long xkey;
    unsigned long long ctr[8];     // C U D E R P I
    long long res[5];              // T X x Y F2
    int status;
    int broken;                    // a barrier wait timed out
};

enum { ST_RUNNING = 0, ST_DONE = 1, ST_OVERFLOW = 2, ST_CANCELED = 3, ST_BROKEN = 4 };

struct Info {
    unsigned bad;
    unsigned maxf1;
    unsigned nA;
    unsigned pad;
};

struct Params {
    long long n, N;
    long long stride[4];
    const uint8_t *f1, *f2, *A, *B;
    unsigned M;
    unsigned W;                    // power of two > max f1
    unsigned long long cap;        // flows per bucket
    unsigned *lab;
    unsigned *queue0, *queue1;
    unsigned *bhitv;
    uint2 *pool;
    Ctl *ctl;
    unsigned *labels_out;
    long long max_cycles;
    unsigned long long wait_limit; // wall-clock ticks a barrier wait may take
};

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ unsigned ld_acq(const unsigned *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long ld_acq64(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Append pred-true lanes of a wavefront to a global list with one atomic.
__device__ __forceinline__ bool wave_append(unsigned *counter, bool pred, unsigned &slot)
{
    const unsigned long long m = __ballot(pred);
    if (m == 0) return false;
    const int lead = __ffsll((long long)m) - 1;
    const int lane = __lane_id();
    unsigned base = 0;
    if (lane == lead)
        base = __hip_atomic_fetch_add(counter, (unsigned)__popcll(m), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
    base = __shfl(base, lead);
    slot = base + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
    return pred;
}

// Sense-counting grid barrier for a cooperative launch (all blocks are
// co-resident, so every wait ends).  Thread 0 of each block arrives with a
// release and waits with an acquire at agent scope; the block barriers
// around it extend that ordering to the whole block.  A wait that outlasts
// `limit` wall-clock ticks marks the run broken and returns false, so a
// logic error drains the grid instead of hanging it.
__device__ __forceinline__ bool grid_barrier(Ctl *ctl, unsigned &gen, unsigned long long limit)
{
    __shared__ int s_ok;
    __syncthreads();
    if (gridDim.x > 1) {
        if (threadIdx.x == 0) {
            int ok = 1;
            const unsigned g = gen;
            const unsigned arrived = __hip_atomic_fetch_add(&ctl->bar_count, 1u, __ATOMIC_ACQ_REL,
                                                            __HIP_MEMORY_SCOPE_AGENT);
            if (arrived == gridDim.x - 1) {
                __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&ctl->bar_gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                const unsigned long long t0 = wall_clock64();
                while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                    __builtin_amdgcn_s_sleep(1);
                    if (wall_clock64() - t0 > limit) {
                        __hip_atomic_store(&ctl->broken, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok = 0;
                        break;
                    }
                }
            }
            if (__hip_atomic_load(&ctl->broken, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
            s_ok = ok;
        }
        gen += 1;
    } else if (threadIdx.x == 0) {
        s_ok = 1;
    }
    __syncthreads();
    return s_ok != 0;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Input checks: positive f on real edges, A and B disjoint; also the largest
// f1 (sizes the wheel) and |A|.
__global__ void __launch_bounds__(BLOCK) k_validate(int d, long long n, long long N,
                                                    const uint8_t *f1, const uint8_t *f2,
                                                    const uint8_t *A, const uint8_t *B, Info *info)
{
    const long long gsize = (long long)gridDim.x * BLOCK;
    const long long gtid = (long long)blockIdx.x * BLOCK + threadIdx.x;
    unsigned bad = 0, mx = 0, na = 0;
    for (long long i = gtid; i < (long long)d * N; i += gsize) {
        const long long k = i / N, u = i - k * N;
        long long s = 1;
        for (long long j = 0; j < k; ++j) s *= n;
        const long long c = (u / s) % n;
        if (c < n - 1) {
            const unsigned a = f1[i], b = f2[i];
            if (a == 0 || b == 0) bad |= 1u;
            mx = a > mx ? a : mx;
        }
    }
    for (long long v = gtid; v < N; v += gsize) {
        const bool a = A[v] != 0;
        if (a && B[v] != 0) bad |= 2u;
        na += a;
    }
    // wave reductions, then one atomic per wave
    for (int o = 32; o > 0; o >>= 1) {
        bad |= __shfl_xor(bad, o);
        mx = max(mx, (unsigned)__shfl_xor(mx, o));
        na += __shfl_xor(na, o);
    }
    if (__lane_id() == 0) {
        if (bad) atomicOr(&info->bad, bad);
        if (mx) atomicMax(&info->maxf1, mx);
        if (na) atomicAdd(&info->nA, na);
    }
}

__global__ void k_zero_info(Info *info)
{
    info->bad = 0;
    info->maxf1 = 0;
    info->nA = 0;
}

// Clear the control block (a kernel rather than a memset, so the sequence
// stays valid inside captured graphs).
__global__ void __launch_bounds__(BLOCK) k_reset_ctl(Ctl *ctl)
{
    unsigned *w = reinterpret_cast<unsigned *>(ctl);
    for (unsigned i = threadIdx.x; i < sizeof(Ctl) / 4; i += BLOCK) w[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) ctl->ydir = 0xFFFFFFFFu;
}

template <int D>
__global__ void __launch_bounds__(BLOCK) k_solve(Params p)
{
    __shared__ unsigned s_cnt[MAXW];
    __shared__ unsigned s_base[MAXW];
    __shared__ long long s_next;
    __shared__ unsigned long long s_red[3];

    Ctl *ctl = p.ctl;
    const unsigned tid = threadIdx.x;
    const bool lead_block = blockIdx.x == 0;
    const unsigned long long gsize = (unsigned long long)gridDim.x * BLOCK;
    const unsigned long long gtid = (unsigned long long)blockIdx.x * BLOCK + tid;
    const unsigned Wm = p.W - 1;
    const long long n = p.n, N = p.N;
    unsigned gen = 0;
    bool status_init_broken = false;

    unsigned long long cU = 0, cD = 0, cE = 0;           // per thread
    unsigned long long cC = 0, cR = 0, cP = 0, cI = 0;   // thread 0 of block 0

    // ---- Initialization (Algorithm 3): Label = M on A, 0 elsewhere; A is I_0.
    for (unsigned long long v = gtid; v < (unsigned long long)N; v += gsize) {
        const bool a = p.A[v] != 0;
        p.lab[v] = a ? ((p.M << 1) | IDLE) : IDLE;
        unsigned slot;
        if (wave_append(&ctl->qcount[0], a, slot)) p.queue0[slot] = (unsigned)v;
    }
    if (!grid_barrier(ctl, gen, p.wait_limit)) status_init_broken = true;
    {
        const unsigned nA = ld_acq(&ctl->qcount[0]);
        cU += (gtid == 0) ? nA : 0;
    }

    long long t = 0;
    unsigned cyc = 0;
    int status = status_init_broken ? ST_BROKEN : ST_RUNNING;
    unsigned b_last = 0, nb_last = 0;

    while (status == ST_RUNNING) {
        // ---- Departure (Steps 4-5, Algorithms 7-8) from I_t.
        const unsigned par = cyc & 1u;
        const unsigned *queue = par ? p.queue1 : p.queue0;
        const unsigned nq = ld_acq(&ctl->qcount[par]);
        if (lead_block && tid == 0) {
            __hip_atomic_store(&ctl->qcount[par ^ 1u], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->cnt[t & Wm], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const unsigned long long rounds = (nq + gsize - 1) / gsize;
        for (unsigned long long r = 0; r < rounds; ++r) {
            for (unsigned b = tid; b < p.W; b += BLOCK) s_cnt[b] = 0;
            __syncthreads();
            // one slot per direction keeps the arrays in registers
            unsigned eb[2 * D], epos[2 * D], edst[2 * D], ekey[2 * D];
#pragma unroll
            for (int dir = 0; dir < 2 * D; ++dir) eb[dir] = 0xFFFFFFFFu;
            const unsigned long long idx = r * gsize + gtid;
            if (idx < nq) {
                const unsigned Q = queue[idx];
                const unsigned w = p.lab[Q];
                const long long L = (long long)(w >> 1);
                p.lab[Q] = w | IDLE;
                long long c[D];
                {
                    long long rem = Q;
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        c[k] = rem % n;
                        rem /= n;
                    }
                }
#pragma unroll
                for (int dir = 0; dir < 2 * D; ++dir) {
                    // direction codes ascend with the neighbour's index:
                    // -n^(D-1) .. -1, +1 .. +n^(D-1)
                    const bool lower = dir < D;
                    const int k = lower ? D - 1 - dir : dir - D;
                    const bool exists = lower ? (c[k] >= 1) : (c[k] <= n - 2);
                    if (exists) {
                        const long long P = lower ? (long long)Q - p.stride[k] : (long long)Q + p.stride[k];
                        const long long e = (long long)k * N + (lower ? P : (long long)Q);
                        const unsigned a1 = p.f1[e], a2 = p.f2[e];
                        ++cD;
                        const long long q = L - (long long)a2;
                        const long long Lp = (long long)(p.lab[P] >> 1);
                        if (q > Lp) {
                            const unsigned b = (unsigned)((t + a1) & Wm);
                            eb[dir] = b;
                            epos[dir] = atomicAdd(&s_cnt[b], 1u);
                            edst[dir] = (unsigned)P;
                            // the receiver sees the sender in the opposite direction
                            ekey[dir] = ((unsigned)q << 3) | (unsigned)(2 * D - 1 - dir);
                            ++cE;
                        }
                    }
                }
            }
            __syncthreads();
            for (unsigned b = tid; b < p.W; b += BLOCK) {
                const unsigned k = s_cnt[b];
                if (k) s_base[b] = atomicAdd(&ctl->cnt[b], k);
            }
            __syncthreads();
#pragma unroll
            for (int dir = 0; dir < 2 * D; ++dir) {
                if (eb[dir] != 0xFFFFFFFFu) {
                    const unsigned long long pos = (unsigned long long)s_base[eb[dir]] + epos[dir];
                    if (pos < p.cap)
                        p.pool[(unsigned long long)eb[dir] * p.cap + pos] = make_uint2(edst[dir], ekey[dir]);
                }
            }
            __syncthreads();
        }
        if (!grid_barrier(ctl, gen, p.wait_limit)) { status = ST_BROKEN; break; }

        // ---- Step 1 (Algorithm 4): next delivery time = first non-empty bucket.
        if (tid < 64) {
            long long best = -1;
            bool over = false;
            unsigned long long transit = 0;
            for (unsigned j = tid; j + 1 < p.W; j += 64) {
                const unsigned c = ld_acq(&ctl->cnt[(t + 1 + j) & Wm]);
                transit += c;
                if (c > p.cap) over = true;
                if (c && best < 0) best = (long long)j;
            }
            // smallest j with a non-empty bucket across the wave
            unsigned long long mbest = __ballot(best >= 0);
            long long jmin = -1;
            if (mbest) {
                // candidates are strided by 64; take the minimum value
                long long v = best >= 0 ? best : (long long)1 << 40;
                for (int o = 32; o > 0; o >>= 1) {
                    const long long ov = __shfl_xor(v, o);
                    v = ov < v ? ov : v;
                }
                jmin = v;
            }
            over = __ballot(over) != 0;
            for (int o = 32; o > 0; o >>= 1) transit += __shfl_xor(transit, o);
            if (tid == 0) {
                s_next = over ? -2 : (jmin < 0 ? -1 : t + 1 + jmin);
                if (lead_block) cP = transit > cP ? transit : cP;
            }
        }
        __syncthreads();
        const long long tn = s_next;
        if (tn == -2) { status = ST_OVERFLOW; break; }
        if (tn == -1) { status = ST_DONE; break; }                     // condition 2
        if (p.max_cycles > 0 && (long long)cyc >= p.max_cycles) { status = ST_CANCELED; break; }
        t = tn;
        ++cyc;
        if (lead_block && tid == 0) ++cC;

        // ---- Arrival (Steps 1-3 and 8, Algorithms 4-6, 10).
        const unsigned npar = cyc & 1u;
        unsigned *nqueue = npar ? p.queue1 : p.queue0;
        const unsigned b = (unsigned)(t & Wm);
        const unsigned nb = ld_acq(&ctl->cnt[b]);
        const uint2 *bk = p.pool + (unsigned long long)b * p.cap;
        for (unsigned long long j = gtid; j < nb; j += gsize) {
            const uint2 f = bk[j];
            const unsigned P = f.x, q = f.y >> 3;
            bool imp = false;
            if (q > (p.lab[P] >> 1)) {
                const unsigned old = atomicMax(&p.lab[P], q << 1);
                imp = (q > (old >> 1)) && (old & IDLE);
            }
            unsigned slot;
            if (wave_append(&ctl->qcount[npar], imp, slot)) {
                nqueue[slot] = P;
                ++cU;
                if (p.B[P]) {
                    const unsigned s = atomicAdd(&ctl->bhit, 1u);
                    p.bhitv[s] = P;
                }
            }
        }
        if (lead_block && tid == 0) cR += nb;
        b_last = b;
        nb_last = nb;
        if (!grid_barrier(ctl, gen, p.wait_limit)) { status = ST_BROKEN; break; }
        if (lead_block && tid == 0) {
            const unsigned nI = ld_acq(&ctl->qcount[npar]);
            cI = nI > cI ? nI : cI;
        }

        // ---- Step 6 (Algorithm 2): a vertex of B improved -> T = t.
        const unsigned nbh = ld_acq(&ctl->bhit);
        if (nbh) {
            for (unsigned long long i = gtid; i < nbh; i += gsize) {
                const unsigned P = p.bhitv[i];
                const unsigned long long key =
                    ((unsigned long long)(p.lab[P] >> 1) << 32) | (0xFFFFFFFFull - P);
                atomicMax(&ctl->xkey, key);
            }
            if (!grid_barrier(ctl, gen, p.wait_limit)) { status = ST_BROKEN; break; }
            const unsigned long long xk = ld_acq64(&ctl->xkey);
            const unsigned X = (unsigned)(0xFFFFFFFFull - (xk & 0xFFFFFFFFull));
            const unsigned LX = (unsigned)(xk >> 32);
            for (unsigned long long j = gtid; j < nb_last; j += gsize) {
                const uint2 f = bk[j];
                if (f.x == X && (f.y >> 3) == LX) atomicMin(&ctl->ydir, f.y & 7u);
            }
            if (!grid_barrier(ctl, gen, p.wait_limit)) { status = ST_BROKEN; break; }
            if (lead_block && tid == 0) {
                const unsigned yd = ld_acq(&ctl->ydir);
                const bool lower = (int)yd < D;
                const int k = lower ? D - 1 - (int)yd : (int)yd - D;
                const long long Y = lower ? (long long)X - p.stride[k] : (long long)X + p.stride[k];
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
    (void)b_last;

    // ---- outputs
    if (status == ST_DONE && p.labels_out) {
        for (unsigned long long v = gtid; v < (unsigned long long)N; v += gsize)
            p.labels_out[v] = p.lab[v] >> 1;
    }
    if (tid == 0) {
        s_red[0] = 0;
        s_red[1] = 0;
        s_red[2] = 0;
    }
    __syncthreads();
    if (cU) atomicAdd(&s_red[0], cU);
    if (cD) atomicAdd(&s_red[1], cD);
    if (cE) atomicAdd(&s_red[2], cE);
    __syncthreads();
    if (tid == 0) {
        if (s_red[0]) atomicAdd(&ctl->ctr[1], s_red[0]);
        if (s_red[1]) atomicAdd(&ctl->ctr[2], s_red[1]);
        if (s_red[2]) atomicAdd(&ctl->ctr[3], s_red[2]);
        if (lead_block) {
            ctl->ctr[0] = cC;
            ctl->ctr[4] = cR;
            ctl->ctr[5] = cP;
            ctl->ctr[6] = cI;
            ctl->status = ld_acq((const unsigned *)&ctl->broken) ? ST_BROKEN : status;
            if (status == ST_DONE && ld_acq(&ctl->bhit) == 0) {
                ctl->res[0] = -1;
                ctl->res[1] = -1;
                ctl->res[2] = -1;
                ctl->res[3] = -1;
                ctl->res[4] = -1;
            }
        }
    }
}

__global__ void k_set_byte(uint8_t *p, long long i, uint8_t v) { p[i] = v; }

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct csp_ctx {
    int device = 0;
    int num_cu = 0;
    int max_blocks[5] = {0, 0, 0, 0, 0};
    unsigned long long wall_khz = 100000;
    unsigned *lab = nullptr;
    unsigned *q0 = nullptr, *q1 = nullptr, *bhit = nullptr;
    size_t n_cap = 0;
    uint2 *pool = nullptr;
    size_t pool_cap = 0;            // flows
    Ctl *ctl = nullptr;
    Info *info = nullptr;
    Ctl *h_ctl = nullptr;           // pinned
    Info *h_info = nullptr;         // pinned
    uint8_t *in_buf = nullptr;      // staging for host-pointer solves
    size_t in_cap = 0;
    uint8_t *h_byte = nullptr;      // pinned scratch
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    float last_ms = -1.f;
    unsigned long long pool_hint = 0;
    int blocks_override = 0;
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

#define HIP_TRY(call, what)                                  \
    do {                                                     \
        hipError_t e_ = (call);                              \
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

int ensure_vertex_buffers(csp_ctx *ctx, size_t N)
{
    if (N <= ctx->n_cap && ctx->lab) return CSP_OK;
    for (unsigned **b : {&ctx->lab, &ctx->q0, &ctx->q1, &ctx->bhit}) {
        if (*b) (void)hipFree(*b);
        *b = nullptr;
    }
    ctx->n_cap = 0;
    const size_t want = std::max<size_t>(N, 4096);
    for (unsigned **b : {&ctx->lab, &ctx->q0, &ctx->q1, &ctx->bhit}) {
        hipError_t e = hipMalloc((void **)b, want * sizeof(unsigned));
        if (e != hipSuccess) return fail(ctx, CSP_ENOMEM, "vertex buffers", e);
    }
    ctx->n_cap = want;
    return CSP_OK;
}

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

int blocks_for(csp_ctx *ctx, int d, long long N)
{
    if (ctx->blocks_override > 0) return std::min(ctx->blocks_override, ctx->max_blocks[d]);
    // Few vertices: one block (its barrier is a block barrier).  Otherwise
    // about one block per 8K vertices, up to the co-resident limit.
    long long want = (N + 8191) / 8192;
    if (N <= 16384) want = 1;
    long long mx = (long long)ctx->max_blocks[d];
    return (int)std::max(1ll, std::min(want, mx));
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
    {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
            ctx->wall_khz = (unsigned long long)khz;
    }
    for (int d = 1; d <= 4; ++d) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, solve_kernel(d), BLOCK, 0) != hipSuccess || nb < 1)
            nb = 1;
        nb = std::min(nb, 2);
        ctx->max_blocks[d] = nb * ctx->num_cu;
    }
    if (hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess ||
        hipMalloc((void **)&ctx->ctl, sizeof(Ctl)) != hipSuccess ||
        hipMalloc((void **)&ctx->info, sizeof(Info)) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_ctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_info, sizeof(Info), hipHostMallocDefault) != hipSuccess ||
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
    for (void *p : {(void *)ctx->lab, (void *)ctx->q0, (void *)ctx->q1, (void *)ctx->bhit,
                    (void *)ctx->pool, (void *)ctx->ctl, (void *)ctx->info, (void *)ctx->in_buf})
        if (p) (void)hipFree(p);
    for (void *p : {(void *)ctx->h_ctl, (void *)ctx->h_info, (void *)ctx->h_byte})
        if (p) (void)hipHostFree(p);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    delete ctx;
}

const char *csp_last_error(const csp_ctx *ctx)
{
    return ctx ? ctx->err : "no context";
}

int csp_solve_dev(csp_ctx *ctx, int d, int64_t n, const uint8_t *f1, const uint8_t *f2,
                  const uint8_t *A, const uint8_t *B, uint32_t M, uint32_t *labels,
                  csp_result *out, csp_counters *cnt, int64_t max_cycles, void *stream)
{
    if (!ctx || !out || !f1 || !f2 || !A || !B) return fail(ctx, CSP_EINVAL, "null argument");
    long long N = 0;
    int rc = check_shape(ctx, d, n, M, N);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");

    // validate and size the wheel
    hipLaunchKernelGGL(k_zero_info, dim3(1), dim3(1), 0, s, ctx->info);
    {
        const long long work = (long long)d * N;
        const int vb = (int)std::max(1ll, std::min((work + BLOCK - 1) / BLOCK, (long long)ctx->num_cu * 8));
        hipLaunchKernelGGL(k_validate, dim3(vb), dim3(BLOCK), 0, s, d, (long long)n, N, f1, f2, A, B,
                           ctx->info);
    }
    HIP_TRY(hipGetLastError(), "validate launch");
    HIP_TRY(hipMemcpyAsync(ctx->h_info, ctx->info, sizeof(Info), hipMemcpyDeviceToHost, s), "info copy");
    HIP_TRY(hipStreamSynchronize(s), "validate");
    const Info info = *ctx->h_info;
    if (info.bad & 1u) return fail(ctx, CSP_EINVAL, "an edge has f1 or f2 equal to 0");
    if (info.bad & 2u) return fail(ctx, CSP_EINVAL, "A and B overlap");
    unsigned W = 2;
    while (W <= info.maxf1) W <<= 1;

    rc = ensure_vertex_buffers(ctx, (size_t)N);
    if (rc) return rc;

    // bucket capacity: start at 2 * (directed edges) / W flows per bucket
    unsigned long long cap = ctx->pool_hint ? ctx->pool_hint
                                            : std::max<unsigned long long>(65536ull, (4ull * d * N) / W);
    const int G = blocks_for(ctx, d, N);
    // A bucket holds at most one flow per directed edge, so a capacity of
    // 2dN cannot overflow; doubling up to it always ends.
    const unsigned long long cap_max = std::max<unsigned long long>(2ull * d * N, 64ull);
    cap = std::min(std::max<unsigned long long>(cap, 1ull), cap_max);
    for (;;) {
        rc = grow(ctx, &ctx->pool, ctx->pool_cap, (size_t)(cap * W), "transit pool");
        if (rc) return rc;
        Params p;
        memset(&p, 0, sizeof(p));
        p.n = n;
        p.N = N;
        long long st = 1;
        for (int k = 0; k < 4; ++k) {
            p.stride[k] = st;
            if (k < d) st *= n;
        }
        p.f1 = f1;
        p.f2 = f2;
        p.A = A;
        p.B = B;
        p.M = M;
        p.W = W;
        p.cap = cap;
        p.lab = ctx->lab;
        p.queue0 = ctx->q0;
        p.queue1 = ctx->q1;
        p.bhitv = ctx->bhit;
        p.pool = ctx->pool;
        p.ctl = ctx->ctl;
        p.labels_out = labels;
        p.max_cycles = max_cycles;
        p.wait_limit = ctx->wall_khz * 1000ull * 20ull;    // 20 s
        hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(BLOCK), 0, s, ctx->ctl);
        void *args[] = {&p};
        HIP_TRY(hipEventRecord(ctx->ev0, s), "event");
        HIP_TRY(hipLaunchCooperativeKernel(solve_kernel(d), dim3(G), dim3(BLOCK), args, 0, s),
                "solve launch");
        HIP_TRY(hipEventRecord(ctx->ev1, s), "event");
        HIP_TRY(hipMemcpyAsync(ctx->h_ctl, ctx->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s), "ctl copy");
        HIP_TRY(hipStreamSynchronize(s), "solve");
        const Ctl &c = *ctx->h_ctl;
        if (c.status == ST_OVERFLOW) {
            if (cap >= cap_max) return fail(ctx, CSP_EOVERFLOW, "transit pool overflow at the edge bound");
            cap = std::min(cap * 2, cap_max);
            continue;
        }
        if (c.status == ST_CANCELED) return fail(ctx, CSP_ECANCELED, "cycle cap reached");
        if (c.status == ST_BROKEN) return fail(ctx, CSP_EDEVICE, "grid barrier timed out");
        if (c.status != ST_DONE) return fail(ctx, CSP_EDEVICE, "solve did not finish");
        HIP_TRY(hipEventElapsedTime(&ctx->last_ms, ctx->ev0, ctx->ev1), "event time");
        out->T = c.res[0];
        out->X = c.res[1];
        out->x = c.res[2];
        out->Y = c.res[3];
        out->F2 = c.res[4];
        if (cnt) {
            cnt->C = (int64_t)c.ctr[0];
            cnt->U = (int64_t)c.ctr[1];
            cnt->D = (int64_t)c.ctr[2];
            cnt->E = (int64_t)c.ctr[3];
            cnt->R = (int64_t)c.ctr[4];
            cnt->P = (int64_t)c.ctr[5];
            cnt->I = (int64_t)c.ctr[6];
        }
        return CSP_OK;
    }
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

int csp_set_pool_hint(csp_ctx *ctx, uint64_t flows_per_bucket)
{
    if (!ctx) return CSP_EINVAL;
    ctx->pool_hint = flows_per_bucket;
    return CSP_OK;
}

int csp_set_blocks(csp_ctx *ctx, int blocks)
{
    if (!ctx || blocks < 0) return CSP_EINVAL;
    ctx->blocks_override = blocks;
    return CSP_OK;
}

}  // extern "C"
