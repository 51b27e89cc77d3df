/*
 * csp.h -- C ABI of libcsp, an MI355X (gfx950) solver for the constrained
 * shortest path problem on lattice cubes in Z^d by the water-flow,
 * label-correcting method of I. Matic, "A parallel algorithm for the
 * constrained shortest path problem on lattice graphs" (arXiv:1511.06441).
 *
 * Problem (section 1 of the paper): every edge e of the nearest-neighbour
 * lattice on n^d vertices carries a passage time f1(e) and a weight f2(e),
 * both positive integers.  For disjoint vertex sets A and B and a budget M,
 * find the least total time F1 of a path from A to B whose total weight
 * satisfies F2 < M.
 *
 * Method (sections 1, 4-6, Algorithms 1-11): water of quality M starts on A;
 * crossing e takes f1(e) time units and costs f2(e) quality; water of quality
 * 0 stops.  Label(P) is the best quality that has reached P.  Time advances
 * to the next delivery; vertices whose label improves send water on to every
 * neighbour they would improve.  The answer is the first time a vertex of B
 * receives water (section 5, "Termination").
 *
 * Conventions shared by every entry point:
 *   N = n^d.  Vertex v = sum_k c_k n^k (axis 0 varies fastest).
 *   Edge arrays f1, f2: uint8, SoA [d][N]; entry (k, u) is the edge joining
 *     u and u + n^k, id k*N + u.  Entries with c_k(u) = n-1 have no edge and
 *     are ignored.  Real edges need 1 <= f1, f2 <= 255.
 *   Masks A, B: uint8 [N], nonzero = member.  A and B must be disjoint.
 *   M: 1 <= M <= CSP_MAX_M.  The constraint is strict (F2 < M).
 *   Labels (optional output): uint32 [N], the best quality at each vertex at
 *     the answer time T (at the end of the run when there is no path).
 *
 * Result (section 1, section 5 "Termination"):
 *   T  least F1 (time of the first delivery to B)
 *   X  the vertex of B reached at T with the largest label, smallest index
 *      on ties
 *   x  id of the last edge (Y, X) of an optimal path: the delivery to X at T
 *      carrying its label, from the smallest such Y
 *   Y  the other end of x (the vertex before X)
 *   F2 M - Label(X), the total weight of that path
 *   No path is not an error: CSP_OK with T = X = x = Y = F2 = -1.
 *
 * Counters (optional output): C cycles (distinct delivery times), U label
 * improvements (A counted once at time 0), D neighbour tests, E flows sent,
 * R flows delivered, P peak flows in transit after a sending round, I
 * largest improved set of one cycle.
 *
 * Errors: every entry point returns CSP_OK or a negative code and leaves
 * outputs unspecified on error.  The library never frees caller memory.
 * A context is used by one host thread at a time.
 */
#ifndef CSP_H
#define CSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CSP_MAX_M 0x0FFFFFFFu

enum {
    CSP_OK = 0,
    CSP_EINVAL = -1,     /* bad size, mask, edge value or M */
    CSP_ENOMEM = -2,     /* device allocation failed */
    CSP_EDEVICE = -3,    /* a HIP call failed */
    CSP_EOVERFLOW = -4,  /* transit pool still too small after retries */
    CSP_ECANCELED = -5   /* cycle cap reached before the run ended */
};

typedef struct { int64_t T, X, x, Y, F2; } csp_result;
typedef struct { int64_t C, U, D, E, R, P, I; } csp_counters;

typedef struct csp_ctx csp_ctx;

/* Create a context on HIP device `device`.  The context owns its device
 * scratch (labels, frontier queues, the transit pool) and grows it on
 * demand; it owns no caller buffer. */
int csp_create(int device, csp_ctx **out);
void csp_destroy(csp_ctx *ctx);

/* Error text of the last failing call on ctx (static storage). */
const char *csp_last_error(const csp_ctx *ctx);

/* One solve (sections 4-6, Algorithm 1) on device-resident inputs.
 * f1, f2, A, B are device pointers laid out as above; labels (nullable) is
 * a device uint32 [N] output.  Work is enqueued on `stream` (a hipStream_t,
 * NULL = default stream); the call returns after the result has been copied
 * back, so *out (and *cnt, nullable) are valid on return.
 * max_cycles <= 0 means no cap; otherwise CSP_ECANCELED when it is hit. */
int csp_solve_dev(csp_ctx *ctx, int d, int64_t n,
                  const uint8_t *f1, const uint8_t *f2,
                  const uint8_t *A, const uint8_t *B, uint32_t M,
                  uint32_t *labels, csp_result *out, csp_counters *cnt,
                  int64_t max_cycles, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve, arguments, results and errors as csp_solve_dev, with no device
 * allocation in the call.  All device state of the solve (edge records,
 * frontier lists, candidates, the wheel of flows in transit) lives in one
 * static array of CSP_SCRATCH_BYTES on each GPU, set up by csp_create and
 * held until the process ends; the barrier and result block are the
 * context's.  Every call on a GPU shares that array, so calls that overlap
 * on one GPU race.  Runs only the range-owned kernel.  Errors besides those
 * of csp_solve_dev: CSP_EINVAL when a range of the lattice does not fit in
 * LDS, when the lattice's records, lists and candidates leave the wheel
 * less than 16 flows per bucket of every range, or when a cycle trace is
 * set; CSP_EOVERFLOW when the flows in transit overflow the wheel carved
 * from the array (there is no retry with a larger one); CSP_EDEVICE when
 * the device has no copy of the array. */
#define CSP_SCRATCH_BYTES (256ull << 20)
int csp_solve_dev_noalloc(csp_ctx *ctx, int d, int64_t n,
                          const uint8_t *f1, const uint8_t *f2,
                          const uint8_t *A, const uint8_t *B, uint32_t M,
                          uint32_t *labels, csp_result *out, csp_counters *cnt,
                          int64_t max_cycles, void *stream);

/* Same on host buffers: copies inputs to the device of ctx, solves, copies
 * labels (nullable host uint32 [N]) back.  Synchronous. */
int csp_solve(csp_ctx *ctx, int d, int64_t n,
              const uint8_t *f1, const uint8_t *f2,
              const uint8_t *A, const uint8_t *B, uint32_t M,
              uint32_t *labels, csp_result *out, csp_counters *cnt);

/* Path recovery by repeated solves (section 1; section 5, "Termination"):
 * after (T, X, x = (Y, X), F2), solve again with the same A, B' = {Y} and
 * M' = F2 - f2(x) + 1; that solve ends at Y at time T - f1(x) with weight
 * F2 - f2(x) and names the vertex before Y.  Repeat until it is in A.
 * path (host int64 [cap]) receives the vertices from the A end to X and
 * *len their number; CSP_EINVAL with *len set when cap is too small.  No
 * path gives *len = 0.  Inputs are device pointers as for csp_solve_dev.
 * `scratch_mask` is a caller-owned device uint8 [N] used for B'; it must be
 * all zero on entry and is all zero again on return. */
int csp_reconstruct_dev(csp_ctx *ctx, int d, int64_t n,
                        const uint8_t *f1, const uint8_t *f2,
                        const uint8_t *A, const uint8_t *B, uint32_t M,
                        uint8_t *scratch_mask,
                        int64_t *path, int64_t cap, int64_t *len,
                        csp_result *out, void *stream);

/* Same on host buffers (inputs as for csp_solve; the B' mask lives in ctx).
 * Synchronous. */
int csp_reconstruct(csp_ctx *ctx, int d, int64_t n,
                    const uint8_t *f1, const uint8_t *f2,
                    const uint8_t *A, const uint8_t *B, uint32_t M,
                    int64_t *path, int64_t cap, int64_t *len, csp_result *out);

/* The same cycle on a general graph (section 1 states the problem for any
 * graph with positive integer f1, f2; the lattice is the case the paper
 * studies).  Device arrays: off int64 [nv+1] and, for each directed
 * adjacency entry j (both directions of every edge present, neighbours of
 * a vertex in ascending order), nbr int32 [m], f1 and f2 uint8 [m] (1..255),
 * eid int64 [m] (the edge id reported as x; equal on the two copies of an
 * edge); A, B uint8 [nv]; labels uint32 [nv] (nullable).  m = off[nv].
 * Results, counters and errors as for csp_solve_dev; x is eid of the last
 * edge.  CSP_EINVAL also when off is not non-decreasing within [0, m] or a
 * neighbour index lies outside [0, nv) (checked on the device before any
 * cycle runs).  Labels live in HBM (no LDS ranges). */
int csp_solve_graph_dev(csp_ctx *ctx, int64_t nv, const int64_t *off,
                        const int32_t *nbr, const uint8_t *f1, const uint8_t *f2,
                        const int64_t *eid, const uint8_t *A, const uint8_t *B,
                        uint32_t M, uint32_t *labels, csp_result *out,
                        csp_counters *cnt, int64_t max_cycles, void *stream);

/* Path recovery with memory instead of re-solves (the trade-off section 1
 * sets aside for memory): one solve that logs every label improvement
 * (vertex, t, label and the improvement record of the sender of the best
 * delivery, ties to the smallest sender), then a walk from X's record back
 * to A.  The path, result and counters are identical to csp_reconstruct_dev
 * and csp_solve_dev; path (host, cap entries) receives the vertices A -> X
 * and *len their count (cap too small: CSP_EINVAL with *len set).  Extra
 * device memory: 16 bytes per label improvement (U), 12 bytes per vertex,
 * 4 bytes per wheel and candidate slot; it grows and retries like the
 * wheel.  Needs the range-owned kernel (csp_set_path 0, 1 or 3).
 * Synchronous on `stream`. */
int csp_reconstruct_log_dev(csp_ctx *ctx, int d, int64_t n,
                            const uint8_t *f1, const uint8_t *f2,
                            const uint8_t *A, const uint8_t *B, uint32_t M,
                            int64_t *path, int64_t cap, int64_t *len,
                            csp_result *out, csp_counters *cnt, void *stream);

/* One problem of a batch: device pointers laid out as for csp_solve_dev.
 * labels (nullable) is a device uint32 [n^d] output. */
typedef struct {
    int d;
    int64_t n;
    const uint8_t *f1, *f2, *A, *B;
    uint32_t M;
    uint32_t *labels;
} csp_problem;

/* Many independent solves (sections 4-6, Algorithm 1 for each) in one
 * persistent launch per dimension.  Workgroups take (problem, range) work
 * items, largest problems first; a problem whose lattice does not fit one
 * workgroup's LDS runs on a gang of workgroups that synchronise only among
 * themselves.  Results (and counters, nullable) are written per problem in
 * input order, identical to csp_solve_dev on each problem alone.  Returns
 * the first error; problems whose wheel overflows are re-run with larger
 * pools automatically, and ctx remembers those sizes for the same problem
 * (shape, M and input pointers) in later batches.  Synchronous on `stream`. */
int csp_solve_batch(csp_ctx *ctx, int count, const csp_problem *probs,
                    csp_result *out, csp_counters *cnt, void *stream);

/* Gang size of later batches on ctx: a problem of N vertices runs on about
 * N / vertices_per_workgroup workgroups (more when its ranges would not fit
 * LDS, fewer when neighbouring ranges would lie too far apart); 0, the
 * default, gives every problem the fewest workgroups whose ranges fit LDS.
 * Changes speed, never results. */
int csp_set_batch_target(csp_ctx *ctx, int64_t vertices_per_workgroup);

/* Autotuning of the batch: runs csp_solve_batch on the given problems with
 * vertices_per_workgroup = 0, 65536, 32768, 16384 and 8192, checks that
 * every run gives the same results and counters (else CSP_EDEVICE), and
 * sets the fastest by kernel time (0 unless another is at least 3 % faster)
 * as ctx's batch target.  target and ms (nullable) receive the choice and
 * its kernel time in milliseconds.  csp_autotune_clear resets it to 0. */
int csp_autotune_batch(csp_ctx *ctx, int count, const csp_problem *probs, int64_t *target, float *ms,
                       void *stream);

/* Device time (ms, from HIP events on the solve stream) of the cycle kernel
 * of the last successful solve on ctx (csp_solve_dev, csp_solve,
 * csp_solve_graph_dev; for csp_solve_batch the sum over its launches and
 * retry rounds); excludes input checks and result copies. */
int csp_last_kernel_ms(const csp_ctx *ctx, float *ms);

/* Starting capacity of each timing-wheel bucket, in flows (0 = automatic).
 * A run that overflows a bucket is repeated with twice the capacity, so
 * this changes speed and memory, never results. */
int csp_set_pool_hint(csp_ctx *ctx, uint64_t flows_per_bucket);

/* Workgroups of the cycle kernel for later solves on ctx (0 = automatic;
 * clamped to what the device can keep resident at once).  Changes speed,
 * never results. */
int csp_set_blocks(csp_ctx *ctx, int blocks);

/* Kernel choice for later solves on ctx: 0 = automatic, 1 = range-owned
 * (each workgroup keeps a range of consecutive vertex indices, with their
 * labels in LDS; CSP_EINVAL when a range cannot fit), 2 = global labels,
 * 3 = range-owned with x-pencil ranges for d = 3 (n x t x t vertices; other
 * d as 1).  Automatic: the autotuned choice for the lattice shape, else
 * x-pencils for 3-d lattices of 2^23 vertices or more, else range-owned
 * when a range fits in LDS, else global labels.  Changes speed, never
 * results.  csp_last_path returns the kernel (1 range-owned, 2 global
 * labels) the last solve used. */
int csp_set_path(csp_ctx *ctx, int path);
int csp_last_path(const csp_ctx *ctx);

/* Autotuning of the single-solve kernel for one lattice shape.  Solves the
 * problem (arguments as csp_solve_dev) twice per candidate configuration:
 * workgroup counts of 1/4, 1/2, 1 and 2 times the automatic choice, and for
 * d = 3 both range shapes and the global-label kernel (csp_set_path 1, 3
 * and 2).  Every configuration must
 * give the same result and counters (else CSP_EDEVICE).  The fastest, by
 * kernel time (the automatic configuration unless another is at least 3 %
 * faster), is recorded on ctx and used by later csp_solve_dev,
 * csp_solve and reconstruction calls whose lattice has the same d and n^d,
 * unless csp_set_blocks or csp_set_path set an override.  blocks, path and
 * ms (nullable) receive the choice and its kernel time in milliseconds.
 * Tuning changes speed only, never results.  csp_autotune_clear drops every
 * recorded choice (and resets the batch target, see csp_autotune_batch, and
 * the batch sizes remembered per problem, see csp_solve_batch). */
int csp_autotune(csp_ctx *ctx, int d, int64_t n, const uint8_t *f1, const uint8_t *f2, const uint8_t *A,
                 const uint8_t *B, uint32_t M, int *blocks, int *path, float *ms, void *stream);
int csp_autotune_clear(csp_ctx *ctx);

/* Limit on every barrier and neighbour wait of the single-solve entry points
 * (csp_solve, csp_solve_dev, csp_solve_dev_noalloc, csp_solve_graph_dev, the
 * reconstructions and csp_autotune) for later calls on ctx, in
 * microseconds: a wait longer than this marks the run broken, every
 * workgroup leaves the kernel, and the call fails with CSP_EDEVICE.  -1
 * restores the default (20 s).  A limit far below a cycle's length makes
 * every solve with more than one workgroup fail; it exists so that the
 * failure path can be exercised.  Batches and the server keep their own
 * limit (60 s). */
int csp_set_wait_limit(csp_ctx *ctx, int64_t microseconds);

/* Dense/sparse form of the improved set I_t (section 6, Step 8 condenses
 * the triggered vertices into one list).  Each workgroup of the
 * range-owned kernel collects the vertices of its range whose label rose
 * at t.  Before its deliveries of a cycle it chooses the form from the
 * number of flows it is about to deliver: up to `flows`, an unordered list
 * appended during the deliveries (sparse form); above, the deliveries only
 * mark an improved-vertex bitmap, which a sweep then packs into a list in
 * vertex order (dense form).  0 takes the dense form every cycle; a value
 * of 2^32 - 1 or more never; -1 (the default) restores the automatic
 * choice (the autotuned value for the lattice shape, else 4096 for ranges
 * of 32,768 vertices or more and never for smaller ones).
 * Changes speed, never results.  csp_autotune tries, on the configuration
 * it chose, the thresholds never, 0, 2048, 4096, 8192 and 16384 and
 * records the fastest (when at least 3 % faster than the automatic one);
 * csp_tuned_dense_threshold reports what it recorded for a shape (-1:
 * nothing, the automatic choice applies). */
int csp_set_dense_threshold(csp_ctx *ctx, int64_t flows);
int csp_tuned_dense_threshold(const csp_ctx *ctx, int d, int64_t n, int64_t *flows);

/* Cycle trace for later csp_solve_dev calls on ctx (off when cap = 0):
 * trace is a device buffer of cap rows of four int64, one row per time at
 * which water is delivered (section 4, Algorithm 1's loop): t, flows
 * delivered at t, |I_t| (vertices whose label improved at t), flows sent
 * from I_t.  The last row's "sent" is 0 (the run ends before sending).
 * Rows beyond cap are counted but not written; csp_last_trace_rows gives
 * the count of the last successful solve.  The trace needs the
 * range-owned kernel (csp_set_path 0, 1 or 3); a solve that would take the
 * global-label kernel returns CSP_EINVAL. */
int csp_set_trace(csp_ctx *ctx, int64_t *trace, int64_t cap);
int csp_last_trace_rows(const csp_ctx *ctx, int64_t *rows);

/* Phase timing of the cycle kernel (off by default; on = 1 or 2).  When on, workgroup 0
 * accumulates wall-clock time per phase; csp_last_phase_us fills us[6] with
 * microseconds spent in: departure work, the barrier after it, finding the
 * next time, arrival work, the barrier after it, and the frontier gather,
 * for the last successful solve.  The general-graph solve fills the same
 * slots (finding the next time is part of its barrier, so that slot is 0;
 * the last slot is the listing of each chunk's improved vertices). */
int csp_set_phase_timing(csp_ctx *ctx, int on);
int csp_last_phase_us(const csp_ctx *ctx, double *us);

/* Phase timing over every workgroup of the range-owned kernel: with
 * csp_set_phase_timing(ctx, 2) each workgroup times its own phases, and
 * after a solve mean[6] and max[6] receive, per phase, the mean over the
 * workgroups and the largest single workgroup's total, in microseconds:
 * slot 0 the sending step (Steps 4-5 inside the range), 1 arriving at
 * the barrier (completing the workgroup's accesses, counting in, and the
 * release for the last to arrive), 2 waiting for the neighbouring ranges'
 * arrival and testing the candidates they shipped (before the release),
 * 4 waiting for the barrier's release, 3 the deliveries (Steps 1-3, 8) and
 * building I_t.  Zero when the last solve took the global-label kernel. */
int csp_last_phase_spread(const csp_ctx *ctx, double *mean, double *max);

/* Micro-benchmarks of the device resources the cycle is bound by (no
 * solve; timed with HIP events on `stream`; buffers from the context).
 *   kind 0: copy p0 bytes (a multiple of 16) device to device, p1 times;
 *           r[0] = GB/s of bytes read plus bytes written.
 *   kind 1: p0 32-bit atomic maxima at hashed positions of p1 words (a power
 *           of two); r[0] = G atomics/s.
 *   kind 2: one workgroup per CU, each doing p0 16-byte loads at hashed
 *           positions of its own slab of 2^p2 records (p2 in 10..18; 0 means
 *           16, a 1 MiB slab) per round, p1 rounds (the edge record fetches
 *           of the sending step); r[0] = G loads/s, r[1] = us per round.
 *   kind 3: p0 barriers among p1 (2..CUs) workgroups of a cooperative launch:
 *           r[0] = us per barrier of the cycle loop's kind; r[1] = us per
 *           fully fenced barrier after every member wrote p2 KiB with plain
 *           stores.  Each barrier's combined minimum is checked (CSP_EDEVICE
 *           if one is wrong).
 * CSP_EINVAL for an unknown kind or sizes out of range. */
int csp_microbench(csp_ctx *ctx, int kind, int64_t p0, int64_t p1, int64_t p2, double *r, void *stream);

/* ---- Serving: continuous batching of solves and reconstructions --------
 *
 * A server runs one persistent kernel whose workers (one workgroup per CU)
 * keep taking work while it runs: requests submitted while others are on
 * the GPU are admitted as soon as job slots, workers and arena memory free
 * up, in submission order, and run beside them.  A request is one solve
 * (sections 4-6) and, when asked, the path reconstruction of section 1 and
 * section 5 "Termination"
 * (repeated solves with B' = {Y}, M' = F2 - f2(x) + 1 until Y is in A),
 * carried out by the same workers on device-resident state.  Results are
 * identical to csp_solve_dev / csp_reconstruct_dev on the request alone.
 *
 * The server owns an HBM arena of `arena_bytes` for per-request state
 * (packed edges, frontier lists, timing wheel, candidate buffers); a
 * request's footprint is about 20 bytes per vertex plus 8 bytes per wheel
 * flow (6 d N flows to start, doubled on overflow).  Admission waits until
 * the footprint fits.  The caller keeps a request's f1, f2, A, B (device
 * memory) valid and unchanged until its completion is returned, and makes
 * sure they are complete on the device before submitting (the workers read
 * them from their own stream).
 *
 * Progress is made inside csp_serve_submit and csp_serve_poll; call poll
 * regularly.  The workers are one cooperative launch, so all of them are
 * resident before any takes work (a request's gang of workers waits for
 * its members at a barrier).  When the server has nothing to do the workers
 * leave, so the GPU is free for other kernels; the next admitted request
 * starts them again, and their launch waits for the CUs other kernels hold.
 * If the host stops polling for 2 s the workers leave once every published
 * slot has been taken.  A request whose gang barrier timed out completes
 * with CSP_EDEVICE and its job slot is cleared for reuse.  One host thread
 * uses a server at a time. */
typedef struct csp_server csp_server;

typedef struct {
    int d;
    int64_t n;
    const uint8_t *f1, *f2, *A, *B;   /* device pointers, as for csp_solve_dev */
    uint32_t M;
    int reconstruct;                  /* nonzero: also the path A -> X */
    uint64_t tag;                     /* returned unchanged in the completion */
} csp_request;

typedef struct {
    uint64_t tag;
    int status;                       /* CSP_OK or this request's error */
    csp_result res;                   /* as from csp_solve_dev */
    csp_counters cnt;                 /* the first solve */
    csp_counters cnt_chain;           /* the reconstruction re-solves: U, D, E, R
                                         summed; C, P, I of the last one */
    int64_t solves;                   /* 1 + re-solves */
    int64_t path_len;                 /* vertices of the path A -> X (0 if none
                                         or not asked for) */
    const int64_t *path;              /* owned by the server; valid until the
                                         next csp_serve_poll or csp_serve_close */
} csp_completion;

/* Create a server on ctx's device with an arena of arena_bytes (>= 1 MiB)
 * and at most max_jobs (1..4096) requests on the GPU at once. */
int csp_serve_open(csp_ctx *ctx, uint64_t arena_bytes, int max_jobs, csp_server **out);

/* Queue a request.  CSP_EINVAL for bad shapes or null pointers, CSP_ENOMEM
 * when it could never fit the arena.  Errors found on the device (a zero
 * edge, A and B not disjoint) come back in the completion's status. */
int csp_serve_submit(csp_server *s, const csp_request *req);

/* Collect up to cap completions (in completion order) into out; *count
 * gets how many.  Never blocks. */
int csp_serve_poll(csp_server *s, csp_completion *out, int cap, int *count);

/* Requests waiting for admission or collection, and requests on the GPU. */
int csp_serve_pending(const csp_server *s, int *queued, int *running);

/* Finish the requests on the GPU, stop the workers and free the server.
 * Requests not yet admitted are dropped. */
int csp_serve_close(csp_server *s);

#ifdef __cplusplus
}
#endif

#endif /* CSP_H */
