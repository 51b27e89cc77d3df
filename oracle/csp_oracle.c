/*
 * csp_oracle.c -- CPU oracle for the water-flow constrained-shortest-path
 * method of I. Matic, "A parallel algorithm for the constrained shortest path
 * problem on lattice graphs" (arXiv:1511.06441).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header or table with the HIP path.
 *
 * It is a plain, single-threaded, cycle-by-cycle simulation written for
 * readability, not speed:
 *
 *   Problem (section 1): undirected graph, every edge e has a passage time
 *   f1(e) and a weight f2(e), both positive integers.  Among paths from A to
 *   B (disjoint) find the least total time F1 subject to total weight F2 < M.
 *
 *   Water model (section 1): A holds water of quality M, every other vertex
 *   quality 0.  Crossing e takes f1(e) time units and costs f2(e) quality;
 *   water of quality 0 does not move.  Label(P) is the best quality that has
 *   reached P.  The first time a vertex of B receives water is the answer.
 *
 * Each unit of water in transit over an edge is a "flow" (destination,
 * quality, source, arrival time).  The paper's regular active edges and its
 * phantom edges (sections 1 and 6, Steps 3 and 5) are both flows here: a
 * phantom is nothing but a second flow on the same edge carrying better
 * water.  The cycle below is section 6's Steps 1-9 in order:
 *
 *   Step 1   m = least remaining time of all flows in transit; Time += m;
 *            flows whose time runs out are delivered ("just used").
 *   Step 2/3 TempLabel(Q) = best quality delivered to Q this cycle (regular
 *            and phantom alike), ties to the smallest source vertex.
 *   Step 8   Q whose TempLabel beats Label(Q) takes it (Label keeps the best
 *            water ever received; this is the improved set I_t).
 *   Step 6   if some vertex of B improved, stop: Time is the answer.
 *   Step 4/5 every improved Q sends water over each edge (Q,P) whose
 *            far end would be improved: Label(Q) - f2 > Label(P).  The new
 *            flow arrives at Time + f1(Q,P).
 *   Step 7/9 delivered flows are removed (they leave their bucket).
 *
 * Readings taken where the text is loose (all listed in the design notes):
 * the constraint is strict (F2 < M, so a label >= 1 is needed to move);
 * termination reports the cycle in which B's label first becomes positive;
 * the departure test uses labels after this cycle's deliveries; the old flow
 * on an edge whose source is relabelled stays in transit (it is delivered
 * and rejected later); the minimum in Step 1 runs over phantoms as well.
 *
 * Output (section 1 and section 5 "Termination"): T = F1 of the optimum,
 * X in B its endpoint (largest label, ties to the smallest index), the last
 * edge x = (Y, X) (the delivering flow; ties to the smallest Y), and
 * F2 = M - Label(X).  No path: T = X = x = Y = F2 = -1.  Final labels are
 * L_T(v) for every v (L_infinity when there is no path).
 *
 * Counters (not in the paper, used for throughput figures):
 *   C  cycles executed (distinct delivery times)
 *   U  label improvements, including A at time 0
 *   D  neighbour tests made while sending water
 *   E  flows sent
 *   R  flows delivered
 *   P  peak number of flows in transit right after a sending round
 *   I  largest improved set of one cycle
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

/* f1 <= 255, so a flow sent at t arrives before t + 256: a circular array of
 * 256 buckets indexed by arrival time holds every flow in transit. */
#define NB 256

typedef struct {
    int32_t dst;
    int32_t src;
    int64_t q;    /* quality carried on arrival */
    int64_t adj;  /* adjacency entry (in src's list) the flow travels on */
} flow_t;

typedef struct {
    flow_t *v;
    int64_t n, cap;
} bucket_t;

static int bucket_push(bucket_t *b, flow_t f)
{
    if (b->n == b->cap) {
        int64_t nc = b->cap ? 2 * b->cap : 64;
        flow_t *nv = (flow_t *)realloc(b->v, (size_t)nc * sizeof(flow_t));
        if (!nv) return ORC_ENOMEM;
        b->v = nv;
        b->cap = nc;
    }
    b->v[b->n++] = f;
    return ORC_OK;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * Build the nearest-neighbour lattice on n^d vertices as adjacency lists.
 * Vertex v = sum_k c_k n^k.  Edge (k, u) joins u and u + n^k and has id
 * k*N + u; its times are f1[k*N+u], f2[k*N+u].  Each vertex lists its
 * neighbours in ascending index order: v - n^(d-1), ..., v - 1, v + 1, ...,
 * v + n^(d-1).
 *
 * off has N+1 entries; nbr, a1, a2, eid have off[N] entries.  Passing
 * nbr == NULL only fills off (to size the other arrays).
 */
int orc_lattice_adjacency(int d, int64_t n, const uint8_t *f1, const uint8_t *f2,
                          int64_t *off, int32_t *nbr, uint8_t *a1, uint8_t *a2, int64_t *eid)
{
    if (d < 1 || d > 4 || n < 2) return ORC_EINVAL;
    int64_t N = 1, stride[4];
    for (int k = 0; k < d; ++k) { stride[k] = N; N *= n; }
    if (N > INT32_MAX) return ORC_EINVAL;
    int64_t pos = 0;
    for (int64_t v = 0; v < N; ++v) {
        off[v] = pos;
        for (int k = d - 1; k >= 0; --k) {          /* lower neighbours, far axes first */
            int64_t c = (v / stride[k]) % n;
            if (c >= 1) {
                int64_t u = v - stride[k];
                if (nbr) {
                    nbr[pos] = (int32_t)u;
                    a1[pos] = f1[k * N + u];
                    a2[pos] = f2[k * N + u];
                    eid[pos] = k * N + u;
                }
                ++pos;
            }
        }
        for (int k = 0; k < d; ++k) {               /* upper neighbours, near axes first */
            int64_t c = (v / stride[k]) % n;
            if (c <= n - 2) {
                if (nbr) {
                    nbr[pos] = (int32_t)(v + stride[k]);
                    a1[pos] = f1[k * N + v];
                    a2[pos] = f2[k * N + v];
                    eid[pos] = k * N + v;
                }
                ++pos;
            }
        }
    }
    off[N] = pos;
    return ORC_OK;
}

/*
 * The cycle on a general graph given as adjacency lists (neighbours of each
 * vertex in ascending order, both directions of every edge present, with
 * equal f1, f2 and edge id on the two copies).
 *
 *   label   out, nv entries (may be NULL)
 *   res     out, {T, X, x, Y, F2}
 *   cnt     out, {C, U, D, E, R, P, I} (may be NULL)
 *   trace   out, up to trace_cap rows {t, delivered, |I_t|, sent} (may be NULL)
 *   max_cycles  stop after this many cycles (<= 0: no limit); res[0] = -2 then
 */
int orc_solve_graph(int64_t nv, const int64_t *off, const int32_t *nbr,
                    const uint8_t *a1, const uint8_t *a2, const int64_t *eid,
                    const uint8_t *A, const uint8_t *B, int64_t M,
                    uint32_t *label_out, int64_t *res, int64_t *cnt,
                    int64_t *trace, int64_t trace_cap, int64_t *trace_len,
                    int64_t max_cycles)
{
    if (nv < 1 || M < 1 || M > UINT32_MAX) return ORC_EINVAL;
    for (int64_t v = 0; v < nv; ++v) {
        if (A[v] && B[v]) return ORC_EINVAL;                    /* A, B disjoint */
        for (int64_t j = off[v]; j < off[v + 1]; ++j)
            if (a1[j] == 0 || a2[j] == 0) return ORC_EINVAL;    /* positive f */
    }

    int rc = ORC_ENOMEM;
    int64_t *L = (int64_t *)malloc((size_t)nv * sizeof(int64_t));       /* Label */
    int64_t *tq = (int64_t *)calloc((size_t)nv, sizeof(int64_t));       /* TempLabel */
    int32_t *tsrc = (int32_t *)malloc((size_t)nv * sizeof(int32_t));
    int64_t *tadj = (int64_t *)malloc((size_t)nv * sizeof(int64_t));
    int32_t *trig = (int32_t *)malloc((size_t)nv * sizeof(int32_t));   /* triggered */
    int32_t *I = (int32_t *)malloc((size_t)nv * sizeof(int32_t));      /* improved set */
    bucket_t *bk = (bucket_t *)calloc(NB, sizeof(bucket_t));
    if (!L || !tq || !tsrc || !tadj || !trig || !I || !bk) goto done;

    int64_t C = 0, U = 0, D = 0, E = 0, R = 0, peak = 0, maxI = 0;
    int64_t in_transit = 0, ntrace = 0;
    int64_t T = -1, X = -1, xe = -1, Y = -1, F2 = -1;

    /* Initialization (Algorithm 3): Label = M on A and 0 elsewhere, Time = 0.
     * The vertices of A are the first improved set. */
    int64_t nI = 0;
    for (int64_t v = 0; v < nv; ++v) {
        L[v] = A[v] ? M : 0;
        if (A[v]) I[nI++] = (int32_t)v;
    }
    U += nI;
    int64_t t = 0;

    for (;;) {
        /* Steps 4-5 (Algorithms 7, 8): every improved Q sends its water over
         * each edge whose far end it would improve.  A Q that already had
         * water in transit simply gets another flow (the paper's phantom). */
        int64_t sent = 0;
        for (int64_t i = 0; i < nI; ++i) {
            int32_t Q = I[i];
            for (int64_t j = off[Q]; j < off[Q + 1]; ++j) {
                int32_t P = nbr[j];
                ++D;
                int64_t q = L[Q] - (int64_t)a2[j];
                if (q > L[P]) {
                    flow_t f = {P, Q, q, j};
                    if (bucket_push(&bk[(t + a1[j]) % NB], f)) goto done;
                    ++sent;
                }
            }
        }
        E += sent;
        in_transit += sent;
        if (in_transit > peak) peak = in_transit;
        if (trace && ntrace > 0 && ntrace <= trace_cap) trace[4 * (ntrace - 1) + 3] = sent;

        /* Terminal condition 2 (section 5, Algorithm 2): nothing in transit. */
        if (in_transit == 0) break;
        if (max_cycles > 0 && C >= max_cycles) { T = -2; break; }

        /* Step 1 (Algorithm 4, with Step 3's phantoms): advance Time by the
         * least remaining time of all flows in transit. */
        int64_t m = 1;
        while (bk[(t + m) % NB].n == 0) ++m;
        t += m;
        ++C;

        /* Steps 1-3 (Algorithms 4, 5, 6): deliver every flow whose time ran
         * out; TempLabel(Q) = best delivered quality, ties to the smallest
         * source. */
        bucket_t *b = &bk[t % NB];
        int64_t ntrig = 0;
        for (int64_t i = 0; i < b->n; ++i) {
            flow_t *f = &b->v[i];
            if (tq[f->dst] == 0) trig[ntrig++] = f->dst;
            if (f->q > tq[f->dst] || (f->q == tq[f->dst] && f->src < tsrc[f->dst])) {
                tq[f->dst] = f->q;
                tsrc[f->dst] = f->src;
                tadj[f->dst] = f->adj;
            }
        }
        R += b->n;
        in_transit -= b->n;
        int64_t delivered = b->n;
        b->n = 0;                                   /* Steps 7, 9: delivered flows leave */

        /* Step 8 (Algorithm 10): triggered vertices whose TempLabel beats the
         * label take it; they form the improved set I_t (ascending). */
        qsort(trig, (size_t)ntrig, sizeof(int32_t), cmp_i32);
        nI = 0;
        for (int64_t i = 0; i < ntrig; ++i) {
            int32_t Q = trig[i];
            if (tq[Q] > L[Q]) {
                L[Q] = tq[Q];
                I[nI++] = Q;
            }
        }
        U += nI;
        if (nI > maxI) maxI = nI;
        if (trace && ntrace < trace_cap) {
            trace[4 * ntrace + 0] = t;
            trace[4 * ntrace + 1] = delivered;
            trace[4 * ntrace + 2] = nI;
            trace[4 * ntrace + 3] = 0;
        }
        ++ntrace;

        /* Step 6 / terminal condition 1 (section 5, Algorithm 2): a vertex of
         * B has received water.  X = best label among them, smallest index
         * on ties; x is the edge its best water came over. */
        for (int64_t i = 0; i < nI; ++i) {
            int32_t Q = I[i];
            if (B[Q] && (X < 0 || L[Q] > L[X])) X = Q;
        }
        if (X >= 0) {
            T = t;
            Y = tsrc[X];
            xe = eid[tadj[X]];
            F2 = M - L[X];
        }
        for (int64_t i = 0; i < ntrig; ++i) tq[trig[i]] = 0;   /* TempLabel cleared */
        if (X >= 0) break;
    }

    if (T < 0) { X = xe = Y = F2 = -1; }
    res[0] = T; res[1] = X; res[2] = xe; res[3] = Y; res[4] = F2;
    if (cnt) {
        cnt[0] = C; cnt[1] = U; cnt[2] = D; cnt[3] = E;
        cnt[4] = R; cnt[5] = peak; cnt[6] = maxI;
    }
    if (trace_len) *trace_len = ntrace;
    if (label_out)
        for (int64_t v = 0; v < nv; ++v) label_out[v] = (uint32_t)L[v];
    rc = ORC_OK;

done:
    if (bk) {
        for (int i = 0; i < NB; ++i) free(bk[i].v);
        free(bk);
    }
    free(L); free(tq); free(tsrc); free(tadj); free(trig); free(I);
    return rc;
}

/* Adjacency of an n^d lattice, allocated here; freed by orc_adj_free. */
typedef struct {
    int64_t nv;
    int64_t *off;
    int32_t *nbr;
    uint8_t *a1, *a2;
    int64_t *eid;
} orc_adj;

static void orc_adj_free(orc_adj *g)
{
    free(g->off); free(g->nbr); free(g->a1); free(g->a2); free(g->eid);
    memset(g, 0, sizeof(*g));
}

static int orc_adj_build(int d, int64_t n, const uint8_t *f1, const uint8_t *f2, orc_adj *g)
{
    memset(g, 0, sizeof(*g));
    if (d < 1 || d > 4 || n < 2) return ORC_EINVAL;
    int64_t N = 1;
    for (int k = 0; k < d; ++k) {
        N *= n;
        if (N > INT32_MAX) return ORC_EINVAL;
    }
    g->nv = N;
    g->off = (int64_t *)malloc((size_t)(N + 1) * sizeof(int64_t));
    if (!g->off) return ORC_ENOMEM;
    int rc = orc_lattice_adjacency(d, n, f1, f2, g->off, NULL, NULL, NULL, NULL);
    if (rc) { orc_adj_free(g); return rc; }
    int64_t m = g->off[N];
    g->nbr = (int32_t *)malloc((size_t)(m ? m : 1) * sizeof(int32_t));
    g->a1 = (uint8_t *)malloc((size_t)(m ? m : 1));
    g->a2 = (uint8_t *)malloc((size_t)(m ? m : 1));
    g->eid = (int64_t *)malloc((size_t)(m ? m : 1) * sizeof(int64_t));
    if (!g->nbr || !g->a1 || !g->a2 || !g->eid) { orc_adj_free(g); return ORC_ENOMEM; }
    return orc_lattice_adjacency(d, n, f1, f2, g->off, g->nbr, g->a1, g->a2, g->eid);
}

/* The cycle on an n^d lattice with SoA edge arrays f1, f2 [d][n^d]. */
int orc_solve_lattice(int d, int64_t n, const uint8_t *f1, const uint8_t *f2,
                      const uint8_t *A, const uint8_t *B, int64_t M,
                      uint32_t *label_out, int64_t *res, int64_t *cnt,
                      int64_t *trace, int64_t trace_cap, int64_t *trace_len,
                      int64_t max_cycles)
{
    orc_adj g;
    int rc = orc_adj_build(d, n, f1, f2, &g);
    if (rc) return rc;
    rc = orc_solve_graph(g.nv, g.off, g.nbr, g.a1, g.a2, g.eid, A, B, M,
                         label_out, res, cnt, trace, trace_cap, trace_len, max_cycles);
    orc_adj_free(&g);
    return rc;
}

/*
 * Path recovery by repeated solves (section 1; section 5, "Termination"):
 * after a solve gives (T, X, x = (Y, X), F2), solve again with the same A,
 * B' = {Y} and M' = F2 - f2(x) + 1 (the text's M' with the strict
 * constraint F2 < M' made to admit weight exactly F2 - f2(x)).  That solve
 * ends at Y with time T - f1(x) and weight F2 - f2(x) and names the vertex
 * before Y.  Repeat until the named vertex is in A.
 *
 * path receives the vertices from the A end to X; *len is their number.
 * Returns ORC_EINVAL with *len set to the needed size if cap is too small.
 * steps (may be NULL) receives one {T, X, x, Y, F2} row per solve.
 *
 * max_steps > 0 stops the chain after that many rows (the first solve is
 * row 0): path then holds only the vertices found so far, ending at X, and
 * *complete is 0.  The chain's steps do not depend on where it stops, so a
 * stopped chain is a prefix of the whole one (used where the whole chain
 * would take hours on the host).
 */
static int reconstruct_graph_upto(int64_t nv, const int64_t *off, const int32_t *nbr,
                                  const uint8_t *a1, const uint8_t *a2, const int64_t *eid,
                                  const uint8_t *A, const uint8_t *B, int64_t M,
                                  int64_t *path, int64_t cap, int64_t *len, int64_t *res,
                                  int64_t *steps, int64_t steps_cap, int64_t max_steps,
                                  int64_t *complete)
{
    *complete = 1;
    int rc = orc_solve_graph(nv, off, nbr, a1, a2, eid, A, B, M, NULL, res,
                             NULL, NULL, 0, NULL, 0);
    if (rc) return rc;
    *len = 0;
    if (res[0] < 0) return ORC_OK;

    uint8_t *Bp = (uint8_t *)calloc((size_t)nv, 1);
    int64_t *rev = (int64_t *)malloc((size_t)(nv + 1) * sizeof(int64_t));
    if (!Bp || !rev) { free(Bp); free(rev); return ORC_ENOMEM; }

    int64_t cur[5];
    memcpy(cur, res, sizeof(cur));
    int64_t n_rev = 0, nsteps = 0;
    rev[n_rev++] = cur[1];                           /* X */
    for (;;) {
        if (steps && nsteps < steps_cap) memcpy(&steps[5 * nsteps], cur, sizeof(cur));
        ++nsteps;
        int64_t Xv = cur[1], Yv = cur[3], x = cur[2];
        rev[n_rev++] = Yv;
        if (A[Yv]) break;
        if (max_steps > 0 && nsteps >= max_steps) { *complete = 0; break; }
        /* f1, f2 of the last edge: the entry of X's list with edge id x */
        int64_t w2 = -1;
        for (int64_t j = off[Xv]; j < off[Xv + 1]; ++j)
            if (eid[j] == x && nbr[j] == Yv) w2 = a2[j];
        if (w2 < 0 || n_rev > nv) { rc = ORC_EINVAL; break; }
        Bp[Yv] = 1;
        int64_t nxt[5];
        rc = orc_solve_graph(nv, off, nbr, a1, a2, eid, A, Bp, cur[4] - w2 + 1,
                             NULL, nxt, NULL, NULL, 0, NULL, 0);
        Bp[Yv] = 0;
        if (rc) break;
        if (nxt[0] < 0 || nxt[1] != Yv) { rc = ORC_EINVAL; break; }
        memcpy(cur, nxt, sizeof(cur));
    }
    if (rc == ORC_OK) {
        *len = n_rev;
        if (n_rev > cap) rc = ORC_EINVAL;
        else
            for (int64_t i = 0; i < n_rev; ++i) path[i] = rev[n_rev - 1 - i];
    }
    free(Bp); free(rev);
    return rc;
}

int orc_reconstruct_graph(int64_t nv, const int64_t *off, const int32_t *nbr,
                          const uint8_t *a1, const uint8_t *a2, const int64_t *eid,
                          const uint8_t *A, const uint8_t *B, int64_t M,
                          int64_t *path, int64_t cap, int64_t *len, int64_t *res,
                          int64_t *steps, int64_t steps_cap)
{
    int64_t complete;
    return reconstruct_graph_upto(nv, off, nbr, a1, a2, eid, A, B, M, path, cap, len, res,
                                  steps, steps_cap, 0, &complete);
}

int orc_reconstruct_lattice_upto(int d, int64_t n, const uint8_t *f1, const uint8_t *f2,
                                 const uint8_t *A, const uint8_t *B, int64_t M,
                                 int64_t *path, int64_t cap, int64_t *len, int64_t *res,
                                 int64_t *steps, int64_t steps_cap, int64_t max_steps,
                                 int64_t *complete)
{
    orc_adj g;
    int rc = orc_adj_build(d, n, f1, f2, &g);
    if (rc) return rc;
    rc = reconstruct_graph_upto(g.nv, g.off, g.nbr, g.a1, g.a2, g.eid, A, B, M,
                                path, cap, len, res, steps, steps_cap, max_steps, complete);
    orc_adj_free(&g);
    return rc;
}

int orc_reconstruct_lattice(int d, int64_t n, const uint8_t *f1, const uint8_t *f2,
                            const uint8_t *A, const uint8_t *B, int64_t M,
                            int64_t *path, int64_t cap, int64_t *len, int64_t *res,
                            int64_t *steps, int64_t steps_cap)
{
    int64_t complete;
    return orc_reconstruct_lattice_upto(d, n, f1, f2, A, B, M, path, cap, len, res,
                                        steps, steps_cap, 0, &complete);
}
