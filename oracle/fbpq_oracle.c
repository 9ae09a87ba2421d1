/*
 * FBPQ oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow CPU implementation, in FP64, of the search that Fast Bilayer
 * Product Quantization accelerates: the Multi-D-ADC search over a second-order
 * inverted multi-index with PQ-encoded displacements (Babenko & Lempitsky,
 * "Improving Bilayer Product Quantization for Billion-Scale Approximate Nearest
 * Neighbors in High Dimensions", Section 2.3). The paper states that FBPQ visits
 * the same points in the same order and returns the same ranking as this
 * search (end of Section 3.1), so this is the definition the GPU path must match.
 * Every distance here is computed by reconstructing the displacement explicitly
 * (O(D) per candidate, Section 2.3.3), never through the FBPQ lookup tables.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library. It shares no code, header or table with the
 * GPU library and includes nothing from it.
 *
 * Readings where the paper is silent (each one is a choice of this oracle):
 *  - half distances are FP64 sums over t = 0..D/2-1 in that order, one
 *    correctly rounded fused multiply-add per coordinate: acc = fma(e, e, acc)
 *    with e = q[t] - c[t] computed in FP64;
 *  - a cell's traversal key is the FP64 sum d1[i] + d2[j]; cells are visited
 *    in ascending (key, a, b), a and b being ranks in the (distance, index)
 *    sorted half lists;
 *  - the candidate list holds exactly min(L, N) points: the last visited cell
 *    is cut in storage order; empty cells are visited and contribute nothing;
 *  - cell id = i*T + j; within a cell points keep their storage order;
 *  - results are ordered by (distance, id); missing entries are (-1, +inf);
 *  - subspace k of the PQ code covers coordinates [k*D/M, (k+1)*D/M).
 *
 * The same search with local codebooks (HBPQ, Section 3.2) takes, instead of
 * the global codebooks R, one set of M/2 codebooks per first-half centroid
 * (Q^i, coding the first half of a displacement in a cell of row i) and one
 * per second-half centroid (S^j, the second half in a cell of column j), as in
 * equation (residual); the traversal is unchanged and the distance is again
 * computed by explicit reconstruction.
 *
 * With optimized product quantization (OPQ, Section 2.1; the optimized
 * variants of Section 3.2) the index lives in a rotated space: a query q
 * enters it as q' = Rot q, Rot an orthogonal D x D matrix. Reading: each
 * coordinate of q' is the FP64 sum over b = 0..D-1 in that order, one fused
 * multiply-add per term, rounded once to FP32 (the search takes FP32 queries).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int D, T, M, Kc;
    int64_t N;
    const float *C1, *C2, *R;
    const int64_t *offsets;
    const uint8_t *codes;
    const uint32_t *ids;
    const float *QL, *SL; /* local codebooks [T][M/2][Kc][D/M] each, or NULL (global R) */
} orc_ix;

/* Squared distance from a query half to every half centroid (equations q1 and
 * q2, Section 2.3.1): d[i] = sum_t (q[t] - C[i][t])^2, t in increasing order. */
/* q' = Rot q for nq queries (OPQ): Rot row-major [D][D], Q and out [nq][D]. */
void orc_rotate(int D, const float *Rot, const float *Q, int64_t nq, float *out)
{
    for (int64_t r = 0; r < nq; ++r)
        for (int a = 0; a < D; ++a) {
            double acc = 0.0;
            for (int b = 0; b < D; ++b) acc = fma((double)Rot[(int64_t)a * D + b], (double)Q[r * D + b], acc);
            out[r * D + a] = (float)acc;
        }
}

void orc_half_dists(const float *qh, const float *Ch, int T, int h, double *d)
{
    for (int i = 0; i < T; ++i) {
        double acc = 0.0;
        for (int t = 0; t < h; ++t) {
            double e = (double)qh[t] - (double)Ch[(int64_t)i * h + t];
            acc = fma(e, e, acc);
        }
        d[i] = acc;
    }
}

/* Closest-codeword list of one half (Section 2.3.3): centroid indices sorted
 * by ascending distance, ties by ascending index. */
typedef struct { double d; int32_t i; } orc_di;
static int orc_cmp_di(const void *x, const void *y)
{
    const orc_di *a = (const orc_di *)x, *b = (const orc_di *)y;
    if (a->d < b->d) return -1;
    if (a->d > b->d) return 1;
    return (a->i > b->i) - (a->i < b->i);
}

/* Returns 0, or -1 when its scratch cannot be allocated (order untouched). */
int orc_rank(const double *d, int T, int32_t *order)
{
    orc_di *tmp = (orc_di *)malloc(sizeof(orc_di) * (size_t)(T > 0 ? T : 1));
    if (!tmp) return -1;
    for (int i = 0; i < T; ++i) { tmp[i].d = d[i]; tmp[i].i = i; }
    qsort(tmp, (size_t)T, sizeof(orc_di), orc_cmp_di);
    for (int i = 0; i < T; ++i) order[i] = tmp[i].i;
    free(tmp);
    return 0;
}

/* ---- multi-sequence traversal (Section 2.3.3) ----------------------------
 * A min-priority queue over cells (a, b) of the rank grid keyed by
 * (d1[u[a]] + d2[v[b]], a, b). It starts from (0, 0). After (a, b) is popped,
 * (a+1, b) is pushed once its other predecessor (a+1, b-1) has been popped
 * (or b = 0), and (a, b+1) once (a-1, b+1) has been popped (or a = 0). Since
 * the key grows along both grid directions, cells leave the queue in
 * ascending (key, a, b).
 * The popped cells always form a staircase (a cell enters the queue only
 * after both its predecessors left it, and the cells of one row leave it in
 * column order), so "was (a, b) popped" is b < width[a], width[a] being the
 * number of cells of row a popped so far: T counters per query instead of a
 * T x T flag array. */
typedef struct { double key; int32_t a, b; } orc_ent;

static int orc_less(const orc_ent *x, const orc_ent *y)
{
    if (x->key != y->key) return x->key < y->key;
    if (x->a != y->a) return x->a < y->a;
    return x->b < y->b;
}

typedef struct {
    orc_ent *h;
    int64_t n;
} orc_heap;

static void orc_push(orc_heap *hp, orc_ent e)
{
    int64_t i = hp->n++;
    hp->h[i] = e;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!orc_less(&hp->h[i], &hp->h[p])) break;
        orc_ent t = hp->h[i]; hp->h[i] = hp->h[p]; hp->h[p] = t;
        i = p;
    }
}

static orc_ent orc_pop(orc_heap *hp)
{
    orc_ent top = hp->h[0];
    hp->h[0] = hp->h[--hp->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < hp->n && orc_less(&hp->h[l], &hp->h[m])) m = l;
        if (r < hp->n && orc_less(&hp->h[r], &hp->h[m])) m = r;
        if (m == i) break;
        orc_ent t = hp->h[i]; hp->h[i] = hp->h[m]; hp->h[m] = t;
        i = m;
    }
    return top;
}

typedef struct {
    double *d1, *d2;
    int32_t *u, *v;
    orc_ent *heap;
    int32_t *width;  /* popped cells per row of the rank grid; rows [0, max_row] dirty after a query */
    orc_di *sort_tmp; /* cap_cand entries: merge-sort scratch of the rerank */
    int64_t cap_cand;
    int64_t *cand_pos;
    int32_t *cand_i, *cand_j;
    orc_di *dl;
} orc_work;

static int orc_work_init(orc_work *w, const orc_ix *ix)
{
    memset(w, 0, sizeof(*w));
    int T = ix->T;
    w->d1 = (double *)malloc(sizeof(double) * T);
    w->d2 = (double *)malloc(sizeof(double) * T);
    w->u = (int32_t *)malloc(sizeof(int32_t) * T);
    w->v = (int32_t *)malloc(sizeof(int32_t) * T);
    w->heap = (orc_ent *)malloc(sizeof(orc_ent) * ((size_t)T + 2));
    w->width = (int32_t *)calloc((size_t)T, sizeof(int32_t));
    return (w->d1 && w->d2 && w->u && w->v && w->heap && w->width) ? 0 : -1;
}

static int orc_work_cand(orc_work *w, int64_t n)
{
    if (n <= w->cap_cand) return 0;
    free(w->cand_pos); free(w->cand_i); free(w->cand_j); free(w->dl); free(w->sort_tmp);
    w->cap_cand = n;
    w->cand_pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    w->cand_i = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    w->cand_j = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    w->dl = (orc_di *)malloc(sizeof(orc_di) * (size_t)n);
    w->sort_tmp = (orc_di *)malloc(sizeof(orc_di) * (size_t)n);
    if (w->cand_pos && w->cand_i && w->cand_j && w->dl && w->sort_tmp) return 0;
    w->cap_cand = 0; /* a failed growth leaves no capacity claimed */
    return -1;
}

static void orc_work_free(orc_work *w)
{
    free(w->d1); free(w->d2); free(w->u); free(w->v); free(w->heap); free(w->width);
    free(w->cand_pos); free(w->cand_i); free(w->cand_j); free(w->dl); free(w->sort_tmp);
}

/* First step of the search (Section 2.3.3): visit cells in ascending order and
 * collect the points they hold until min(L, N) are collected.
 * Writes candidate storage positions and their cells (i, j) into w; optionally
 * records the visited cells (cell id, points taken). Returns the number of
 * candidates, and the number of visited cells in *ncells; -1 when the rank
 * lists cannot be sorted (no memory). */
static int64_t orc_collect(const orc_ix *ix, orc_work *w, const float *q, int64_t L,
                           int64_t *cells_out, int64_t cells_cap, int64_t *ncells)
{
    const int T = ix->T, h = ix->D / 2;
    orc_half_dists(q, ix->C1, T, h, w->d1);
    orc_half_dists(q + h, ix->C2, T, h, w->d2);
    if (orc_rank(w->d1, T, w->u) || orc_rank(w->d2, T, w->v)) return -1;

    const int64_t Leff = L < ix->N ? L : ix->N;
    int64_t total = 0, nc = 0;
    int32_t max_row = 0;
    orc_heap hp = { w->heap, 0 };
    if (Leff > 0) {
        orc_ent e0 = { w->d1[w->u[0]] + w->d2[w->v[0]], 0, 0 };
        orc_push(&hp, e0);
    }
    while (total < Leff && hp.n > 0) {
        orc_ent e = orc_pop(&hp);
        const int a = e.a, b = e.b;
        w->width[a] = b + 1; /* cells of a row leave the queue in column order */
        if (a > max_row) max_row = a;
        if (a + 1 < T && (b == 0 || b - 1 < w->width[a + 1])) {
            orc_ent n1 = { w->d1[w->u[a + 1]] + w->d2[w->v[b]], a + 1, b };
            orc_push(&hp, n1);
        }
        if (b + 1 < T && (a == 0 || b + 1 < w->width[a - 1])) {
            orc_ent n2 = { w->d1[w->u[a]] + w->d2[w->v[b + 1]], a, b + 1 };
            orc_push(&hp, n2);
        }
        const int32_t i = w->u[a], j = w->v[b];
        const int64_t c = (int64_t)i * T + j;
        const int64_t beg = ix->offsets[c], cnt = ix->offsets[c + 1] - beg;
        const int64_t take = cnt < Leff - total ? cnt : Leff - total;
        for (int64_t t = 0; t < take; ++t) {
            w->cand_pos[total + t] = beg + t;
            w->cand_i[total + t] = i;
            w->cand_j[total + t] = j;
        }
        if (cells_out && nc < cells_cap) {
            cells_out[2 * nc] = c;
            cells_out[2 * nc + 1] = take;
        }
        ++nc;
        total += take;
    }
    memset(w->width, 0, sizeof(int32_t) * (size_t)(max_row + 1));
    if (ncells) *ncells = nc;
    return total;
}

/* Squared distance from q to the reconstruction of equation (approximation):
 * x ~ [c1_i; c2_j] + [R_1(b_1); ...; R_M(b_M)], computed coordinate by
 * coordinate in FP64 -- the O(D) rerank of Section 2.3.3. With local
 * codebooks (QL, SL non-NULL) the codeword of subspace k < M/2 comes from
 * Q^i_k and that of subspace M/2 + k from S^j_k (equation residual). */
static double orc_dist(int D, int M, int Kc, const float *C1, const float *C2, const float *R,
                       const float *QL, const float *SL, const float *q, int32_t i, int32_t j,
                       const uint8_t *code)
{
    const int h = D / 2, ds = D / M, mh = M / 2;
    double acc = 0.0;
    for (int t = 0; t < D; ++t) {
        const double c = t < h ? (double)C1[(int64_t)i * h + t] : (double)C2[(int64_t)j * h + (t - h)];
        const int k = t / ds;
        const int64_t w = t - (int64_t)k * ds;
        double r;
        if (!QL) {
            r = (double)R[((int64_t)k * Kc + code[k]) * ds + w];
        } else if (k < mh) {
            r = (double)QL[(((int64_t)i * mh + k) * Kc + code[k]) * ds + w];
        } else {
            r = (double)SL[(((int64_t)j * mh + (k - mh)) * Kc + code[k]) * ds + w];
        }
        const double e = (double)q[t] - (c + r);
        acc += e * e;
    }
    return acc;
}

double orc_point_dist(int D, int T, int M, int Kc, const float *C1, const float *C2,
                      const float *R, const float *q, int32_t i, int32_t j, const uint8_t *code)
{
    (void)T;
    return orc_dist(D, M, Kc, C1, C2, R, NULL, NULL, q, i, j, code);
}

/* The same with local codebooks QL, SL ([T][M/2][Kc][D/M] each). */
double orc_point_dist_local(int D, int T, int M, int Kc, const float *C1, const float *C2,
                            const float *QL, const float *SL, const float *q, int32_t i, int32_t j,
                            const uint8_t *code)
{
    (void)T;
    return orc_dist(D, M, Kc, C1, C2, NULL, QL, SL, q, i, j, code);
}

/* FP64 distances (O(D) reconstruction, equation approximation; with QL and
 * SL the local codebooks of equation residual) from q, in the index's space,
 * to the stored points at storage positions pos[0..n): each point's cell is
 * found in the offsets. Returns 0, or -1 for a position outside [0, N). */
int orc_point_dists(int D, int T, int M, int Kc, int64_t N, const float *C1, const float *C2, const float *R,
                    const float *QL, const float *SL, const int64_t *offsets, const uint8_t *codes,
                    const float *q, int64_t n, const int64_t *pos, double *out)
{
    const int64_t C = (int64_t)T * T;
    for (int64_t e = 0; e < n; ++e) {
        const int64_t p = pos[e];
        if (p < 0 || p >= N) return -1;
        int64_t lo = 0, hi = C - 1; /* the last cell c with offsets[c] <= p */
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (offsets[mid] <= p) lo = mid;
            else hi = mid - 1;
        }
        out[e] = orc_dist(D, M, Kc, C1, C2, R, QL, SL, q, (int32_t)(lo / T), (int32_t)(lo % T), codes + p * M);
    }
    return 0;
}

/* Second step (Section 2.3.3): rerank the candidates by increasing distance,
 * ties by id, and keep the first k. */
static void orc_rerank(const orc_ix *ix, orc_work *w, const float *q, int64_t ncand,
                       int32_t k, int64_t *out_ids, double *out_d)
{
    for (int64_t p = 0; p < ncand; ++p) {
        const int64_t s = w->cand_pos[p];
        w->dl[p].d = orc_dist(ix->D, ix->M, ix->Kc, ix->C1, ix->C2, ix->R, ix->QL, ix->SL, q,
                              w->cand_i[p], w->cand_j[p], ix->codes + s * ix->M);
        w->dl[p].i = (int32_t)p;
    }
    /* stable merge sort by (distance, id); ids are unique */
    {
        int64_t n = ncand;
        orc_di *a = w->dl;
        orc_di *tmp = w->sort_tmp; /* ncand entries, allocated with the candidate arrays */
        for (int64_t width = 1; width < n; width *= 2) {
            for (int64_t lo = 0; lo < n; lo += 2 * width) {
                int64_t mid = lo + width < n ? lo + width : n;
                int64_t hi = lo + 2 * width < n ? lo + 2 * width : n;
                int64_t x = lo, y = mid, o = lo;
                while (x < mid && y < hi) {
                    const uint32_t ix_ = ix->ids[w->cand_pos[a[x].i]];
                    const uint32_t iy_ = ix->ids[w->cand_pos[a[y].i]];
                    int take_x = a[x].d < a[y].d || (a[x].d == a[y].d && ix_ <= iy_);
                    tmp[o++] = take_x ? a[x++] : a[y++];
                }
                while (x < mid) tmp[o++] = a[x++];
                while (y < hi) tmp[o++] = a[y++];
            }
            memcpy(a, tmp, sizeof(orc_di) * (size_t)n);
        }
    }
    for (int32_t r = 0; r < k; ++r) {
        if (r < ncand) {
            out_ids[r] = (int64_t)ix->ids[w->cand_pos[w->dl[r].i]];
            out_d[r] = w->dl[r].d;
        } else {
            out_ids[r] = -1;
            out_d[r] = INFINITY;
        }
    }
}

/* ---- exported entry points ------------------------------------------------ */

static orc_ix orc_make(int D, int T, int M, int Kc, int64_t N, const float *C1, const float *C2,
                       const float *R, const int64_t *offsets, const uint8_t *codes,
                       const uint32_t *ids)
{
    orc_ix ix = { D, T, M, Kc, N, C1, C2, R, offsets, codes, ids, NULL, NULL };
    return ix;
}

/* Visited cells and candidate positions of one query. cells: [cap][2] of
 * (cell id, points taken). Returns the number of candidates, -1 on allocation
 * failure, -2 when pos_cap is too small. */
int64_t orc_visit(int D, int T, int M, int Kc, int64_t N, const float *C1, const float *C2,
                  const float *R, const int64_t *offsets, const uint8_t *codes, const uint32_t *ids,
                  const float *q, int64_t L, int64_t *cells, int64_t cells_cap, int64_t *ncells,
                  int64_t *pos, int64_t pos_cap)
{
    orc_ix ix = orc_make(D, T, M, Kc, N, C1, C2, R, offsets, codes, ids);
    orc_work w;
    if (orc_work_init(&w, &ix)) { orc_work_free(&w); return -1; }
    const int64_t Leff = L < N ? L : N;
    if (orc_work_cand(&w, Leff > 0 ? Leff : 1)) { orc_work_free(&w); return -1; }
    int64_t n = orc_collect(&ix, &w, q, L, cells, cells_cap, ncells);
    if (n < 0) { orc_work_free(&w); return -1; }
    if (n > pos_cap) { orc_work_free(&w); return -2; }
    memcpy(pos, w.cand_pos, sizeof(int64_t) * (size_t)n);
    orc_work_free(&w);
    return n;
}

/* FP64 rank lists of one query: d1, d2 (T each) and u, v (T each). Returns 0,
 * or -1 when the sort scratch cannot be allocated. */
int orc_rank_lists(int D, int T, const float *C1, const float *C2, const float *q,
                   double *d1, double *d2, int32_t *u, int32_t *v)
{
    const int h = D / 2;
    orc_half_dists(q, C1, T, h, d1);
    orc_half_dists(q + h, C2, T, h, d2);
    return (orc_rank(d1, T, u) || orc_rank(d2, T, v)) ? -1 : 0;
}

typedef struct {
    const orc_ix *ix;
    const float *Q;
    int64_t nq;
    const int64_t *L;
    const int32_t *k;
    int32_t kmax;
    int64_t *out_ids;
    double *out_d;
    int64_t *out_ncand, *out_ncells;
    int tid, nth;
    int err;
} orc_job;

static void *orc_worker(void *arg)
{
    orc_job *j = (orc_job *)arg;
    const orc_ix *ix = j->ix;
    orc_work w;
    if (orc_work_init(&w, ix)) { orc_work_free(&w); j->err = -1; return NULL; }
    for (int64_t qi = j->tid; qi < j->nq; qi += j->nth) {
        const int64_t L = j->L[qi];
        const int64_t Leff = L < ix->N ? L : ix->N;
        if (orc_work_cand(&w, Leff > 0 ? Leff : 1)) { j->err = -1; break; }
        const float *q = j->Q + qi * ix->D;
        int64_t nc = 0;
        int64_t n = orc_collect(ix, &w, q, L, NULL, 0, &nc);
        if (n < 0) { j->err = -1; break; }
        orc_rerank(ix, &w, q, n, j->k[qi], j->out_ids + qi * j->kmax, j->out_d + qi * j->kmax);
        for (int32_t r = j->k[qi]; r < j->kmax; ++r) {
            j->out_ids[qi * j->kmax + r] = -1;
            j->out_d[qi * j->kmax + r] = INFINITY;
        }
        if (j->out_ncand) j->out_ncand[qi] = n;
        if (j->out_ncells) j->out_ncells[qi] = nc;
    }
    orc_work_free(&w);
    return NULL;
}

/* Full search for nq queries with per-query budgets L[q] and k[q] <= kmax,
 * queries split statically over nthreads POSIX threads. Outputs are
 * [nq][kmax]. Returns 0, or -1 on allocation failure. */
static int orc_run(orc_ix ix, const float *Q, int64_t nq, const int64_t *L, const int32_t *k, int32_t kmax,
                   int64_t *out_ids, double *out_d, int64_t *out_ncand, int64_t *out_ncells, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    orc_job jobs[256];
    int err = 0;
    for (int t = 0; t < nthreads; ++t) {
        orc_job jb = { &ix, Q, nq, L, k, kmax, out_ids, out_d, out_ncand, out_ncells, t, nthreads, 0 };
        jobs[t] = jb;
    }
    if (nthreads == 1) {
        orc_worker(&jobs[0]);
        return jobs[0].err;
    }
    /* a job whose thread cannot be created runs in the calling thread */
    int started[256];
    for (int t = 0; t < nthreads; ++t) started[t] = pthread_create(&th[t], NULL, orc_worker, &jobs[t]) == 0;
    for (int t = 0; t < nthreads; ++t)
        if (!started[t]) orc_worker(&jobs[t]);
    for (int t = 0; t < nthreads; ++t) {
        if (started[t]) pthread_join(th[t], NULL);
        if (jobs[t].err) err = jobs[t].err;
    }
    return err;
}

int orc_search(int D, int T, int M, int Kc, int64_t N, const float *C1, const float *C2,
               const float *R, const int64_t *offsets, const uint8_t *codes, const uint32_t *ids,
               const float *Q, int64_t nq, const int64_t *L, const int32_t *k, int32_t kmax,
               int64_t *out_ids, double *out_d, int64_t *out_ncand, int64_t *out_ncells,
               int nthreads)
{
    orc_ix ix = orc_make(D, T, M, Kc, N, C1, C2, R, offsets, codes, ids);
    return orc_run(ix, Q, nq, L, k, kmax, out_ids, out_d, out_ncand, out_ncells, nthreads);
}

/* The same search with local codebooks QL, SL ([T][M/2][Kc][D/M] each): the
 * HBPQ query processing of Section 3.2 (the traversal is that of Section 2.3). */
int orc_search_local(int D, int T, int M, int Kc, int64_t N, const float *C1, const float *C2,
                     const float *QL, const float *SL, const int64_t *offsets, const uint8_t *codes,
                     const uint32_t *ids, const float *Q, int64_t nq, const int64_t *L, const int32_t *k,
                     int32_t kmax, int64_t *out_ids, double *out_d, int64_t *out_ncand,
                     int64_t *out_ncells, int nthreads)
{
    orc_ix ix = orc_make(D, T, M, Kc, N, C1, C2, NULL, offsets, codes, ids);
    ix.QL = QL;
    ix.SL = SL;
    return orc_run(ix, Q, nq, L, k, kmax, out_ids, out_d, out_ncand, out_ncells, nthreads);
}
