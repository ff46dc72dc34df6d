/*
 * oracle.c -- plain FP64 CPU reference for the multi-RHS AMG-Krylov solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code with the GPU path.
 *
 * What it computes, and where each step comes from:
 *
 *  - A X = B with n x m blocks (paper, Section 1, the equation A X = B); the m
 *    columns are solved as simultaneous *independent* problems with their
 *    own Krylov scalars (paper, Section 2.2), stored interleaved X[i*m + j]
 *    so a matrix entry is loaded once for all m columns (Sections 2.2-2.3).
 *  - Classical algebraic multigrid (paper, Section 2.1, citing Trottenberg et
 *    al.), set up the Ruge-Stueben way: classical strength of connection,
 *    the first coarsening pass, direct interpolation, Galerkin coarse
 *    operators R A P with R = P^T, stopping at a small coarse grid solved by
 *    a dense LU (the paper's "direct" method, Section 2.1, Table 1).
 *  - Jacobi and Chebyshev smoothers (Section 2.1, Table 1); Chebyshev with
 *    polynomial order 2 as in the configuration example of Section 2.4.
 *  - Symmetric Gauss-Seidel (Section 2.1, Table 1; the smoother of the runs
 *    of Section 3.1, "hybrid symmetric Gauss-Seidel") in its l1-hybrid form:
 *    Gauss-Seidel inside blocks of consecutive rows, Jacobi across blocks,
 *    with the l1 diagonal of Baker, Falgout, Kolev and Yang, "Multigrid
 *    smoothers for ultraparallel computing", SISC 33 (2011).
 *  - V(1,1) cycle as the preconditioner of CG (Hestenes-Stiefel) or of
 *    right-preconditioned BiCGStab (van der Vorst), both cited in Section 2.1,
 *    or as a solver on its own (the stationary multigrid iteration).
 *
 * The paper gives no formulas for these methods; each routine below says
 * which textbook definition it follows.  Everything is sequential FP64
 * except that independent row loops carry an OpenMP pragma (each row is
 * computed by exactly one thread with a fixed order of operations, so the
 * results do not depend on the thread count).  Dot products are sums over
 * 64 fixed chunks of rows (each chunk in row order, then the chunks in
 * order), likewise independent of the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* progress lines on stderr, one per Krylov iteration (off by default) */
static int g_verbose = 0;
void orc_set_verbose(int v) { g_verbose = v; }

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EBREAKDOWN (-5)

#define ORC_MAXLEV 64

/* ------------------------------------------------------------------------ */
/* CSR container                                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int nr, nc;      /* rows, columns */
    int *rp;         /* nr + 1 */
    int *ci;         /* nnz, sorted per row */
    double *v;       /* nnz */
} ocsr;

static int nnz_of(const ocsr *a) { return a->rp[a->nr]; }

static void csr_free(ocsr *a)
{
    free(a->rp); free(a->ci); free(a->v);
    a->rp = NULL; a->ci = NULL; a->v = NULL;
}

static int csr_alloc(ocsr *a, int nr, int nc, int nnz)
{
    a->nr = nr; a->nc = nc;
    a->rp = (int *)calloc((size_t)nr + 1, sizeof(int));
    a->ci = (int *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int));
    a->v = (double *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    return (a->rp && a->ci && a->v) ? 0 : -1;
}

/* ------------------------------------------------------------------------ */
/* Multi-column products: Y = A X with X, Y interleaved (row-major n x m).   */
/* The "blas2" operation of the paper's Section 2.3 for NV columns.          */
/* ------------------------------------------------------------------------ */
static void spmm(const ocsr *a, int m, const double *X, double *Y)
{
    int i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < a->nr; i++) {
        double *y = Y + (size_t)i * m;
        int j, k;
        for (j = 0; j < m; j++) y[j] = 0.0;
        for (k = a->rp[i]; k < a->rp[i + 1]; k++) {
            const double aik = a->v[k];
            const double *x = X + (size_t)a->ci[k] * m;
            for (j = 0; j < m; j++) y[j] += aik * x[j];
        }
    }
}

/* R = B - A X */
static void residual(const ocsr *a, int m, const double *B, const double *X,
                     double *R)
{
    int i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < a->nr; i++) {
        double *r = R + (size_t)i * m;
        const double *b = B + (size_t)i * m;
        int j, k;
        for (j = 0; j < m; j++) r[j] = 0.0;
        for (k = a->rp[i]; k < a->rp[i + 1]; k++) {
            const double aik = a->v[k];
            const double *x = X + (size_t)a->ci[k] * m;
            for (j = 0; j < m; j++) r[j] += aik * x[j];
        }
        for (j = 0; j < m; j++) r[j] = b[j] - r[j];
    }
}

/* Dot products and norms are sums over rows taken in NCHUNK fixed,
 * contiguous chunks of rows: each chunk is summed in row order, then the
 * chunk sums in chunk order.  The order depends only on n, never on the
 * thread count, so the chunks can run in parallel and every result is
 * reproducible. */
#define NCHUNK 64

static int chunk_lo(int n, int c) { return (int)(((int64_t)n * c) / NCHUNK); }

/* column j of  b - A x  (one column only), returned as its 2-norm squared */
static double residual_col_norm2(const ocsr *a, int m, int j, const double *B,
                                 const double *X)
{
    double part[NCHUNK], s = 0.0;
    int c;
#pragma omp parallel for schedule(static)
    for (c = 0; c < NCHUNK; c++) {
        double t = 0.0;
        int i, k;
        for (i = chunk_lo(a->nr, c); i < chunk_lo(a->nr, c + 1); i++) {
            double ax = 0.0, r;
            for (k = a->rp[i]; k < a->rp[i + 1]; k++)
                ax += a->v[k] * X[(size_t)a->ci[k] * m + j];
            r = B[(size_t)i * m + j] - ax;
            t += r * r;
        }
        part[c] = t;
    }
    for (c = 0; c < NCHUNK; c++) s += part[c];
    return s;
}

static double dot_col(int n, int m, int j, const double *X, const double *Y)
{
    double part[NCHUNK], s = 0.0;
    int c;
#pragma omp parallel for schedule(static)
    for (c = 0; c < NCHUNK; c++) {
        double t = 0.0;
        int i;
        for (i = chunk_lo(n, c); i < chunk_lo(n, c + 1); i++)
            t += X[(size_t)i * m + j] * Y[(size_t)i * m + j];
        part[c] = t;
    }
    for (c = 0; c < NCHUNK; c++) s += part[c];
    return s;
}

/* all m column dots in one pass over the rows; column j is summed in the
 * same order as dot_col */
static void dots(int n, int m, const double *X, const double *Y, double *out)
{
    double *part = (double *)calloc((size_t)NCHUNK * m + 1, sizeof(double));
    int c, j;
#pragma omp parallel for schedule(static)
    for (c = 0; c < NCHUNK; c++) {
        double *t = part + (size_t)c * m;
        int i, jj;
        for (i = chunk_lo(n, c); i < chunk_lo(n, c + 1); i++) {
            const double *x = X + (size_t)i * m, *y = Y + (size_t)i * m;
            for (jj = 0; jj < m; jj++) t[jj] += x[jj] * y[jj];
        }
    }
    for (j = 0; j < m; j++) out[j] = 0.0;
    for (c = 0; c < NCHUNK; c++)
        for (j = 0; j < m; j++) out[j] += part[(size_t)c * m + j];
    free(part);
}

/* ------------------------------------------------------------------------ */
/* Setup step 1: strength of connection.                                     */
/* Classical (Ruge-Stueben) negative-coupling form: j is a strong            */
/* connection of i when -a_ij >= theta * max_{k != i} (-a_ik).  Rows with no */
/* negative off-diagonal have no strong connections.                         */
/* ------------------------------------------------------------------------ */
static int strength(const ocsr *a, double theta, int **srp_out, int **sci_out)
{
    int n = a->nr, i, k;
    int *srp = (int *)calloc((size_t)n + 1, sizeof(int));
    int *sci;
    if (!srp) return -1;
    for (i = 0; i < n; i++) {
        double mx = 0.0;
        int cnt = 0;
        for (k = a->rp[i]; k < a->rp[i + 1]; k++)
            if (a->ci[k] != i && -a->v[k] > mx) mx = -a->v[k];
        if (mx > 0.0)
            for (k = a->rp[i]; k < a->rp[i + 1]; k++)
                if (a->ci[k] != i && -a->v[k] >= theta * mx) cnt++;
        srp[i + 1] = srp[i] + cnt;
    }
    sci = (int *)malloc((size_t)(srp[n] > 0 ? srp[n] : 1) * sizeof(int));
    if (!sci) { free(srp); return -1; }
    for (i = 0; i < n; i++) {
        double mx = 0.0;
        int pos = srp[i];
        for (k = a->rp[i]; k < a->rp[i + 1]; k++)
            if (a->ci[k] != i && -a->v[k] > mx) mx = -a->v[k];
        if (mx > 0.0)
            for (k = a->rp[i]; k < a->rp[i + 1]; k++)
                if (a->ci[k] != i && -a->v[k] >= theta * mx) sci[pos++] = a->ci[k];
    }
    *srp_out = srp; *sci_out = sci;
    return 0;
}

/* pattern transpose of an n x n pattern */
static int pattern_transpose(int n, const int *rp, const int *ci, int **trp_out,
                             int **tci_out)
{
    int i, k;
    int nnz = rp[n];
    int *trp = (int *)calloc((size_t)n + 1, sizeof(int));
    int *tci = (int *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int));
    int *fill = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    if (!trp || !tci || !fill) { free(trp); free(tci); free(fill); return -1; }
    for (k = 0; k < nnz; k++) trp[ci[k] + 1]++;
    for (i = 0; i < n; i++) trp[i + 1] += trp[i];
    memcpy(fill, trp, (size_t)n * sizeof(int));
    for (i = 0; i < n; i++)
        for (k = rp[i]; k < rp[i + 1]; k++) tci[fill[ci[k]]++] = i;
    free(fill);
    *trp_out = trp; *tci_out = tci;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Setup step 2: Ruge-Stueben first coarsening pass (Trottenberg et al.,     */
/* Multigrid, Appendix A).  Weight lambda_i = |S_i^T| initially; repeatedly  */
/* take the undecided point of largest weight (ties: lowest index) as C,     */
/* make every undecided point that depends strongly on it F and raise the    */
/* weights of the undecided points those new F points depend on, then lower  */
/* the weights of the undecided points the new C point depends on.  No      */
/* second pass.  A binary max-heap with lazy deletion finds the next point.  */
/* ------------------------------------------------------------------------ */
typedef struct { int lam, idx; } hent;
typedef struct { hent *a; size_t n, cap; } heap_t;

static int hbetter(hent x, hent y)   /* x before y ? */
{
    return x.lam > y.lam || (x.lam == y.lam && x.idx < y.idx);
}

static int hpush(heap_t *h, int lam, int idx)
{
    size_t c;
    if (h->n == h->cap) {
        size_t nc = h->cap ? 2 * h->cap : 1024;
        hent *na = (hent *)realloc(h->a, nc * sizeof(hent));
        if (!na) return -1;
        h->a = na; h->cap = nc;
    }
    c = h->n++;
    h->a[c].lam = lam; h->a[c].idx = idx;
    while (c > 0) {
        size_t p = (c - 1) / 2;
        if (!hbetter(h->a[c], h->a[p])) break;
        { hent t = h->a[c]; h->a[c] = h->a[p]; h->a[p] = t; }
        c = p;
    }
    return 0;
}

static hent hpop(heap_t *h)
{
    hent top = h->a[0];
    size_t c = 0;
    h->a[0] = h->a[--h->n];
    for (;;) {
        size_t l = 2 * c + 1, r = l + 1, b = c;
        if (l < h->n && hbetter(h->a[l], h->a[b])) b = l;
        if (r < h->n && hbetter(h->a[r], h->a[b])) b = r;
        if (b == c) break;
        { hent t = h->a[c]; h->a[c] = h->a[b]; h->a[b] = t; }
        c = b;
    }
    return top;
}

enum { PT_U = 0, PT_C = 1, PT_F = 2 };

static int rs_first_pass(int n, const int *srp, const int *sci, const int *trp,
                         const int *tci, int *state)
{
    int *lam = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    heap_t h = {NULL, 0, 0};
    int i, k, kk;
    if (!lam) return -1;
    for (i = 0; i < n; i++) {
        state[i] = PT_U;
        lam[i] = trp[i + 1] - trp[i];
        if (hpush(&h, lam[i], i)) { free(lam); free(h.a); return -1; }
    }
    while (h.n > 0) {
        hent e = hpop(&h);
        i = e.idx;
        if (state[i] != PT_U || e.lam != lam[i]) continue;   /* stale */
        state[i] = PT_C;
        for (k = trp[i]; k < trp[i + 1]; k++) {              /* j in S_i^T */
            int j = tci[k];
            if (state[j] != PT_U) continue;
            state[j] = PT_F;
            for (kk = srp[j]; kk < srp[j + 1]; kk++) {       /* l in S_j */
                int l = sci[kk];
                if (state[l] == PT_U) {
                    lam[l]++;
                    if (hpush(&h, lam[l], l)) { free(lam); free(h.a); return -1; }
                }
            }
        }
        for (k = srp[i]; k < srp[i + 1]; k++) {              /* j in S_i */
            int j = sci[k];
            if (state[j] == PT_U) {
                lam[j]--;
                if (hpush(&h, lam[j], j)) { free(lam); free(h.a); return -1; }
            }
        }
    }
    free(lam); free(h.a);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Setup step 3: direct interpolation (Stueben, "Algebraic multigrid: an     */
/* introduction with applications", 2001).  C rows are unit rows.  For an F  */
/* point i with interpolatory set P_i = C n S_i and neighbourhood N_i:       */
/*   w_ik = -alpha_i a_ik / a_ii (a_ik < 0),                                */
/*   alpha_i = sum_{N_i} a_ij^- / sum_{P_i} a_ik^-,                         */
/*   w_ik = -beta_i a_ik / a_ii (a_ik > 0),                                 */
/*   beta_i = sum_{N_i} a_ij^+ / sum_{P_i} a_ik^+;                          */
/* when P_i has no positive entry the positive part of N_i is added to the   */
/* diagonal instead.  Coarse points are numbered by increasing fine index.   */
/* ------------------------------------------------------------------------ */
static int direct_interp(const ocsr *a, const int *srp, const int *sci,
                         const int *state, ocsr *P)
{
    int n = a->nr, i, k, nc = 0, nnz = 0;
    int *cidx = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    if (!cidx) return -1;
    for (i = 0; i < n; i++) cidx[i] = (state[i] == PT_C) ? nc++ : -1;
    /* count */
    for (i = 0; i < n; i++) {
        if (state[i] == PT_C) { nnz++; continue; }
        for (k = srp[i]; k < srp[i + 1]; k++)
            if (state[sci[k]] == PT_C) nnz++;
    }
    if (csr_alloc(P, n, nc, nnz)) { free(cidx); return -1; }
    nnz = 0;
    for (i = 0; i < n; i++) {
        if (state[i] == PT_C) {
            P->ci[nnz] = cidx[i]; P->v[nnz] = 1.0; nnz++;
        } else {
            double aii = 0.0, sneg_n = 0.0, spos_n = 0.0, sneg_p = 0.0,
                   spos_p = 0.0, alpha, beta, d;
            int s;
            for (k = a->rp[i]; k < a->rp[i + 1]; k++) {
                int j = a->ci[k];
                double aij = a->v[k];
                if (j == i) { aii += aij; continue; }
                if (aij < 0.0) sneg_n += aij; else spos_n += aij;
            }
            /* interpolatory set: strong C neighbours, values from row i */
            s = srp[i];
            for (k = a->rp[i]; k < a->rp[i + 1]; k++) {
                int j = a->ci[k];
                while (s < srp[i + 1] && sci[s] < j) s++;
                if (s < srp[i + 1] && sci[s] == j && state[j] == PT_C) {
                    if (a->v[k] < 0.0) sneg_p += a->v[k]; else spos_p += a->v[k];
                }
            }
            d = aii;
            if (spos_p == 0.0) d += spos_n;
            alpha = (sneg_p != 0.0) ? sneg_n / sneg_p : 0.0;
            beta = (spos_p != 0.0) ? spos_n / spos_p : 0.0;
            s = srp[i];
            for (k = a->rp[i]; k < a->rp[i + 1]; k++) {
                int j = a->ci[k];
                while (s < srp[i + 1] && sci[s] < j) s++;
                if (s < srp[i + 1] && sci[s] == j && state[j] == PT_C) {
                    double aij = a->v[k];
                    P->ci[nnz] = cidx[j];
                    P->v[nnz] = (aij < 0.0) ? -alpha * aij / d : -beta * aij / d;
                    nnz++;
                }
            }
        }
        P->rp[i + 1] = nnz;
    }
    free(cidx);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Aggressive coarsening (the paper's mg_agg_num_levels / mg_num_paths,     */
/* Section 2.4): after the first RS pass, a second RS pass runs over the C   */
/* points alone, on their distance-two strength: for C points i != j, j is   */
/* a strong connection of i when the paths of length one or two from i to j  */
/* in S number at least num_paths (one for j in S_i, one for every k in S_i  */
/* with j in S_k).  C points the second pass makes F become F.               */
/* ------------------------------------------------------------------------ */
static int aggressive_second_pass(int n, const int *srp, const int *sci, int num_paths,
                                  int *state)
{
    int *loc = (int *)malloc((size_t)(n + 1) * sizeof(int));
    int *pts = (int *)malloc((size_t)(n + 1) * sizeof(int));
    int *paths = (int *)calloc((size_t)(n + 1), sizeof(int));
    int *s2rp, *s2ci = NULL, *t2rp, *t2ci, *st2;
    int nc = 0, i, a, k, kk, cap = 16, cnt = 0;
    if (!loc || !pts || !paths) return -1;
    for (i = 0; i < n; i++) {
        loc[i] = -1;
        if (state[i] == PT_C) { loc[i] = nc; pts[nc++] = i; }
    }
    s2rp = (int *)calloc((size_t)nc + 1, sizeof(int));
    s2ci = (int *)malloc((size_t)cap * sizeof(int));
    if (!s2rp || !s2ci) return -1;
    for (a = 0; a < nc; a++) {
        i = pts[a];
        /* count the paths to every point, then keep the C points reached
           often enough, in increasing index (scan of the row's reach) */
        for (k = srp[i]; k < srp[i + 1]; k++) {
            int j = sci[k];
            paths[j]++;
            for (kk = srp[j]; kk < srp[j + 1]; kk++) paths[sci[kk]]++;
        }
        {
            int b;
            for (b = 0; b < nc; b++) {
                int j = pts[b];
                if (j != i && paths[j] >= num_paths) {
                    if (cnt == cap) {
                        cap *= 2;
                        s2ci = (int *)realloc(s2ci, (size_t)cap * sizeof(int));
                        if (!s2ci) return -1;
                    }
                    s2ci[cnt++] = b;
                }
            }
        }
        for (k = srp[i]; k < srp[i + 1]; k++) {
            int j = sci[k];
            paths[j] = 0;
            for (kk = srp[j]; kk < srp[j + 1]; kk++) paths[sci[kk]] = 0;
        }
        s2rp[a + 1] = cnt;
    }
    if (pattern_transpose(nc, s2rp, s2ci, &t2rp, &t2ci)) return -1;
    st2 = (int *)malloc((size_t)(nc + 1) * sizeof(int));
    if (!st2 || rs_first_pass(nc, s2rp, s2ci, t2rp, t2ci, st2)) return -1;
    for (a = 0; a < nc; a++) state[pts[a]] = st2[a];
    free(loc); free(pts); free(paths); free(s2rp); free(s2ci); free(t2rp); free(t2ci); free(st2);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Multipass interpolation (Stueben 2001, multi-pass interpolation), used on */
/* the aggressively coarsened levels.  C points have unit rows (pass 0).     */
/* Pass p takes every F point not yet interpolated that depends strongly on  */
/* a point of an earlier pass; its interpolatory set P_i is its strong        */
/* neighbours of earlier passes, its weights w_ij those of direct            */
/* interpolation over P_i, and its row is sum_{j in P_i} w_ij (row of j).     */
/* Pass 1 is therefore direct interpolation.  Unreached F points keep a      */
/* zero row; entries that come out exactly 0.0 are dropped.                  */
/* ------------------------------------------------------------------------ */
typedef struct { int n, cap; int *c; double *v; } orow;

static int orow_push(orow *r, int c, double v)
{
    if (r->n == r->cap) {
        r->cap = r->cap ? 2 * r->cap : 4;
        r->c = (int *)realloc(r->c, (size_t)r->cap * sizeof(int));
        r->v = (double *)realloc(r->v, (size_t)r->cap * sizeof(double));
        if (!r->c || !r->v) return -1;
    }
    r->c[r->n] = c; r->v[r->n] = v; r->n++;
    return 0;
}

static int is_strong(const int *srp, const int *sci, int i, int j)
{
    int k;
    for (k = srp[i]; k < srp[i + 1]; k++) if (sci[k] == j) return 1;
    return 0;
}

static int multipass_interp(const ocsr *a, const int *srp, const int *sci, const int *state,
                            ocsr *P)
{
    int n = a->nr, nc = 0, i, k, p, nnz = 0, q;
    int *cidx = (int *)malloc((size_t)(n + 1) * sizeof(int));
    int *pass = (int *)malloc((size_t)(n + 1) * sizeof(int));
    int *newp = (int *)malloc((size_t)(n + 1) * sizeof(int));
    orow *row = (orow *)calloc((size_t)(n + 1), sizeof(orow));
    double *acc;
    if (!cidx || !pass || !newp || !row) return -1;
    for (i = 0; i < n; i++) {
        cidx[i] = state[i] == PT_C ? nc++ : -1;
        pass[i] = state[i] == PT_C ? 0 : -1;
        if (state[i] == PT_C && orow_push(&row[i], cidx[i], 1.0)) return -1;
    }
    acc = (double *)calloc((size_t)nc + 1, sizeof(double));
    if (!acc) return -1;
    for (p = 1;; p++) {
        int m = 0;
        for (i = 0; i < n; i++) {
            if (pass[i] >= 0) continue;
            for (k = srp[i]; k < srp[i + 1]; k++)
                if (pass[sci[k]] >= 0 && pass[sci[k]] < p) { newp[m++] = i; break; }
        }
        if (m == 0) break;
        for (q = 0; q < m; q++) pass[newp[q]] = p;
        for (q = 0; q < m; q++) {
            double aii = 0.0, sneg_n = 0.0, spos_n = 0.0, sneg_p = 0.0, spos_p = 0.0, d,
                   alpha, beta;
            int c;
            i = newp[q];
            for (k = a->rp[i]; k < a->rp[i + 1]; k++) {
                int j = a->ci[k];
                double aij = a->v[k];
                if (j == i) { aii += aij; continue; }
                if (aij < 0.0) sneg_n += aij; else spos_n += aij;
                if (pass[j] >= 0 && pass[j] < p && is_strong(srp, sci, i, j)) {
                    if (aij < 0.0) sneg_p += aij; else spos_p += aij;
                }
            }
            d = aii + (spos_p == 0.0 ? spos_n : 0.0);
            alpha = (sneg_p != 0.0) ? sneg_n / sneg_p : 0.0;
            beta = (spos_p != 0.0) ? spos_n / spos_p : 0.0;
            for (k = a->rp[i]; k < a->rp[i + 1]; k++) {
                int j = a->ci[k], e;
                double aij = a->v[k], w;
                if (j == i || !(pass[j] >= 0 && pass[j] < p && is_strong(srp, sci, i, j)))
                    continue;
                w = (aij < 0.0) ? -alpha * aij / d : -beta * aij / d;
                for (e = 0; e < row[j].n; e++) acc[row[j].c[e]] += w * row[j].v[e];
            }
            /* collect the accumulated coarse columns in increasing order */
            for (k = a->rp[i]; k < a->rp[i + 1]; k++) {
                int j = a->ci[k], e;
                if (j == i || !(pass[j] >= 0 && pass[j] < p && is_strong(srp, sci, i, j)))
                    continue;
                for (e = 0; e < row[j].n; e++) {
                    c = row[j].c[e];
                    if (acc[c] != 0.0) {
                        /* insertion keeps the row sorted; each column once */
                        int t = row[i].n, found = 0;
                        for (t = 0; t < row[i].n; t++) if (row[i].c[t] == c) { found = 1; break; }
                        if (!found && orow_push(&row[i], c, 0.0)) return -1;
                    }
                }
            }
            {
                int t, u;
                for (t = 1; t < row[i].n; t++)
                    for (u = t; u > 0 && row[i].c[u] < row[i].c[u - 1]; u--) {
                        int tc = row[i].c[u]; row[i].c[u] = row[i].c[u - 1]; row[i].c[u - 1] = tc;
                    }
                for (t = 0; t < row[i].n; t++) { row[i].v[t] = acc[row[i].c[t]]; }
                for (t = 0; t < row[i].n; t++) acc[row[i].c[t]] = 0.0;
            }
            /* columns whose sum was exactly zero were never added; clear them */
            for (k = a->rp[i]; k < a->rp[i + 1]; k++) {
                int j = a->ci[k], e;
                if (j == i) continue;
                for (e = 0; e < row[j].n; e++) acc[row[j].c[e]] = 0.0;
            }
        }
    }
    for (i = 0; i < n; i++) nnz += row[i].n;
    if (csr_alloc(P, n, nc, nnz)) return -1;
    nnz = 0;
    for (i = 0; i < n; i++) {
        for (k = 0; k < row[i].n; k++) { P->ci[nnz] = row[i].c[k]; P->v[nnz] = row[i].v[k]; nnz++; }
        P->rp[i + 1] = nnz;
        free(row[i].c); free(row[i].v);
    }
    free(cidx); free(pass); free(newp); free(row); free(acc);
    return 0;
}

/* full transpose of a CSR matrix (values included) */
static int csr_transpose(const ocsr *a, ocsr *t)
{
    int i, k, nnz = nnz_of(a);
    int *fill;
    if (csr_alloc(t, a->nc, a->nr, nnz)) return -1;
    fill = (int *)malloc((size_t)(a->nc > 0 ? a->nc : 1) * sizeof(int));
    if (!fill) return -1;
    for (k = 0; k < nnz; k++) t->rp[a->ci[k] + 1]++;
    for (i = 0; i < a->nc; i++) t->rp[i + 1] += t->rp[i];
    memcpy(fill, t->rp, (size_t)a->nc * sizeof(int));
    for (i = 0; i < a->nr; i++)
        for (k = a->rp[i]; k < a->rp[i + 1]; k++) {
            int p = fill[a->ci[k]]++;
            t->ci[p] = i;
            t->v[p] = a->v[k];
        }
    free(fill);
    return 0;
}

static int cmp_int(const void *x, const void *y)
{
    int a = *(const int *)x, b = *(const int *)y;
    return (a > b) - (a < b);
}

/* C = A B (Gustavson row by row with a dense accumulator; entries that come
 * out exactly 0.0 are dropped; columns sorted). */
static int csr_matmul(const ocsr *A, const ocsr *B, ocsr *C)
{
    int n = A->nr, nc = B->nc, i, k, kk;
    double *acc = (double *)calloc((size_t)(nc > 0 ? nc : 1), sizeof(double));
    int *mark = (int *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int));
    int *list = (int *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int));
    size_t cap = 1024, nnz = 0;
    int *ci = (int *)malloc(cap * sizeof(int));
    double *v = (double *)malloc(cap * sizeof(double));
    int *rp = (int *)calloc((size_t)n + 1, sizeof(int));
    if (!acc || !mark || !list || !ci || !v || !rp) return -1;
    for (k = 0; k < nc; k++) mark[k] = -1;
    for (i = 0; i < n; i++) {
        int len = 0, t;
        for (k = A->rp[i]; k < A->rp[i + 1]; k++) {
            int j = A->ci[k];
            double aij = A->v[k];
            for (kk = B->rp[j]; kk < B->rp[j + 1]; kk++) {
                int c = B->ci[kk];
                if (mark[c] != i) { mark[c] = i; acc[c] = 0.0; list[len++] = c; }
                acc[c] += aij * B->v[kk];
            }
        }
        qsort(list, (size_t)len, sizeof(int), cmp_int);
        if (nnz + (size_t)len > cap) {
            while (nnz + (size_t)len > cap) cap *= 2;
            ci = (int *)realloc(ci, cap * sizeof(int));
            v = (double *)realloc(v, cap * sizeof(double));
            if (!ci || !v) return -1;
        }
        for (t = 0; t < len; t++) {
            double x = acc[list[t]];
            if (x != 0.0) { ci[nnz] = list[t]; v[nnz] = x; nnz++; }
        }
        rp[i + 1] = (int)nnz;
    }
    free(acc); free(mark); free(list);
    C->nr = n; C->nc = nc; C->rp = rp; C->ci = ci; C->v = v;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Dense LU with partial pivoting (row-major n x n), in place.               */
/* ------------------------------------------------------------------------ */
static int dense_lu(int n, double *a, int *piv)
{
    int i, j, k;
    for (k = 0; k < n; k++) {
        int p = k;
        double mx = fabs(a[(size_t)k * n + k]);
        for (i = k + 1; i < n; i++)
            if (fabs(a[(size_t)i * n + k]) > mx) { mx = fabs(a[(size_t)i * n + k]); p = i; }
        piv[k] = p;
        if (mx == 0.0) return -1;
        if (p != k)
            for (j = 0; j < n; j++) {
                double t = a[(size_t)k * n + j];
                a[(size_t)k * n + j] = a[(size_t)p * n + j];
                a[(size_t)p * n + j] = t;
            }
        for (i = k + 1; i < n; i++) {
            double l = a[(size_t)i * n + k] / a[(size_t)k * n + k];
            a[(size_t)i * n + k] = l;
            for (j = k + 1; j < n; j++) a[(size_t)i * n + j] -= l * a[(size_t)k * n + j];
        }
    }
    return 0;
}

/* solve with the factors for one right-hand side x (in place) */
static void dense_lu_solve(int n, const double *lu, const int *piv, double *x)
{
    int i, j;
    for (i = 0; i < n; i++)
        if (piv[i] != i) { double t = x[i]; x[i] = x[piv[i]]; x[piv[i]] = t; }
    for (i = 0; i < n; i++) {
        double s = x[i];
        for (j = 0; j < i; j++) s -= lu[(size_t)i * n + j] * x[j];
        x[i] = s;
    }
    for (i = n - 1; i >= 0; i--) {
        double s = x[i];
        for (j = i + 1; j < n; j++) s -= lu[(size_t)i * n + j] * x[j];
        x[i] = s / lu[(size_t)i * n + i];
    }
}

/* ------------------------------------------------------------------------ */
/* Counter-based uniform numbers for the Lanczos start vector: SplitMix64    */
/* (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",    */
/* OOPSLA 2014).  Element i of stream `key` is the finaliser applied to      */
/* key*G + (i+1)*G with G = 0x9E3779B97F4A7C15, mapped to [-1, 1) through    */
/* its top 53 bits.                                                          */
/* ------------------------------------------------------------------------ */
static double sm64_uniform(uint64_t key, uint64_t i)
{
    const uint64_t G = 0x9E3779B97F4A7C15ULL;
    uint64_t z = key * G + (i + 1) * G;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

/* number of eigenvalues of the symmetric tridiagonal (a, b) below x
 * (Sturm sequence count) */
static int sturm_count(int k, const double *a, const double *b, double x)
{
    int i, c = 0;
    double q = 1.0;
    for (i = 0; i < k; i++) {
        double bb = (i > 0) ? b[i] * b[i] : 0.0;
        q = a[i] - x - ((i > 0) ? bb / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) c++;
    }
    return c;
}

/* Largest Ritz value of `steps` Lanczos steps on D^{-1/2} A D^{-1/2}, start
 * vector from SplitMix64 stream `key` (no reorthogonalisation; the largest
 * eigenvalue of the tridiagonal found by bisection on the Sturm count). */
static double lanczos_lmax(const ocsr *a, int steps, uint64_t key)
{
    int n = a->nr, i, j, k = 0;
    double *dsq = (double *)malloc((size_t)n * sizeof(double));
    double *v = (double *)calloc((size_t)n, sizeof(double));
    double *vp = (double *)calloc((size_t)n, sizeof(double));
    double *w = (double *)malloc((size_t)n * sizeof(double));
    double *t = (double *)malloc((size_t)n * sizeof(double));
    double al[64], be[64], nrm = 0.0, lo, hi;
    if (steps > n) steps = n;
    if (steps > 63) steps = 63;
    for (i = 0; i < n; i++) {
        double d = 0.0;
        for (j = a->rp[i]; j < a->rp[i + 1]; j++)
            if (a->ci[j] == i) d += a->v[j];
        dsq[i] = 1.0 / sqrt(d);
        v[i] = sm64_uniform(key, (uint64_t)i);
        nrm += v[i] * v[i];
    }
    nrm = sqrt(nrm);
    for (i = 0; i < n; i++) v[i] /= nrm;
    be[0] = 0.0;
    for (j = 0; j < steps; j++) {
        double alpha = 0.0, beta = 0.0;
        for (i = 0; i < n; i++) t[i] = dsq[i] * v[i];
        spmm(a, 1, t, w);
        for (i = 0; i < n; i++) w[i] *= dsq[i];
        for (i = 0; i < n; i++) alpha += w[i] * v[i];
        for (i = 0; i < n; i++) w[i] -= alpha * v[i] + be[j] * vp[i];
        for (i = 0; i < n; i++) beta += w[i] * w[i];
        beta = sqrt(beta);
        al[j] = alpha;
        k = j + 1;
        if (j + 1 < steps) {
            be[j + 1] = beta;
            if (beta == 0.0) break;
            for (i = 0; i < n; i++) { vp[i] = v[i]; v[i] = w[i] / beta; }
        }
    }
    /* Gershgorin interval, then bisection for the k-th (largest) eigenvalue */
    lo = 1e300; hi = -1e300;
    for (i = 0; i < k; i++) {
        double r = ((i > 0) ? fabs(be[i]) : 0.0) + ((i + 1 < k) ? fabs(be[i + 1]) : 0.0);
        if (al[i] - r < lo) lo = al[i] - r;
        if (al[i] + r > hi) hi = al[i] + r;
    }
    for (i = 0; i < 200; i++) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(k, al, be, mid) >= k) hi = mid; else lo = mid;
    }
    free(dsq); free(v); free(vp); free(w); free(t);
    return hi;
}

/* ------------------------------------------------------------------------ */
/* Hierarchy                                                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    int nlev;                 /* levels 0..nlev-1; level nlev-1 is coarsest */
    ocsr A[ORC_MAXLEV];
    ocsr P[ORC_MAXLEV];       /* P[l]: n_l x n_{l+1}, l < nlev-1 */
    ocsr R[ORC_MAXLEV];       /* R[l] = P[l]^T */
    int *cf[ORC_MAXLEV];      /* C/F marker of level l (l < nlev-1) */
    double *dinv[ORC_MAXLEV]; /* 1 / a_ii */
    double lmax[ORC_MAXLEV];  /* Lanczos estimate of lambda_max(D^-1 A) */
    double *lu;               /* LU factors of the coarsest matrix */
    int *piv;
} ohier;

#define ORC_LANCZOS_KEY 7ULL

static int csr_copy(const ocsr *src, ocsr *dst)
{
    int nnz = nnz_of(src);
    if (csr_alloc(dst, src->nr, src->nc, nnz)) return -1;
    memcpy(dst->rp, src->rp, ((size_t)src->nr + 1) * sizeof(int));
    memcpy(dst->ci, src->ci, (size_t)nnz * sizeof(int));
    memcpy(dst->v, src->v, (size_t)nnz * sizeof(double));
    return 0;
}

void orc_hier_free(ohier *h)
{
    int l;
    if (!h) return;
    for (l = 0; l < h->nlev; l++) {
        csr_free(&h->A[l]);
        if (l + 1 < h->nlev) { csr_free(&h->P[l]); csr_free(&h->R[l]); }
        free(h->cf[l]);
        free(h->dinv[l]);
    }
    free(h->lu); free(h->piv);
    free(h);
}

/*
 * Build the hierarchy: levels are added while the current level has more
 * than `max_coarse` rows.  Returns ORC_EBREAKDOWN when more than
 * `max_levels` levels would be needed, when a level fails to shrink below
 * 0.9 of its parent, or when the coarsest matrix is singular.
 */
int orc_build(int n, const int *rp, const int *ci, const double *v, double theta,
              int max_coarse, int max_levels, int lanczos_steps, int agg_levels, int num_paths,
              ohier **out)
{
    ohier *h = (ohier *)calloc(1, sizeof(ohier));
    ocsr a0;
    int l, i, k, nL;
    if (!h) return ORC_ENOMEM;
    if (max_levels > ORC_MAXLEV) max_levels = ORC_MAXLEV;
    a0.nr = n; a0.nc = n; a0.rp = (int *)rp; a0.ci = (int *)ci; a0.v = (double *)v;
    if (csr_copy(&a0, &h->A[0])) { free(h); return ORC_ENOMEM; }
    h->nlev = 1;
    for (l = 0; h->A[l].nr > max_coarse; l++) {
        int *srp, *sci, *trp, *tci;
        ocsr AP;
        if (l + 1 >= max_levels) { orc_hier_free(h); return ORC_EBREAKDOWN; }
        if (strength(&h->A[l], theta, &srp, &sci)) { orc_hier_free(h); return ORC_ENOMEM; }
        if (pattern_transpose(h->A[l].nr, srp, sci, &trp, &tci)) { orc_hier_free(h); return ORC_ENOMEM; }
        h->cf[l] = (int *)malloc((size_t)h->A[l].nr * sizeof(int));
        if (!h->cf[l] || rs_first_pass(h->A[l].nr, srp, sci, trp, tci, h->cf[l])) {
            orc_hier_free(h); return ORC_ENOMEM;
        }
        if (l < agg_levels) {
            if (aggressive_second_pass(h->A[l].nr, srp, sci, num_paths, h->cf[l]) ||
                multipass_interp(&h->A[l], srp, sci, h->cf[l], &h->P[l])) {
                orc_hier_free(h); return ORC_ENOMEM;
            }
        } else if (direct_interp(&h->A[l], srp, sci, h->cf[l], &h->P[l])) {
            orc_hier_free(h); return ORC_ENOMEM;
        }
        free(srp); free(sci); free(trp); free(tci);
        if (csr_transpose(&h->P[l], &h->R[l])) { orc_hier_free(h); return ORC_ENOMEM; }
        if (csr_matmul(&h->A[l], &h->P[l], &AP)) { orc_hier_free(h); return ORC_ENOMEM; }
        if (csr_matmul(&h->R[l], &AP, &h->A[l + 1])) { orc_hier_free(h); return ORC_ENOMEM; }
        csr_free(&AP);
        h->nlev = l + 2;
        if (h->A[l + 1].nr == 0 || (double)h->A[l + 1].nr > 0.9 * (double)h->A[l].nr) {
            orc_hier_free(h); return ORC_EBREAKDOWN;
        }
    }
    for (l = 0; l < h->nlev; l++) {
        ocsr *a = &h->A[l];
        h->dinv[l] = (double *)malloc((size_t)a->nr * sizeof(double));
        for (i = 0; i < a->nr; i++) {
            double d = 0.0;
            for (k = a->rp[i]; k < a->rp[i + 1]; k++)
                if (a->ci[k] == i) d += a->v[k];
            h->dinv[l][i] = 1.0 / d;
        }
        h->lmax[l] = (l + 1 < h->nlev)
                         ? lanczos_lmax(a, lanczos_steps, (ORC_LANCZOS_KEY << 32) + (uint64_t)l)
                         : 0.0;
    }
    nL = h->A[h->nlev - 1].nr;
    h->lu = (double *)calloc((size_t)nL * nL + 1, sizeof(double));
    h->piv = (int *)malloc(((size_t)nL + 1) * sizeof(int));
    {
        ocsr *a = &h->A[h->nlev - 1];
        for (i = 0; i < nL; i++)
            for (k = a->rp[i]; k < a->rp[i + 1]; k++)
                h->lu[(size_t)i * nL + a->ci[k]] = a->v[k];
    }
    if (dense_lu(nL, h->lu, h->piv)) { orc_hier_free(h); return ORC_EBREAKDOWN; }
    *out = h;
    return ORC_OK;
}

/* ---- accessors (copy out) ------------------------------------------------ */
int orc_hier_nlev(const ohier *h) { return h->nlev; }

/* which: 0 = A, 1 = P, 2 = R.  info[0..2] = rows, cols, nnz */
int orc_hier_info(const ohier *h, int which, int l, int *info)
{
    const ocsr *a;
    if (l < 0 || l >= h->nlev) return ORC_EINVAL;
    if (which != 0 && l >= h->nlev - 1) return ORC_EINVAL;
    a = which == 0 ? &h->A[l] : which == 1 ? &h->P[l] : &h->R[l];
    info[0] = a->nr; info[1] = a->nc; info[2] = nnz_of(a);
    return ORC_OK;
}

int orc_hier_copy(const ohier *h, int which, int l, int *rp, int *ci, double *v)
{
    const ocsr *a;
    if (l < 0 || l >= h->nlev) return ORC_EINVAL;
    if (which != 0 && l >= h->nlev - 1) return ORC_EINVAL;
    a = which == 0 ? &h->A[l] : which == 1 ? &h->P[l] : &h->R[l];
    memcpy(rp, a->rp, ((size_t)a->nr + 1) * sizeof(int));
    memcpy(ci, a->ci, (size_t)nnz_of(a) * sizeof(int));
    memcpy(v, a->v, (size_t)nnz_of(a) * sizeof(double));
    return ORC_OK;
}

int orc_hier_cf(const ohier *h, int l, int *cf)
{
    if (l < 0 || l >= h->nlev - 1) return ORC_EINVAL;
    memcpy(cf, h->cf[l], (size_t)h->A[l].nr * sizeof(int));
    return ORC_OK;
}

double orc_hier_lmax(const ohier *h, int l) { return h->lmax[l]; }

/* ------------------------------------------------------------------------ */
/* Smoothers (on D^-1 A)                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int smoother;      /* 0 = Jacobi, 1 = Chebyshev, 2 = l1-hybrid symmetric GS */
    double omega;      /* Jacobi damping */
    int degree;        /* Chebyshev degree */
    double lo_frac;    /* Chebyshev interval [lo_frac*hi, hi] */
    double hi_frac;    /* hi = hi_frac * lambda_max estimate */
    int gs_block;      /* Gauss-Seidel block size (rows) */
} smopt;

/* damped Jacobi: x <- x + omega D^-1 (b - A x); t is an n x m temporary */
static void jacobi(const ocsr *a, const double *dinv, double omega, int m,
                   const double *b, double *x, double *t)
{
    int i;
    residual(a, m, b, x, t);
#pragma omp parallel for schedule(static)
    for (i = 0; i < a->nr; i++) {
        int j;
        for (j = 0; j < m; j++)
            x[(size_t)i * m + j] += omega * dinv[i] * t[(size_t)i * m + j];
    }
}

/*
 * Chebyshev acceleration of Jacobi on [lo, hi] (Saad, Iterative Methods for
 * Sparse Linear Systems, 2nd ed., Algorithm 12.1, applied to D^-1 A):
 *   theta = (hi+lo)/2, delta = (hi-lo)/2, sigma = theta/delta, rho = 1/sigma,
 *   r = D^-1 (b - A x), d = r / theta,
 *   for k = 1..degree: x += d; if k < degree:
 *      r -= D^-1 A d; rho' = 1/(2 sigma - rho);
 *      d = rho' rho d + (2 rho'/delta) r; rho = rho'.
 * r, d, t are n x m temporaries.
 */
static void chebyshev(const ocsr *a, const double *dinv, double lo, double hi,
                      int degree, int m, const double *b, double *x, double *r,
                      double *d, double *t)
{
    double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
    double sigma = theta / delta, rho = 1.0 / sigma;
    size_t nm = (size_t)a->nr * m, q;
    int k, i;
    residual(a, m, b, x, r);
#pragma omp parallel for schedule(static)
    for (i = 0; i < a->nr; i++) {
        int j;
        for (j = 0; j < m; j++) {
            r[(size_t)i * m + j] *= dinv[i];
            d[(size_t)i * m + j] = r[(size_t)i * m + j] / theta;
        }
    }
    for (k = 1; k <= degree; k++) {
        for (q = 0; q < nm; q++) x[q] += d[q];
        if (k < degree) {
            double rn;
            spmm(a, m, d, t);
            rn = 1.0 / (2.0 * sigma - rho);
#pragma omp parallel for schedule(static)
            for (i = 0; i < a->nr; i++) {
                int j;
                for (j = 0; j < m; j++) {
                    size_t p = (size_t)i * m + j;
                    r[p] -= dinv[i] * t[p];
                    d[p] = rn * rho * d[p] + (2.0 * rn / delta) * r[p];
                }
            }
            rho = rn;
        }
    }
}

/*
 * l1-hybrid Gauss-Seidel sweep (Baker, Falgout, Kolev, Yang 2011).  The rows
 * are cut into blocks of B consecutive rows; block k holds rows
 * [kB, min(n, kB + B)).  With d_i = a_ii + sum over j outside i's block of
 * |a_ij|, one forward sweep computes, row by row in increasing order inside
 * each block (the blocks are independent of each other),
 *   xn_i = xo_i + (b_i - sum_{j in block, j < i} a_ij xn_j
 *                      - sum_{all other j} a_ij xo_j) / d_i,
 * i.e. Gauss-Seidel inside a block and Jacobi (old values) across blocks;
 * the backward sweep runs each block's rows in decreasing order and uses the
 * new values of the rows j > i of the block.  xo and xn are n x m and must
 * not overlap.  With B >= n this is plain Gauss-Seidel; with B = 1 it is
 * l1-Jacobi.
 */
static void hgs_sweep(const ocsr *a, int B, int backward, int m, const double *b,
                      const double *xo, double *xn)
{
    int n = a->nr, nblk = (n + B - 1) / B, blk;
#pragma omp parallel for schedule(static)
    for (blk = 0; blk < nblk; blk++) {
        int lo = blk * B, hi = lo + B < n ? lo + B : n, s, j;
        for (s = 0; s < hi - lo; s++) {
            int i = backward ? hi - 1 - s : lo + s, k;
            double d = 0.0;
            for (k = a->rp[i]; k < a->rp[i + 1]; k++) {
                int c = a->ci[k];
                if (c == i) d += a->v[k];
                else if (c < lo || c >= hi) d += fabs(a->v[k]);
            }
            for (j = 0; j < m; j++) {
                double acc = 0.0;
                for (k = a->rp[i]; k < a->rp[i + 1]; k++) {
                    int c = a->ci[k];
                    int fresh = c >= lo && c < hi && (backward ? c > i : c < i);
                    acc += a->v[k] * (fresh ? xn[(size_t)c * m + j] : xo[(size_t)c * m + j]);
                }
                xn[(size_t)i * m + j] = xo[(size_t)i * m + j] + (b[(size_t)i * m + j] - acc) / d;
            }
        }
    }
}

/* symmetric sweep: forward from x into t, then backward from t into x */
static void hgs_symmetric(const ocsr *a, int B, int m, const double *b, double *x, double *t)
{
    hgs_sweep(a, B, 0, m, b, x, t);
    hgs_sweep(a, B, 1, m, b, t, x);
}

/* ------------------------------------------------------------------------ */
/* V(1,1) cycle from a zero initial guess:                                   */
/*   pre-smooth, r = b - A x, b_c = R r, recurse (coarsest: direct LU),      */
/*   x += P x_c, post-smooth.                                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int m;
    double *b[ORC_MAXLEV], *x[ORC_MAXLEV], *r[ORC_MAXLEV], *d[ORC_MAXLEV],
        *t[ORC_MAXLEV];
    double *col;   /* nL scratch */
} vws;

static void vws_free(vws *w, int nlev)
{
    int l;
    for (l = 0; l < nlev; l++) {
        free(w->b[l]); free(w->x[l]); free(w->r[l]); free(w->d[l]); free(w->t[l]);
    }
    free(w->col);
}

static int vws_alloc(vws *w, const ohier *h, int m)
{
    int l;
    memset(w, 0, sizeof(*w));
    w->m = m;
    for (l = 0; l < h->nlev; l++) {
        size_t nm = (size_t)h->A[l].nr * m + 1;
        w->b[l] = (double *)calloc(nm, sizeof(double));
        w->x[l] = (double *)calloc(nm, sizeof(double));
        w->r[l] = (double *)calloc(nm, sizeof(double));
        w->d[l] = (double *)calloc(nm, sizeof(double));
        w->t[l] = (double *)calloc(nm, sizeof(double));
        if (!w->b[l] || !w->x[l] || !w->r[l] || !w->d[l] || !w->t[l]) return -1;
    }
    w->col = (double *)malloc(((size_t)h->A[h->nlev - 1].nr + 1) * sizeof(double));
    return w->col ? 0 : -1;
}

static void smooth(const ohier *h, int l, const smopt *so, int m, const double *b,
                   double *x, vws *w)
{
    if (so->smoother == 0)
        jacobi(&h->A[l], h->dinv[l], so->omega, m, b, x, w->t[l]);
    else if (so->smoother == 2)
        hgs_symmetric(&h->A[l], so->gs_block, m, b, x, w->t[l]);
    else
        chebyshev(&h->A[l], h->dinv[l], so->lo_frac * so->hi_frac * h->lmax[l],
                  so->hi_frac * h->lmax[l], so->degree, m, b, x, w->r[l], w->d[l],
                  w->t[l]);
}

static void coarse_solve(const ohier *h, int m, const double *b, double *x, double *col)
{
    int nL = h->A[h->nlev - 1].nr, i, j;
    for (j = 0; j < m; j++) {
        for (i = 0; i < nL; i++) col[i] = b[(size_t)i * m + j];
        dense_lu_solve(nL, h->lu, h->piv, col);
        for (i = 0; i < nL; i++) x[(size_t)i * m + j] = col[i];
    }
}

static void vcycle_level(const ohier *h, int l, const smopt *so, int m,
                         const double *b, double *x, vws *w)
{
    size_t nm = (size_t)h->A[l].nr * m;
    if (l == h->nlev - 1) { coarse_solve(h, m, b, x, w->col); return; }
    memset(x, 0, nm * sizeof(double));
    smooth(h, l, so, m, b, x, w);
    residual(&h->A[l], m, b, x, w->r[l]);
    spmm(&h->R[l], m, w->r[l], w->b[l + 1]);
    vcycle_level(h, l + 1, so, m, w->b[l + 1], w->x[l + 1], w);
    {
        /* x += P x_c */
        spmm(&h->P[l], m, w->x[l + 1], w->t[l]);
        size_t q;
        for (q = 0; q < nm; q++) x[q] += w->t[l][q];
    }
    smooth(h, l, so, m, b, x, w);
}

int orc_vcycle(const ohier *h, int smoother, double omega, int degree,
               double lo_frac, double hi_frac, int gs_block, int m, const double *b, double *x)
{
    vws w;
    smopt so = {smoother, omega, degree, lo_frac, hi_frac, gs_block};
    if (smoother == 2 && gs_block < 1) return ORC_EINVAL;
    if (vws_alloc(&w, h, m)) { vws_free(&w, h->nlev); return ORC_ENOMEM; }
    vcycle_level(h, 0, &so, m, b, x, &w);
    vws_free(&w, h->nlev);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The same V(1,1) cycle carried out in FP32 (the reduced-precision          */
/* preconditioner of Section 2.3): every level matrix, D^-1, the coarsest    */
/* inverse and every vector rounded to float, every sum accumulated in       */
/* float, the steps in the order of the FP64 cycle above.  Scalars of the    */
/* smoothers (omega, the Chebyshev coefficients) are formed in FP64 and      */
/* rounded once.  The input b is rounded to float at level 0 and the result  */
/* is returned widened to FP64.  The coarsest level multiplies by the        */
/* inverse of A_L (from the FP64 LU factors, rounded to float).              */
/* ------------------------------------------------------------------------ */
typedef struct { int nr, nc; const int *rp, *ci; float *v; } fcsr;

typedef struct {
    fcsr A[ORC_MAXLEV], P[ORC_MAXLEV], R[ORC_MAXLEV];
    float *dinv[ORC_MAXLEV];
    float *inv;                  /* nL x nL, row-major */
    int nlev, m;
    float *b[ORC_MAXLEV], *x[ORC_MAXLEV], *r[ORC_MAXLEV], *d[ORC_MAXLEV], *t[ORC_MAXLEV];
} fws;

static float *f_of(const double *v, size_t n)
{
    float *f = (float *)malloc((n + 1) * sizeof(float));
    size_t q;
    if (f) for (q = 0; q < n; q++) f[q] = (float)v[q];
    return f;
}

static void fcsr_of(const ocsr *a, fcsr *f)
{
    f->nr = a->nr; f->nc = a->nc; f->rp = a->rp; f->ci = a->ci;
    f->v = f_of(a->v, (size_t)nnz_of(a));
}

static void fspmm(const fcsr *a, int m, const float *X, float *Y)
{
    int i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < a->nr; i++) {
        float *y = Y + (size_t)i * m;
        int j, k;
        for (j = 0; j < m; j++) y[j] = 0.0f;
        for (k = a->rp[i]; k < a->rp[i + 1]; k++) {
            const float aik = a->v[k];
            const float *x = X + (size_t)a->ci[k] * m;
            for (j = 0; j < m; j++) y[j] += aik * x[j];
        }
    }
}

static void fresidual(const fcsr *a, int m, const float *B, const float *X, float *R)
{
    size_t q, nm = (size_t)a->nr * m;
    fspmm(a, m, X, R);
    for (q = 0; q < nm; q++) R[q] = B[q] - R[q];
}

static void fsmooth(const fws *f, const ohier *h, int l, const smopt *so, int m,
                    const float *b, float *x)
{
    const fcsr *a = &f->A[l];
    const float *dinv = f->dinv[l];
    float *r = f->r[l], *d = f->d[l], *t = f->t[l];
    size_t nm = (size_t)a->nr * m, q;
    int i, j, k;
    if (so->smoother == 0) {
        const float w = (float)so->omega;
        fresidual(a, m, b, x, t);
        for (i = 0; i < a->nr; i++)
            for (j = 0; j < m; j++) x[(size_t)i * m + j] += w * dinv[i] * t[(size_t)i * m + j];
    } else if (so->smoother == 2) {
        /* symmetric l1-hybrid Gauss-Seidel: forward x -> t, backward t -> x */
        int B = so->gs_block, n = a->nr, nblk = (n + B - 1) / B, pass, blk;
        for (pass = 0; pass < 2; pass++) {
            const float *xo = pass ? t : x;
            float *xn = pass ? x : t;
            for (blk = 0; blk < nblk; blk++) {
                int lo = blk * B, hi = lo + B < n ? lo + B : n, s2;
                for (s2 = 0; s2 < hi - lo; s2++) {
                    int ii = pass ? hi - 1 - s2 : lo + s2;
                    double dd = 0.0;
                    const ocsr *a64 = &h->A[l];
                    float dl;
                    for (k = a64->rp[ii]; k < a64->rp[ii + 1]; k++) {
                        int c = a64->ci[k];
                        if (c == ii) dd += a64->v[k];
                        else if (c < lo || c >= hi) dd += fabs(a64->v[k]);
                    }
                    dl = (float)dd;
                    for (j = 0; j < m; j++) {
                        float acc = 0.0f;
                        for (k = a->rp[ii]; k < a->rp[ii + 1]; k++) {
                            int c = a->ci[k];
                            int fresh = c >= lo && c < hi && (pass ? c > ii : c < ii);
                            acc += a->v[k] * (fresh ? xn[(size_t)c * m + j] : xo[(size_t)c * m + j]);
                        }
                        xn[(size_t)ii * m + j] =
                            xo[(size_t)ii * m + j] + (b[(size_t)ii * m + j] - acc) / dl;
                    }
                }
            }
        }
    } else {
        double lo = so->lo_frac * so->hi_frac * h->lmax[l], hi = so->hi_frac * h->lmax[l];
        double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
        double sigma = theta / delta, rho = 1.0 / sigma;
        const float ft = (float)theta;
        fresidual(a, m, b, x, r);
        for (i = 0; i < a->nr; i++)
            for (j = 0; j < m; j++) {
                r[(size_t)i * m + j] *= dinv[i];
                d[(size_t)i * m + j] = r[(size_t)i * m + j] / ft;
            }
        for (k = 1; k <= so->degree; k++) {
            for (q = 0; q < nm; q++) x[q] += d[q];
            if (k < so->degree) {
                double rn = 1.0 / (2.0 * sigma - rho);
                const float c1 = (float)(rn * rho), c2 = (float)(2.0 * rn / delta);
                fspmm(a, m, d, t);
                for (i = 0; i < a->nr; i++)
                    for (j = 0; j < m; j++) {
                        size_t p2 = (size_t)i * m + j;
                        r[p2] -= dinv[i] * t[p2];
                        d[p2] = c1 * d[p2] + c2 * r[p2];
                    }
                rho = rn;
            }
        }
    }
}

static void fvcycle_level(const fws *f, const ohier *h, int l, const smopt *so, int m,
                          const float *b, float *x)
{
    size_t nm = (size_t)f->A[l].nr * m, q;
    if (l == f->nlev - 1) {
        int nL = f->A[l].nr, i, k, j;
        for (i = 0; i < nL; i++)
            for (j = 0; j < m; j++) {
                float acc = 0.0f;
                for (k = 0; k < nL; k++) acc += f->inv[(size_t)i * nL + k] * b[(size_t)k * m + j];
                x[(size_t)i * m + j] = acc;
            }
        return;
    }
    memset(x, 0, nm * sizeof(float));
    fsmooth(f, h, l, so, m, b, x);
    fresidual(&f->A[l], m, b, x, f->r[l]);
    fspmm(&f->R[l], m, f->r[l], f->b[l + 1]);
    fvcycle_level(f, h, l + 1, so, m, f->b[l + 1], f->x[l + 1]);
    fspmm(&f->P[l], m, f->x[l + 1], f->t[l]);
    for (q = 0; q < nm; q++) x[q] += f->t[l][q];
    fsmooth(f, h, l, so, m, b, x);
}

int orc_vcycle32(const ohier *h, int smoother, double omega, int degree, double lo_frac,
                 double hi_frac, int gs_block, int m, const double *b, double *x)
{
    fws f;
    smopt so = {smoother, omega, degree, lo_frac, hi_frac, gs_block};
    int l, i, k, nL = h->A[h->nlev - 1].nr, rc = ORC_OK;
    size_t n0 = (size_t)h->A[0].nr * m, q;
    float *b0, *x0;
    double *col;
    if (smoother == 2 && gs_block < 1) return ORC_EINVAL;
    memset(&f, 0, sizeof(f));
    f.nlev = h->nlev; f.m = m;
    for (l = 0; l < h->nlev; l++) {
        size_t nm = (size_t)h->A[l].nr * m + 1;
        fcsr_of(&h->A[l], &f.A[l]);
        if (l + 1 < h->nlev) { fcsr_of(&h->P[l], &f.P[l]); fcsr_of(&h->R[l], &f.R[l]); }
        f.dinv[l] = f_of(h->dinv[l], (size_t)h->A[l].nr);
        f.b[l] = (float *)calloc(nm, sizeof(float));
        f.x[l] = (float *)calloc(nm, sizeof(float));
        f.r[l] = (float *)calloc(nm, sizeof(float));
        f.d[l] = (float *)calloc(nm, sizeof(float));
        f.t[l] = (float *)calloc(nm, sizeof(float));
    }
    /* inverse of the coarsest matrix: LU solves against unit vectors (FP64) */
    f.inv = (float *)malloc(((size_t)nL * nL + 1) * sizeof(float));
    col = (double *)malloc(((size_t)nL + 1) * sizeof(double));
    for (k = 0; k < nL; k++) {
        for (i = 0; i < nL; i++) col[i] = (i == k) ? 1.0 : 0.0;
        dense_lu_solve(nL, h->lu, h->piv, col);
        for (i = 0; i < nL; i++) f.inv[(size_t)i * nL + k] = (float)col[i];
    }
    free(col);
    b0 = f_of(b, n0);
    x0 = (float *)calloc(n0 + 1, sizeof(float));
    fvcycle_level(&f, h, 0, &so, m, b0, x0);
    for (q = 0; q < n0; q++) x[q] = (double)x0[q];
    free(b0); free(x0); free(f.inv);
    for (l = 0; l < h->nlev; l++) {
        free(f.A[l].v); free(f.P[l].v); free(f.R[l].v); free(f.dinv[l]);
        free(f.b[l]); free(f.x[l]); free(f.r[l]); free(f.d[l]); free(f.t[l]);
    }
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Krylov solvers, one independent set of scalars per column.                */
/* Stopping test: ||r_j|| / ||b_j|| <= tol on the recurrence residual; when  */
/* it passes, the true residual of that column is recomputed, and if it does */
/* not pass the column restarts from its current iterate.  A zero column of  */
/* B gives a zero solution in 0 iterations.                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int method;        /* 0 = CG, 1 = BiCGStab */
    int flexible;      /* CG: 0 Fletcher-Reeves beta, 1 flexible (Polak-Ribiere) */
    int max_iters;
    double tol;
    int x0_given;
    int precond;       /* 1 = V-cycle, 0 = none (identity) */
    int merged;        /* CG: 1 = merged form (x's update deferred, see pcg) */
} kopt;

static void apply_prec(const ohier *h, const kopt *ko, const smopt *so, int m,
                       const double *r, double *z, vws *w)
{
    if (ko->precond) vcycle_level(h, 0, so, m, r, z, w);
    else memcpy(z, r, (size_t)h->A[0].nr * m * sizeof(double));
}

/*
 * Preconditioned CG per column (Hestenes-Stiefel; Section 2.1):
 *   r = b - A x, z = M r, p = z;
 *   loop: q = A p, alpha = (r, z)/(p, q), x += alpha p, r -= alpha q,
 *         test ||r||/||b||, z = M r, beta = (r_new, z_new)/(r, z)
 *         (flexible: -alpha (z_new, q)/(r, z)), p = z + beta p.
 * Merged form (ko->merged; Section 2.1's merged formulations regroup the
 * vector updates so fewer passes read and write the vectors): the
 * recurrences and every operation on an element are the same, but x's
 * update of iteration k is postponed into the pass of iteration k + 1 that
 * forms p = z + beta p, which reads the old p anyway (here: the same
 * iteration's last pass, so nothing is pending when the loop ends).  A
 * column's pending alpha is applied before its true residual is formed, so
 * x, and every other result, equals the standard form's.
 */
static void apply_pending_x(int n, int m, const int *only, const double *xp,
                            const double *p, double *X)
{
    int i, j;
#pragma omp parallel for private(j) schedule(static)
    for (i = 0; i < n; i++)
        for (j = 0; j < m; j++)
            if ((only == NULL || only[j]) && xp[j] != 0.0) {
                size_t k = (size_t)i * m + j;
                X[k] += xp[j] * p[k];
            }
}

static int pcg(const ohier *h, const kopt *ko, const smopt *so, int m,
               const double *B, double *X, int *iters, double *relres,
               int *conv, int *restarts, vws *w)
{
    const ocsr *A = &h->A[0];
    int n = A->nr, j, it, i, rc = ORC_OK;
    size_t nm = (size_t)n * m;
    double *r = (double *)malloc(nm * sizeof(double));
    double *z = (double *)malloc(nm * sizeof(double));
    double *p = (double *)malloc(nm * sizeof(double));
    double *q = (double *)malloc(nm * sizeof(double));
    double *bn = (double *)malloc((size_t)m * sizeof(double));
    double *rz = (double *)malloc((size_t)m * sizeof(double));
    double *rzn = (double *)malloc((size_t)m * sizeof(double));
    double *zq = (double *)malloc((size_t)m * sizeof(double));
    double *pq = (double *)malloc((size_t)m * sizeof(double));
    double *rr = (double *)malloc((size_t)m * sizeof(double));
    double *alpha = (double *)malloc((size_t)m * sizeof(double));
    double *beta = (double *)malloc((size_t)m * sizeof(double));
    int *act = (int *)malloc((size_t)m * sizeof(int));
    int *rst = (int *)calloc((size_t)m, sizeof(int));
    double *xp = (double *)calloc((size_t)m, sizeof(double));   /* merged: pending alpha */
    int *one = (int *)calloc((size_t)m, sizeof(int));
    if (!r || !z || !p || !q || !bn || !rz || !rzn || !zq || !pq || !rr || !alpha ||
        !beta || !act || !rst || !xp || !one)
        return ORC_ENOMEM;

    if (!ko->x0_given) memset(X, 0, nm * sizeof(double));
    residual(A, m, B, X, r);
    dots(n, m, B, B, bn);
    dots(n, m, r, r, rr);
    for (j = 0; j < m; j++) {
        bn[j] = sqrt(bn[j]);
        iters[j] = 0; conv[j] = 0; act[j] = 1; restarts[j] = 0;
        if (bn[j] == 0.0) {
            for (i = 0; i < n; i++) X[(size_t)i * m + j] = 0.0;
            relres[j] = 0.0; conv[j] = 1; act[j] = 0;
            continue;
        }
        relres[j] = sqrt(rr[j]) / bn[j];
        if (relres[j] <= ko->tol) { conv[j] = 1; act[j] = 0; }
    }
    apply_prec(h, ko, so, m, r, z, w);
    memcpy(p, z, nm * sizeof(double));
    dots(n, m, r, z, rz);

    for (it = 1; it <= ko->max_iters; it++) {
        int any = 0;
        for (j = 0; j < m; j++) any |= act[j];
        if (!any) break;
        if (g_verbose) { fprintf(stderr, "[oracle] CG iteration %d\n", it); fflush(stderr); }
        /* q = A p, alpha = (r, z) / (p, q) */
        spmm(A, m, p, q);
        dots(n, m, p, q, pq);
        for (j = 0; j < m; j++) {
            alpha[j] = 0.0;
            if (!act[j]) continue;
            if (!(pq[j] > 0.0) || !isfinite(pq[j])) { act[j] = 0; rc = ORC_EBREAKDOWN; continue; }
            alpha[j] = rz[j] / pq[j];
        }
        /* x += alpha p (merged: pending), r -= alpha q (active columns) */
        if (ko->merged)
            for (j = 0; j < m; j++) xp[j] = act[j] ? alpha[j] : 0.0;
#pragma omp parallel for private(j) schedule(static)
        for (i = 0; i < n; i++)
            for (j = 0; j < m; j++)
                if (act[j]) {
                    size_t k = (size_t)i * m + j;
                    if (!ko->merged) X[k] += alpha[j] * p[k];
                    r[k] -= alpha[j] * q[k];
                }
        dots(n, m, r, r, rr);
        for (j = 0; j < m; j++) {
            if (!act[j]) continue;
            iters[j] = it;
            relres[j] = sqrt(rr[j]) / bn[j];
            if (relres[j] <= ko->tol) {
                double tr;
                if (ko->merged) {   /* bring x_j up to date first */
                    one[j] = 1;
                    apply_pending_x(n, m, one, xp, p, X);
                    one[j] = 0;
                    xp[j] = 0.0;
                }
                tr = sqrt(residual_col_norm2(A, m, j, B, X)) / bn[j];
                if (tr <= ko->tol) { conv[j] = 1; act[j] = 0; }
                else {
                    /* recurrence drifted: restart column j from its iterate */
                    for (i = 0; i < n; i++) {
                        double ax = 0.0;
                        int k;
                        for (k = A->rp[i]; k < A->rp[i + 1]; k++)
                            ax += A->v[k] * X[(size_t)A->ci[k] * m + j];
                        r[(size_t)i * m + j] = B[(size_t)i * m + j] - ax;
                    }
                    relres[j] = tr;
                    rst[j] = 1;
                    restarts[j]++;
                }
            }
        }
        /* z = M r, beta, p = z + beta p */
        apply_prec(h, ko, so, m, r, z, w);
        dots(n, m, r, z, rzn);
        if (ko->flexible) dots(n, m, z, q, zq);
        for (j = 0; j < m; j++) {
            beta[j] = 0.0;
            if (!act[j]) continue;
            if (rst[j]) {
                beta[j] = 0.0; rst[j] = 0;
            } else if (ko->flexible) {
                /* (z_new, r_new - r_old) = -alpha (z_new, q) */
                beta[j] = -alpha[j] * zq[j] / rz[j];
            } else {
                beta[j] = rzn[j] / rz[j];
            }
            rz[j] = rzn[j];
        }
        /* merged: the pending x += alpha p_old, before p changes */
        if (ko->merged) {
            apply_pending_x(n, m, NULL, xp, p, X);
            for (j = 0; j < m; j++) xp[j] = 0.0;
        }
#pragma omp parallel for private(j) schedule(static)
        for (i = 0; i < n; i++)
            for (j = 0; j < m; j++)
                if (act[j]) {
                    size_t k = (size_t)i * m + j;
                    p[k] = z[k] + beta[j] * p[k];
                }
    }
    for (j = 0; j < m; j++) if (!conv[j] && rc == ORC_OK) rc = ORC_NOT_CONVERGED;
    free(r); free(z); free(p); free(q); free(bn); free(rz); free(rzn); free(zq);
    free(pq); free(rr); free(alpha); free(beta); free(act); free(rst); free(xp); free(one);
    return rc;
}

/*
 * Right-preconditioned BiCGStab (van der Vorst 1992), per column:
 *   r = b - A x, rh = r, rho = alpha = omega = 1, v = p = 0;
 *   loop: rho' = (rh, r); beta = (rho'/rho)(alpha/omega);
 *         p = r + beta (p - omega v); ph = M p; v = A ph;
 *         alpha = rho' / (rh, v); s = r - alpha v;
 *         if ||s||/||b|| <= tol: x += alpha ph, done;
 *         sh = M s; t = A sh; omega = (t, s)/(t, t);
 *         x += alpha ph + omega sh; r = s - omega t; rho = rho'.
 * Breakdown (|rho'| or |(rh, v)| <= 1e-300 ||b||^2, or omega == 0)
 * restarts the column with rh = r, rho = alpha = omega = 1, p = v = 0; two
 * breakdowns without a completed iteration in between stop the column with
 * ORC_EBREAKDOWN.
 */
static void bicg_reset(int n, int m, int j, const double *r, double *rh, double *p,
                       double *v)
{
    size_t i, k;
    for (i = 0; i < (size_t)n; i++) {
        k = i * m + j;
        rh[k] = r[k]; p[k] = 0.0; v[k] = 0.0;
    }
}

static int bicgstab(const ohier *h, const kopt *ko, const smopt *so, int m,
                    const double *B, double *X, int *iters, double *relres,
                    int *conv, int *restarts, vws *w)
{
    const ocsr *A = &h->A[0];
    int n = A->nr, j, it, rc = ORC_OK;
    size_t nm = (size_t)n * m, k, i;
    double *r = (double *)malloc(nm * sizeof(double));
    double *rh = (double *)malloc(nm * sizeof(double));
    double *p = (double *)calloc(nm, sizeof(double));
    double *v = (double *)calloc(nm, sizeof(double));
    double *ph = (double *)calloc(nm, sizeof(double));
    double *s = (double *)calloc(nm, sizeof(double));
    double *sh = (double *)calloc(nm, sizeof(double));
    double *t = (double *)calloc(nm, sizeof(double));
    double *bn = (double *)malloc((size_t)m * sizeof(double));
    double *rho = (double *)malloc((size_t)m * sizeof(double));
    double *alp = (double *)malloc((size_t)m * sizeof(double));
    double *omg = (double *)malloc((size_t)m * sizeof(double));
    double *beta = (double *)malloc((size_t)m * sizeof(double));
    double *d1 = (double *)malloc((size_t)m * sizeof(double));
    double *d2 = (double *)malloc((size_t)m * sizeof(double));
    int *act = (int *)malloc((size_t)m * sizeof(int));
    int *brk = (int *)calloc((size_t)m, sizeof(int));   /* breakdowns in a row */
    int *rst = (int *)calloc((size_t)m, sizeof(int));   /* restart pending */
    int *skip = (int *)calloc((size_t)m, sizeof(int));  /* rest of iteration skipped */
    int *half = (int *)calloc((size_t)m, sizeof(int));  /* converged at s */
    int *upd = (int *)calloc((size_t)m, sizeof(int));   /* column updated this step */
    if (!r || !rh || !p || !v || !ph || !s || !sh || !t || !bn || !rho || !alp ||
        !omg || !beta || !d1 || !d2 || !act || !brk || !rst || !skip || !half || !upd)
        return ORC_ENOMEM;

    if (!ko->x0_given) memset(X, 0, nm * sizeof(double));
    residual(A, m, B, X, r);
    memcpy(rh, r, nm * sizeof(double));
    dots(n, m, B, B, bn);
    dots(n, m, r, r, d1);
    for (j = 0; j < m; j++) {
        bn[j] = sqrt(bn[j]);
        rho[j] = alp[j] = omg[j] = 1.0;
        iters[j] = 0; conv[j] = 0; act[j] = 1; restarts[j] = 0;
        if (bn[j] == 0.0) {
            for (i = 0; i < (size_t)n; i++) X[i * m + j] = 0.0;
            relres[j] = 0.0; conv[j] = 1; act[j] = 0;
            continue;
        }
        relres[j] = sqrt(d1[j]) / bn[j];
        if (relres[j] <= ko->tol) { conv[j] = 1; act[j] = 0; }
    }

    for (it = 1; it <= ko->max_iters; it++) {
        int any = 0;
        for (j = 0; j < m; j++) any |= act[j];
        if (!any) break;
        if (g_verbose) { fprintf(stderr, "[oracle] BiCGStab iteration %d\n", it); fflush(stderr); }
        /* rho' = (rh, r), beta, p = r + beta (p - omega v) */
        for (j = 0; j < m; j++)
            if (act[j] && rst[j]) {
                bicg_reset(n, m, j, r, rh, p, v);
                rho[j] = alp[j] = omg[j] = 1.0;
                rst[j] = 0;
            }
        dots(n, m, rh, r, d1);
        for (j = 0; j < m; j++) {
            double tiny;
            upd[j] = 0;
            if (!act[j]) continue;
            tiny = 1e-300 * bn[j] * bn[j];
            if (fabs(d1[j]) <= tiny) {
                if (++brk[j] >= 2) { act[j] = 0; rc = ORC_EBREAKDOWN; continue; }
                bicg_reset(n, m, j, r, rh, p, v);
                rho[j] = alp[j] = omg[j] = 1.0;
                d1[j] = dot_col(n, m, j, rh, r);
                restarts[j]++;
            }
            beta[j] = (d1[j] / rho[j]) * (alp[j] / omg[j]);
            rho[j] = d1[j];
            upd[j] = 1;
        }
#pragma omp parallel for private(j, k) schedule(static)
        for (i = 0; i < (size_t)n; i++)
            for (j = 0; j < m; j++)
                if (upd[j]) {
                    k = i * m + j;
                    p[k] = r[k] + beta[j] * (p[k] - omg[j] * v[k]);
                }
        apply_prec(h, ko, so, m, p, ph, w);
        spmm(A, m, ph, v);
        /* alpha = rho' / (rh, v), s = r - alpha v */
        dots(n, m, rh, v, d1);
        for (j = 0; j < m; j++) {
            double tiny;
            upd[j] = 0;
            if (!act[j]) continue;
            iters[j] = it;
            tiny = 1e-300 * bn[j] * bn[j];
            if (fabs(d1[j]) <= tiny) {
                if (++brk[j] >= 2) { act[j] = 0; rc = ORC_EBREAKDOWN; continue; }
                rst[j] = 1; skip[j] = 1;
                restarts[j]++;
                continue;
            }
            alp[j] = rho[j] / d1[j];
            upd[j] = 1;
        }
#pragma omp parallel for private(j, k) schedule(static)
        for (i = 0; i < (size_t)n; i++)
            for (j = 0; j < m; j++)
                if (upd[j]) {
                    k = i * m + j;
                    s[k] = r[k] - alp[j] * v[k];
                }
        dots(n, m, s, s, d2);
        for (j = 0; j < m; j++)
            if (upd[j] && sqrt(d2[j]) / bn[j] <= ko->tol) {
                for (i = 0; i < (size_t)n; i++) {
                    k = i * m + j;
                    X[k] += alp[j] * ph[k];
                    r[k] = s[k];
                }
                half[j] = 1;
            }
        apply_prec(h, ko, so, m, s, sh, w);
        spmm(A, m, sh, t);
        /* omega = (t, s)/(t, t); x += alpha ph + omega sh; r = s - omega t */
        dots(n, m, t, s, d1);
        dots(n, m, t, t, d2);
        for (j = 0; j < m; j++) {
            upd[j] = 0;
            if (!act[j]) continue;
            if (skip[j] || half[j]) continue;
            omg[j] = (d2[j] > 0.0) ? d1[j] / d2[j] : 0.0;
            upd[j] = 1;
        }
#pragma omp parallel for private(j, k) schedule(static)
        for (i = 0; i < (size_t)n; i++)
            for (j = 0; j < m; j++)
                if (upd[j]) {
                    k = i * m + j;
                    X[k] += alp[j] * ph[k] + omg[j] * sh[k];
                    r[k] = s[k] - omg[j] * t[k];
                }
        dots(n, m, r, r, d1);
        for (j = 0; j < m; j++) {
            if (!act[j]) continue;
            if (skip[j]) { skip[j] = 0; continue; }
            if (upd[j]) {
                if (omg[j] == 0.0) {
                    if (++brk[j] >= 2) { act[j] = 0; rc = ORC_EBREAKDOWN; continue; }
                    rst[j] = 1;
                    restarts[j]++;
                } else {
                    brk[j] = 0;
                }
            }
            relres[j] = sqrt(d1[j]) / bn[j];
            if (half[j] || relres[j] <= ko->tol) {
                double tr = sqrt(residual_col_norm2(A, m, j, B, X)) / bn[j];
                half[j] = 0;
                if (tr <= ko->tol) { conv[j] = 1; act[j] = 0; }
                else {
                    /* recurrence drifted: restart column j from its iterate */
                    for (i = 0; i < (size_t)n; i++) {
                        double ax = 0.0;
                        int kk;
                        for (kk = A->rp[i]; kk < A->rp[i + 1]; kk++)
                            ax += A->v[kk] * X[(size_t)A->ci[kk] * m + j];
                        r[i * m + j] = B[i * m + j] - ax;
                    }
                    relres[j] = tr;
                    rst[j] = 1;
                    restarts[j]++;
                }
            }
        }
    }
    for (j = 0; j < m; j++) if (!conv[j] && rc == ORC_OK) rc = ORC_NOT_CONVERGED;
    free(r); free(rh); free(p); free(v); free(ph); free(s); free(sh); free(t);
    free(bn); free(rho); free(alp); free(omg); free(beta); free(d1); free(d2);
    free(act); free(brk); free(rst); free(skip); free(half); free(upd);
    return rc;
}

/*
 * Pipelined BiCGStab (Cools and Vanroose, Parallel Computing 2017; Section
 * 2.1 lists it), right-preconditioned: the BiCGStab above on K = A M,
 * rewritten so that neither product with K in an iteration waits for a dot
 * product.  With s = K p, z = K s, v = K z, w = K r, t = K w, q = r - alpha s
 * (BiCGStab's s) and y = K q, every vector follows from a recurrence:
 *   p = r + beta (p - omega s),  s = w + beta (s - omega z),
 *   z = t + beta (z - omega v),  q = r - alpha s,  y = w - alpha z,
 *   [v = K z],  omega = (q, y) / (y, y),
 *   r' = q - omega y,  w' = y - omega (t - alpha v),  [t' = K w'],
 *   beta' = (alpha / omega) (rh, r') / (rh, r),
 *   alpha' = (rh, r') / ((rh, w') + beta' (rh, s) - beta' omega (rh, z)).
 * x follows the M-images of the same recurrences (the V-cycle inside each
 * product with K already yields zh = M z and wh = M w; rt = M r):
 *   ph = rt + beta (ph - omega sh),  sh = wh + beta (sh - omega zh),
 *   qh = rt - alpha sh,  x += alpha ph + omega qh,
 *   rt' = qh - omega (wh - alpha zh).
 * In exact arithmetic the iterates are those of BiCGStab.  Start, and
 * restart of a column from its iterate: rh = r, rt = M r, w = A rt,
 * wh = M w, t = A wh, alpha = (rh, r) / (rh, w), beta = 0.  A column
 * converges at the half step as in BiCGStab (||q|| <= tol ||b||:
 * x += alpha ph).  A breakdown (|(rh, r)| or the denominator of alpha
 * <= 1e-300 ||b||^2, or omega = 0) stops the column with ORC_EBREAKDOWN:
 * restarting it would take two more products with K for that column alone.
 */
static void col_copy(int n, int m, int j, const double *src, double *dst)
{
    size_t i;
    for (i = 0; i < (size_t)n; i++) dst[i * m + j] = src[i * m + j];
}

typedef struct {
    double *r, *rh, *rt, *w, *wh, *t, *p, *s, *z, *v, *ph, *sh, *zh, *q, *y, *qh, *ta, *tb;
} pbvec;

/* (re)start the columns with mask[j]: rh = r, rt = M r, w = A rt, wh = M w,
 * t = A wh, p = s = z = v = ph = sh = zh = 0, alpha, beta = 0.  The products
 * run over every column; only the masked ones take the results. */
static void pb_start_cols(const ohier *h, const kopt *ko, const smopt *so, int m,
                          const int *mask, pbvec *V, double *bn, double *rho, double *alp,
                          double *omg, double *beta, int *act, int *rc, vws *w)
{
    const ocsr *A = &h->A[0];
    int n = A->nr, j;
    double d1, d2, tiny;
    apply_prec(h, ko, so, m, V->r, V->ta, w);
    for (j = 0; j < m; j++) if (mask[j]) col_copy(n, m, j, V->ta, V->rt);
    spmm(A, m, V->rt, V->tb);
    for (j = 0; j < m; j++) if (mask[j]) col_copy(n, m, j, V->tb, V->w);
    apply_prec(h, ko, so, m, V->w, V->ta, w);
    for (j = 0; j < m; j++) if (mask[j]) col_copy(n, m, j, V->ta, V->wh);
    spmm(A, m, V->wh, V->tb);
    for (j = 0; j < m; j++) {
        size_t i, k;
        if (!mask[j]) continue;
        col_copy(n, m, j, V->tb, V->t);
        col_copy(n, m, j, V->r, V->rh);
        for (i = 0; i < (size_t)n; i++) {
            k = i * m + j;
            V->p[k] = V->s[k] = V->z[k] = V->v[k] = V->ph[k] = V->sh[k] = V->zh[k] = 0.0;
        }
        d1 = dot_col(n, m, j, V->rh, V->r);
        d2 = dot_col(n, m, j, V->rh, V->w);
        tiny = 1e-300 * bn[j] * bn[j];
        if (fabs(d1) <= tiny || fabs(d2) <= tiny) { act[j] = 0; *rc = ORC_EBREAKDOWN; continue; }
        rho[j] = d1;
        alp[j] = d1 / d2;
        beta[j] = 0.0;
        omg[j] = 1.0;
    }
}

static int pbicgstab(const ohier *h, const kopt *ko, const smopt *so, int m,
                     const double *B, double *X, int *iters, double *relres,
                     int *conv, int *restarts, vws *w)
{
    const ocsr *A = &h->A[0];
    int n = A->nr, j, it, rc = ORC_OK, bad = 0;
    size_t nm = (size_t)n * m, i, k;
    pbvec V;
    double **all[] = {&V.r, &V.rh, &V.rt, &V.w, &V.wh, &V.t, &V.p, &V.s, &V.z, &V.v, &V.ph,
                      &V.sh, &V.zh, &V.q, &V.y, &V.qh, &V.ta, &V.tb};
    double *bn = (double *)malloc((size_t)m * sizeof(double));
    double *rho = (double *)malloc((size_t)m * sizeof(double));
    double *alp = (double *)malloc((size_t)m * sizeof(double));
    double *omg = (double *)malloc((size_t)m * sizeof(double));
    double *beta = (double *)malloc((size_t)m * sizeof(double));
    double *qq = (double *)malloc((size_t)m * sizeof(double));
    double *qy = (double *)malloc((size_t)m * sizeof(double));
    double *yy = (double *)malloc((size_t)m * sizeof(double));
    double *rs = (double *)malloc((size_t)m * sizeof(double));
    double *rz = (double *)malloc((size_t)m * sizeof(double));
    double *rr = (double *)malloc((size_t)m * sizeof(double));
    double *rhr = (double *)malloc((size_t)m * sizeof(double));
    double *rhw = (double *)malloc((size_t)m * sizeof(double));
    int *act = (int *)malloc((size_t)m * sizeof(int));
    int *half = (int *)calloc((size_t)m, sizeof(int));
    int *full = (int *)calloc((size_t)m, sizeof(int));   /* takes the omega step */
    int *rst = (int *)calloc((size_t)m, sizeof(int));    /* restart from its iterate */
    for (j = 0; j < (int)(sizeof(all) / sizeof(all[0])); j++) {
        *all[j] = (double *)calloc(nm + 1, sizeof(double));
        bad |= *all[j] == NULL;
    }
    if (bad || !bn || !rho || !alp || !omg || !beta || !qq || !qy || !yy || !rs || !rz || !rr ||
        !rhr || !rhw || !act || !half || !full || !rst)
        return ORC_ENOMEM;

    if (!ko->x0_given) memset(X, 0, nm * sizeof(double));
    residual(A, m, B, X, V.r);
    dots(n, m, B, B, bn);
    dots(n, m, V.r, V.r, rr);
    for (j = 0; j < m; j++) {
        bn[j] = sqrt(bn[j]);
        iters[j] = 0; conv[j] = 0; act[j] = 1; restarts[j] = 0;
        if (bn[j] == 0.0) {
            for (i = 0; i < (size_t)n; i++) X[i * m + j] = 0.0;
            relres[j] = 0.0; conv[j] = 1; act[j] = 0;
            continue;
        }
        relres[j] = sqrt(rr[j]) / bn[j];
        if (relres[j] <= ko->tol) { conv[j] = 1; act[j] = 0; }
    }
    pb_start_cols(h, ko, so, m, act, &V, bn, rho, alp, omg, beta, act, &rc, w);

    for (it = 1; it <= ko->max_iters; it++) {
        int any = 0;
        for (j = 0; j < m; j++) any |= act[j];
        if (!any) break;
        if (g_verbose) { fprintf(stderr, "[oracle] pipelined BiCGStab iteration %d\n", it); fflush(stderr); }
        /* the recurrences of p, s, z (and ph, sh) from their old values; q, y, qh */
#pragma omp parallel for private(j, k) schedule(static)
        for (i = 0; i < (size_t)n; i++)
            for (j = 0; j < m; j++)
                if (act[j]) {
                    double po, so_, zo, pho, sho;
                    k = i * m + j;
                    po = V.p[k]; so_ = V.s[k]; zo = V.z[k]; pho = V.ph[k]; sho = V.sh[k];
                    V.p[k] = V.r[k] + beta[j] * (po - omg[j] * so_);
                    V.s[k] = V.w[k] + beta[j] * (so_ - omg[j] * zo);
                    V.z[k] = V.t[k] + beta[j] * (zo - omg[j] * V.v[k]);
                    V.ph[k] = V.rt[k] + beta[j] * (pho - omg[j] * sho);
                    V.sh[k] = V.wh[k] + beta[j] * (sho - omg[j] * V.zh[k]);
                    V.q[k] = V.r[k] - alp[j] * V.s[k];
                    V.y[k] = V.w[k] - alp[j] * V.z[k];
                    V.qh[k] = V.rt[k] - alp[j] * V.sh[k];
                }
        dots(n, m, V.q, V.q, qq);
        dots(n, m, V.q, V.y, qy);
        dots(n, m, V.y, V.y, yy);
        dots(n, m, V.rh, V.s, rs);
        dots(n, m, V.rh, V.z, rz);
        for (j = 0; j < m; j++) {
            half[j] = full[j] = rst[j] = 0;
            if (!act[j]) continue;
            iters[j] = it;
            if (sqrt(qq[j]) / bn[j] <= ko->tol) { half[j] = 1; continue; }
            omg[j] = yy[j] > 0.0 ? qy[j] / yy[j] : 0.0;
            if (omg[j] == 0.0) { act[j] = 0; rc = ORC_EBREAKDOWN; continue; }
            full[j] = 1;
        }
        /* v = K z: zh = M z, v = A zh */
        apply_prec(h, ko, so, m, V.z, V.zh, w);
        spmm(A, m, V.zh, V.v);
#pragma omp parallel for private(j, k) schedule(static)
        for (i = 0; i < (size_t)n; i++)
            for (j = 0; j < m; j++) {
                k = i * m + j;
                if (half[j]) {
                    X[k] += alp[j] * V.ph[k];
                    V.r[k] = V.q[k];
                } else if (full[j]) {
                    X[k] += alp[j] * V.ph[k] + omg[j] * V.qh[k];
                    V.r[k] = V.q[k] - omg[j] * V.y[k];
                    V.w[k] = V.y[k] - omg[j] * (V.t[k] - alp[j] * V.v[k]);
                    V.rt[k] = V.qh[k] - omg[j] * (V.wh[k] - alp[j] * V.zh[k]);
                }
            }
        /* t = K w: wh = M w, t = A wh */
        apply_prec(h, ko, so, m, V.w, V.wh, w);
        spmm(A, m, V.wh, V.t);
        dots(n, m, V.r, V.r, rr);
        dots(n, m, V.rh, V.r, rhr);
        dots(n, m, V.rh, V.w, rhw);
        for (j = 0; j < m; j++) {
            double tiny, del;
            if (!half[j] && !full[j]) continue;
            relres[j] = sqrt(rr[j]) / bn[j];
            if (half[j] || relres[j] <= ko->tol) {
                double tr = sqrt(residual_col_norm2(A, m, j, B, X)) / bn[j];
                if (tr <= ko->tol) { conv[j] = 1; act[j] = 0; }
                else {
                    /* recurrence drifted: restart column j from its iterate */
                    for (i = 0; i < (size_t)n; i++) {
                        double ax = 0.0;
                        int kk;
                        for (kk = A->rp[i]; kk < A->rp[i + 1]; kk++)
                            ax += A->v[kk] * X[(size_t)A->ci[kk] * m + j];
                        V.r[i * m + j] = B[i * m + j] - ax;
                    }
                    relres[j] = tr;
                    rst[j] = 1;
                    restarts[j]++;
                }
                continue;
            }
            tiny = 1e-300 * bn[j] * bn[j];
            beta[j] = (alp[j] / omg[j]) * (rhr[j] / rho[j]);
            del = rhw[j] + beta[j] * rs[j] - beta[j] * omg[j] * rz[j];
            if (fabs(rhr[j]) <= tiny || fabs(del) <= tiny) { act[j] = 0; rc = ORC_EBREAKDOWN; continue; }
            alp[j] = rhr[j] / del;
            rho[j] = rhr[j];
        }
        any = 0;
        for (j = 0; j < m; j++) any |= rst[j];
        if (any) pb_start_cols(h, ko, so, m, rst, &V, bn, rho, alp, omg, beta, act, &rc, w);
    }
    for (j = 0; j < m; j++) if (!conv[j] && rc == ORC_OK) rc = ORC_NOT_CONVERGED;
    for (j = 0; j < (int)(sizeof(all) / sizeof(all[0])); j++) free(*all[j]);
    free(bn); free(rho); free(alp); free(omg); free(beta); free(qq); free(qy); free(yy);
    free(rs); free(rz); free(rr); free(rhr); free(rhw); free(act); free(half); free(full);
    free(rst);
    return rc;
}

/*
 * Multigrid as a standalone solver (Section 2.1, Table 1 lists MultiGrid as
 * a solver as well as a preconditioner): the stationary iteration
 *   x <- x + V(b - A x),
 * V the V(1,1) cycle, per column until ||b - A x|| / ||b|| <= tol.  The
 * residual is recomputed from x every iteration (it is the true residual);
 * converged columns stay frozen.
 */
static int mgsolve(const ohier *h, const kopt *ko, const smopt *so, int m,
                   const double *B, double *X, int *iters, double *relres, int *conv,
                   int *restarts, vws *w)
{
    const ocsr *A = &h->A[0];
    int n = A->nr, j, it, i;
    size_t nm = (size_t)n * m;
    double *r = (double *)malloc(nm * sizeof(double) + 8);
    double *z = (double *)malloc(nm * sizeof(double) + 8);
    double *bn = (double *)malloc((size_t)m * sizeof(double));
    double *rr = (double *)malloc((size_t)m * sizeof(double));
    int *act = (int *)malloc((size_t)m * sizeof(int));
    if (!r || !z || !bn || !rr || !act) return ORC_ENOMEM;

    if (!ko->x0_given) memset(X, 0, nm * sizeof(double));
    residual(A, m, B, X, r);
    dots(n, m, B, B, bn);
    dots(n, m, r, r, rr);
    for (j = 0; j < m; j++) {
        bn[j] = sqrt(bn[j]);
        iters[j] = 0; conv[j] = 0; act[j] = 1; restarts[j] = 0;
        if (bn[j] == 0.0) {
            for (i = 0; i < n; i++) X[(size_t)i * m + j] = 0.0;
            relres[j] = 0.0; conv[j] = 1; act[j] = 0;
            continue;
        }
        relres[j] = sqrt(rr[j]) / bn[j];
        if (relres[j] <= ko->tol) { conv[j] = 1; act[j] = 0; }
    }
    for (it = 1; it <= ko->max_iters; it++) {
        int any = 0;
        for (j = 0; j < m; j++) any |= act[j];
        if (!any) break;
        if (g_verbose) { fprintf(stderr, "[oracle] MG iteration %d\n", it); fflush(stderr); }
        apply_prec(h, ko, so, m, r, z, w);
#pragma omp parallel for private(j) schedule(static)
        for (i = 0; i < n; i++)
            for (j = 0; j < m; j++)
                if (act[j]) X[(size_t)i * m + j] += z[(size_t)i * m + j];
        residual(A, m, B, X, r);
        dots(n, m, r, r, rr);
        for (j = 0; j < m; j++) {
            if (!act[j]) continue;
            iters[j] = it;
            relres[j] = sqrt(rr[j]) / bn[j];
            if (relres[j] <= ko->tol) { conv[j] = 1; act[j] = 0; }
        }
    }
    free(r); free(z); free(bn); free(rr); free(act);
    for (j = 0; j < m; j++) if (!conv[j]) return ORC_NOT_CONVERGED;
    return ORC_OK;
}

/*
 * Solve A X = B (A = level 0 of h).  X is the initial guess when x0_given,
 * the solution on return.  Per-column outputs: iterations, recurrence
 * relative residual, true relative residual, converged flag, and restarts
 * (breakdown restarts plus true-residual restarts of the column).
 */
int orc_solve(const ohier *h, int method, int smoother, double omega, int degree,
              double lo_frac, double hi_frac, int gs_block, int flexible, int precond,
              int merged, int max_iters, double tol, int x0_given, int m, const double *B,
              double *X, int *iters, double *relres, double *true_relres, int *conv,
              int *restarts)
{
    vws w;
    kopt ko = {method, flexible, max_iters, tol, x0_given, precond, merged};
    smopt so = {smoother, omega, degree, lo_frac, hi_frac, gs_block};
    int rc, j, n = h->A[0].nr;
    size_t q, nm = (size_t)n * m;
    double *t;
    if (m < 1 || (smoother == 2 && gs_block < 1)) return ORC_EINVAL;
    for (q = 0; q < nm; q++) if (!isfinite(B[q])) return ORC_EINVAL;
    if (vws_alloc(&w, h, m)) { vws_free(&w, h->nlev); return ORC_ENOMEM; }
    if (method == 0) rc = pcg(h, &ko, &so, m, B, X, iters, relres, conv, restarts, &w);
    else if (method == 2) rc = mgsolve(h, &ko, &so, m, B, X, iters, relres, conv, restarts, &w);
    else if (method == 3) rc = pbicgstab(h, &ko, &so, m, B, X, iters, relres, conv, restarts, &w);
    else rc = bicgstab(h, &ko, &so, m, B, X, iters, relres, conv, restarts, &w);
    vws_free(&w, h->nlev);
    t = (double *)malloc(nm * sizeof(double));
    if (!t) return ORC_ENOMEM;
    residual(&h->A[0], m, B, X, t);
    {
        double *bb = (double *)malloc((size_t)m * sizeof(double));
        double *tt = (double *)malloc((size_t)m * sizeof(double));
        dots(n, m, B, B, bb);
        dots(n, m, t, t, tt);
        for (j = 0; j < m; j++)
            true_relres[j] = bb[j] > 0.0 ? sqrt(tt[j]) / sqrt(bb[j]) : 0.0;
        free(bb); free(tt);
    }
    free(t);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Single operations on caller CSR arrays, for the tests.                    */
/* ------------------------------------------------------------------------ */
void orc_spmm(int n, int ncols, const int *rp, const int *ci, const double *v, int m,
              const double *X, double *Y)
{
    ocsr a;
    a.nr = n; a.nc = ncols; a.rp = (int *)rp; a.ci = (int *)ci; a.v = (double *)v;
    spmm(&a, m, X, Y);
}

void orc_jacobi(int n, const int *rp, const int *ci, const double *v,
                const double *dinv, double omega, int m, const double *b, double *x)
{
    ocsr a;
    double *t = (double *)malloc((size_t)n * m * sizeof(double) + 8);
    a.nr = n; a.nc = n; a.rp = (int *)rp; a.ci = (int *)ci; a.v = (double *)v;
    jacobi(&a, dinv, omega, m, b, x, t);
    free(t);
}

void orc_chebyshev(int n, const int *rp, const int *ci, const double *v,
                   const double *dinv, double lo, double hi, int degree, int m,
                   const double *b, double *x)
{
    ocsr a;
    size_t nm = (size_t)n * m + 1;
    double *r = (double *)malloc(nm * sizeof(double));
    double *d = (double *)malloc(nm * sizeof(double));
    double *t = (double *)malloc(nm * sizeof(double));
    a.nr = n; a.nc = n; a.rp = (int *)rp; a.ci = (int *)ci; a.v = (double *)v;
    chebyshev(&a, dinv, lo, hi, degree, m, b, x, r, d, t);
    free(r); free(d); free(t);
}

void orc_hgs_sweep(int n, const int *rp, const int *ci, const double *v, int B,
                   int backward, int m, const double *b, const double *xo, double *xn)
{
    ocsr a;
    a.nr = n; a.nc = n; a.rp = (int *)rp; a.ci = (int *)ci; a.v = (double *)v;
    hgs_sweep(&a, B, backward, m, b, xo, xn);
}

double orc_lanczos(int n, const int *rp, const int *ci, const double *v, int steps,
                   unsigned long long key)
{
    ocsr a;
    a.nr = n; a.nc = n; a.rp = (int *)rp; a.ci = (int *)ci; a.v = (double *)v;
    return lanczos_lmax(&a, steps, (uint64_t)key);
}

double orc_sm64_uniform(unsigned long long key, unsigned long long i)
{
    return sm64_uniform((uint64_t)key, (uint64_t)i);
}

/* dense LU solve of an n x n row-major system, m columns of b (n x m) */
int orc_dense_solve(int n, const double *a, int m, double *b)
{
    double *lu = (double *)malloc((size_t)n * n * sizeof(double) + 8);
    int *piv = (int *)malloc((size_t)n * sizeof(int) + 4);
    double *col = (double *)malloc((size_t)n * sizeof(double) + 8);
    int i, j, rc = 0;
    memcpy(lu, a, (size_t)n * n * sizeof(double));
    if (dense_lu(n, lu, piv)) rc = ORC_EBREAKDOWN;
    else
        for (j = 0; j < m; j++) {
            for (i = 0; i < n; i++) col[i] = b[(size_t)i * m + j];
            dense_lu_solve(n, lu, piv, col);
            for (i = 0; i < n; i++) b[(size_t)i * m + j] = col[i];
        }
    free(lu); free(piv); free(col);
    return rc;
}

/* strength pattern and RS split of a caller matrix (for pin tests) */
int orc_rs_split(int n, const int *rp, const int *ci, const double *v, double theta,
                 int *state)
{
    ocsr a;
    int *srp, *sci, *trp, *tci, rc;
    a.nr = n; a.nc = n; a.rp = (int *)rp; a.ci = (int *)ci; a.v = (double *)v;
    if (strength(&a, theta, &srp, &sci)) return ORC_ENOMEM;
    if (pattern_transpose(n, srp, sci, &trp, &tci)) return ORC_ENOMEM;
    rc = rs_first_pass(n, srp, sci, trp, tci, state);
    free(srp); free(sci); free(trp); free(tci);
    return rc ? ORC_ENOMEM : ORC_OK;
}

/* C/F split of the aggressive coarsening (first pass, then the second pass
 * over the C points on their distance-two strength) */
int orc_agg_split(int n, const int *rp, const int *ci, const double *v, double theta,
                  int num_paths, int *state)
{
    ocsr a;
    int *srp, *sci, *trp, *tci, rc;
    a.nr = n; a.nc = n; a.rp = (int *)rp; a.ci = (int *)ci; a.v = (double *)v;
    if (strength(&a, theta, &srp, &sci)) return ORC_ENOMEM;
    if (pattern_transpose(n, srp, sci, &trp, &tci)) return ORC_ENOMEM;
    rc = rs_first_pass(n, srp, sci, trp, tci, state) ||
         aggressive_second_pass(n, srp, sci, num_paths, state);
    free(srp); free(sci); free(trp); free(tci);
    return rc ? ORC_ENOMEM : ORC_OK;
}

int orc_strength_count(int n, const int *rp, const int *ci, const double *v,
                       double theta, int *counts)
{
    ocsr a;
    int *srp, *sci, i;
    a.nr = n; a.nc = n; a.rp = (int *)rp; a.ci = (int *)ci; a.v = (double *)v;
    if (strength(&a, theta, &srp, &sci)) return ORC_ENOMEM;
    for (i = 0; i < n; i++) counts[i] = srp[i + 1] - srp[i];
    free(srp); free(sci);
    return ORC_OK;
}

/* threads the OpenMP row loops use (1 without OpenMP) */
#ifdef _OPENMP
#include <omp.h>
#endif
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ======================================================================== */
/* Learned warm start: a bias-free 3D convolutional network (test oracle).  */
/* Volumes are N^3 grids, voxel r = x + N y + N^2 z, channels last:          */
/* a[r*C + c].  A layer is a 3x3x3 cross-correlation with zero padding:      */
/*   out[r, co] = sum_t sum_ci W[co][ci][t] in[r + off(t), ci],              */
/* tap t = (dz+1)*9 + (dy+1)*3 + (dx+1), off(t) = dx + N dy + N^2 dz, terms  */
/* with a neighbour outside the grid are zero.  FP64 throughout; callers    */
/* pass operands already rounded to BF16 when they compare with a BF16 path. */
/* ======================================================================== */
static int nbr_of(int N, long r, int t, long *u)
{
    int x = (int)(r % N), y = (int)((r / N) % N), z = (int)(r / ((long)N * N));
    int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    int xx = x + dx, yy = y + dy, zz = z + dz;
    if (xx < 0 || xx >= N || yy < 0 || yy >= N || zz < 0 || zz >= N) return 0;
    *u = r + dx + (long)N * dy + (long)N * N * dz;
    return 1;
}

/* forward: out (n x cout) from in (n x cin), W [cout][cin][27] */
void orc_conv3d_fwd(int N, int cin, int cout, const double *in, const double *W, double *out)
{
    long n = (long)N * N * N, r;
#pragma omp parallel for schedule(static)
    for (r = 0; r < n; r++) {
        int co, ci, t;
        for (co = 0; co < cout; co++) {
            double s = 0.0;
            for (t = 0; t < 27; t++) {
                long u;
                if (!nbr_of(N, r, t, &u)) continue;
                for (ci = 0; ci < cin; ci++)
                    s += W[((long)co * cin + ci) * 27 + t] * in[u * cin + ci];
            }
            out[r * cout + co] = s;
        }
    }
}

/* input gradient: din[r, ci] = sum_t sum_co W[co][ci][t] g[r - off(t), co]
 * (the adjoint of the forward map) */
void orc_conv3d_dgrad(int N, int cin, int cout, const double *g, const double *W, double *din)
{
    long n = (long)N * N * N, r;
#pragma omp parallel for schedule(static)
    for (r = 0; r < n; r++) {
        int co, ci, t;
        for (ci = 0; ci < cin; ci++) din[r * cin + ci] = 0.0;
        for (t = 0; t < 27; t++) {
            long u;
            /* r = u + off(t)  <=>  u is the neighbour of r at the mirrored tap */
            if (!nbr_of(N, r, 26 - t, &u)) continue;
            for (ci = 0; ci < cin; ci++) {
                double s = 0.0;
                for (co = 0; co < cout; co++)
                    s += W[((long)co * cin + ci) * 27 + t] * g[u * cout + co];
                din[r * cin + ci] += s;
            }
        }
    }
}

/* weight gradient: dW[co][ci][t] = sum_r g[r, co] in[r + off(t), ci] */
void orc_conv3d_wgrad(int N, int cin, int cout, const double *g, const double *in, double *dW)
{
    long n = (long)N * N * N;
    int co, ci, t;
    for (co = 0; co < cout; co++)
        for (ci = 0; ci < cin; ci++)
            for (t = 0; t < 27; t++) {
                double s = 0.0;
                long r, u;
                for (r = 0; r < n; r++)
                    if (nbr_of(N, r, t, &u)) s += g[r * cout + co] * in[u * cin + ci];
                dW[((long)co * cin + ci) * 27 + t] = s;
            }
}

/* round-to-nearest-even of a binary32 value to bfloat16, returned as the
 * double it represents */
double orc_bf16_round(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}
