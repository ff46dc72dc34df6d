/*
 * Drives every entry point of the oracle on small inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).  Exit status
 * 0 means every call returned its expected code; the sanitizers abort the
 * process on the first invalid access or undefined operation.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct ohier ohier;
int orc_build(int n, const int *rp, const int *ci, const double *v, double theta,
              int max_coarse, int max_levels, int lanczos_steps, int agg_levels, int num_paths,
              ohier **out);
void orc_hier_free(ohier *h);
int orc_hier_nlev(const ohier *h);
int orc_hier_info(const ohier *h, int which, int l, int *info);
int orc_hier_copy(const ohier *h, int which, int l, int *rp, int *ci, double *v);
int orc_hier_cf(const ohier *h, int l, int *cf);
double orc_hier_lmax(const ohier *h, int l);
int orc_vcycle(const ohier *h, int smoother, double omega, int degree, double lo_frac,
               double hi_frac, int gs_block, int m, const double *b, double *x);
int orc_solve(const ohier *h, int method, int smoother, double omega, int degree,
              double lo_frac, double hi_frac, int gs_block, int flexible, int precond,
              int merged, int max_iters, double tol, int x0_given, int m, const double *B, double *X,
              int *iters, double *relres, double *true_relres, int *conv, int *restarts);
void orc_spmm(int n, int ncols, const int *rp, const int *ci, const double *v, int m,
              const double *X, double *Y);
void orc_hgs_sweep(int n, const int *rp, const int *ci, const double *v, int B, int backward,
                   int m, const double *b, const double *xo, double *xn);
double orc_lanczos(int n, const int *rp, const int *ci, const double *v, int steps,
                   unsigned long long key);
int orc_rs_split(int n, const int *rp, const int *ci, const double *v, double theta, int *st);
void orc_conv3d_fwd(int N, int cin, int cout, const double *in, const double *W, double *out);
void orc_conv3d_dgrad(int N, int cin, int cout, const double *g, const double *W, double *din);
void orc_conv3d_wgrad(int N, int cin, int cout, const double *g, const double *in, double *dW);

#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); exit(1); } } while (0)

/* 7-point operator on an N^3 grid with per-cell coefficient k (harmonic
 * face means), Dirichlet faces weighted by the cell's own coefficient */
static void stencil(int N, const double *k, int **rp, int **ci, double **v)
{
    int n = N * N * N, nnz = 0, i;
    *rp = malloc((n + 1) * sizeof(int));
    *ci = malloc(7 * n * sizeof(int));
    *v = malloc(7 * n * sizeof(double));
    (*rp)[0] = 0;
    for (i = 0; i < n; i++) {
        int x = i % N, y = (i / N) % N, z = i / (N * N), d;
        int nb[6] = {x > 0 ? i - 1 : -1, x < N - 1 ? i + 1 : -1, y > 0 ? i - N : -1,
                     y < N - 1 ? i + N : -1, z > 0 ? i - N * N : -1, z < N - 1 ? i + N * N : -1};
        int cols[7], c = 0, a, b;
        double vals[7], diag = 0.0;
        for (d = 0; d < 6; d++) {
            double w = nb[d] >= 0 ? 2 * k[i] * k[nb[d]] / (k[i] + k[nb[d]]) : k[i];
            diag += w;
            if (nb[d] >= 0) { cols[c] = nb[d]; vals[c] = -w; c++; }
        }
        cols[c] = i; vals[c] = diag; c++;
        for (a = 1; a < c; a++)          /* sort by column */
            for (b = a; b > 0 && cols[b] < cols[b - 1]; b--) {
                int t = cols[b]; double tv = vals[b];
                cols[b] = cols[b - 1]; vals[b] = vals[b - 1]; cols[b - 1] = t; vals[b - 1] = tv;
            }
        for (a = 0; a < c; a++) { (*ci)[nnz] = cols[a]; (*v)[nnz] = vals[a]; nnz++; }
        (*rp)[i + 1] = nnz;
    }
}

static double urand(unsigned *s) { *s = *s * 1664525u + 1013904223u; return (*s >> 8) / 16777216.0 * 2 - 1; }

static void exercise(int N, double jump, int agg_levels, int num_paths)
{
    int n = N * N * N, m = 3, l, method, smoother, j, rc;
    int *rp, *ci;
    double *v, *k = malloc(n * sizeof(double));
    unsigned seed = 7u + (unsigned)N;
    ohier *h = NULL;
    for (j = 0; j < n; j++) k[j] = (j / 8) % 2 ? jump : 1.0;
    stencil(N, k, &rp, &ci, &v);
    CHECK(orc_build(n, rp, ci, v, 0.25, 20, 40, 10, agg_levels, num_paths, &h) == 0);
    for (l = 0; l < orc_hier_nlev(h); l++) {
        int info[3], w;
        for (w = 0; w < 3; w++) {
            if (orc_hier_info(h, w, l, info)) continue;
            int *r2 = malloc((info[0] + 1) * sizeof(int));
            int *c2 = malloc((info[2] + 1) * sizeof(int));
            double *v2 = malloc((info[2] + 1) * sizeof(double));
            orc_hier_copy(h, w, l, r2, c2, v2);
            free(r2); free(c2); free(v2);
        }
        orc_hier_info(h, 0, l, info);
        int *cf = malloc(info[0] * sizeof(int));
        orc_hier_cf(h, l, cf);
        free(cf);
        CHECK(isfinite(orc_hier_lmax(h, l)) || l == orc_hier_nlev(h) - 1);
    }
    double *B = malloc((size_t)n * m * sizeof(double)), *X = malloc((size_t)n * m * sizeof(double));
    double *Y = malloc((size_t)n * m * sizeof(double)), rr[3], tr[3];
    int it[3], cv[3], rs[3];
    for (j = 0; j < n * m; j++) B[j] = urand(&seed);
    for (j = 0; j < n; j++) B[j * m + 1] = 0.0;         /* a zero column */
    orc_spmm(n, n, rp, ci, v, m, B, Y);
    orc_hgs_sweep(n, rp, ci, v, 8, 0, m, B, Y, X);
    orc_hgs_sweep(n, rp, ci, v, 8, 1, m, B, X, Y);
    CHECK(orc_lanczos(n, rp, ci, v, 10, 7ull << 32) > 0.0);
    int *st = malloc(n * sizeof(int));
    CHECK(orc_rs_split(n, rp, ci, v, 0.25, st) == 0);
    free(st);
    for (smoother = 0; smoother < 3; smoother++)
        CHECK(orc_vcycle(h, smoother, 2.0 / 3.0, 2, 0.3, 1.1, 8, m, B, X) == 0);
    for (method = 0; method < 4; method++)
        for (smoother = 0; smoother < 3; smoother++) {
            rc = orc_solve(h, method, smoother, 2.0 / 3.0, 2, 0.3, 1.1, 8, 0, 1, 0, 200, 1e-8, 0,
                           m, B, X, it, rr, tr, cv, rs);
            CHECK(rc == 0);
            /* merged CG form */
            rc = orc_solve(h, method, smoother, 2.0 / 3.0, 2, 0.3, 1.1, 8, 0, 1, 1, 200, 1e-8, 0,
                           m, B, X, it, rr, tr, cv, rs);
            CHECK(rc == 0);
            /* given initial guess, iteration cap, no preconditioner */
            for (j = 0; j < n * m; j++) X[j] = urand(&seed);
            rc = orc_solve(h, method, smoother, 2.0 / 3.0, 2, 0.3, 1.1, 8, 1, method != 2,
                           method == 0, 1, 1e-14, 1, m, B, X, it, rr, tr, cv, rs);
            CHECK(rc == 1);
        }
    B[5] = NAN;
    CHECK(orc_solve(h, 0, 0, 2.0 / 3.0, 2, 0.3, 1.1, 8, 0, 1, 0, 10, 1e-8, 0, m, B, X, it, rr, tr,
                    cv, rs) == -1);
    orc_hier_free(h);
    free(B); free(X); free(Y); free(k); free(rp); free(ci); free(v);
}

static void cnn(void)
{
    int N = 6, n = N * N * N, i;
    unsigned seed = 3u;
    double *x = malloc(n * 2 * sizeof(double)), *W = malloc(3 * 2 * 27 * sizeof(double));
    double *y = malloc(n * 3 * sizeof(double)), *d = malloc(n * 2 * sizeof(double));
    double *dW = malloc(3 * 2 * 27 * sizeof(double));
    for (i = 0; i < n * 2; i++) x[i] = urand(&seed);
    for (i = 0; i < 3 * 2 * 27; i++) W[i] = urand(&seed);
    orc_conv3d_fwd(N, 2, 3, x, W, y);
    orc_conv3d_dgrad(N, 2, 3, y, W, d);
    orc_conv3d_wgrad(N, 2, 3, y, x, dW);
    free(x); free(W); free(y); free(d); free(dW);
}

int main(void)
{
    exercise(6, 1.0, 0, 1);
    exercise(7, 1000.0, 0, 1);    /* ragged blocks, jump coefficient */
    exercise(9, 1.0, 1, 1);       /* aggressive coarsening, multipass interpolation */
    exercise(9, 1000.0, 2, 2);
    cnn();
    printf("oracle driver ok\n");
    return 0;
}
