/* Runs every oracle routine on small convection-diffusion systems, for a build of the oracle
 * with AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py). Exits
 * non-zero if a routine fails where it must succeed; the sanitizers abort on a memory error or
 * undefined behaviour. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_gs_scale(int n, const int* rp, const int* ci, const double* val, const double* b, int p,
                 double* val_out, double* b_out, double* norm, double* weight);
void orc_spmv(int n, const int* rp, const int* ci, const double* val, const double* x, double* y);
int orc_ilu0(int n, const int* rp, const int* ci, const double* val, double* lu);
int orc_arnoldi(int n, const int* rp, const int* ci, const double* val, const double* r0, int m,
                double* V, double* H, double eps_b);
int orc_gmres(int n, const int* rp, const int* ci, const double* val, const double* b, double* x,
              int m, double tol, int maxit, double eps_b, const double* wts, const double* lu,
              double* hist, int* info_i, double* info_d);
int orc_bicgstab(int n, const int* rp, const int* ci, const double* val, const double* b,
                 double* x, double tol, int maxit, double eps_b, const double* wts,
                 const double* lu, double* hist, int* info_i, double* info_d);
int orc_gmres_ir(int n, const int* rp, const int* ci, const double* val, const double* b,
                 double* x, int m, double tol, int maxit, double eps_b, const double* wts,
                 int* info_i, double* info_d);
int orc_bicgstab_ir(int n, const int* rp, const int* ci, const double* val, const double* b,
                    double* x, double tol, int maxit, double eps_b, const double* wts,
                    double delta, int fallback, int run_cap, int* info_i, double* info_d);
double orc_default_breakdown_eps(void);

/* 5-point convection-diffusion on an N x N grid with a jump of J on the centre square. */
static int build(int N, double J, int** rp_o, int** ci_o, double** val_o, double** b_o) {
    int n = N * N, k = 0;
    int* rp = malloc(sizeof(int) * (n + 1));
    int* ci = malloc(sizeof(int) * 5 * n);
    double* val = malloc(sizeof(double) * 5 * n);
    double* b = malloc(sizeof(double) * n);
    if (!rp || !ci || !val || !b) return 0;
    for (int iy = 0; iy < N; ++iy)
        for (int ix = 0; ix < N; ++ix) {
            int i = iy * N + ix;
            double a = (4 * ix > N && 4 * ix < 3 * N && 4 * iy > N && 4 * iy < 3 * N) ? J : 1.0;
            rp[i] = k;
            if (iy > 0) { ci[k] = i - N; val[k++] = -a - 0.3; }
            if (ix > 0) { ci[k] = i - 1; val[k++] = -a - 0.2; }
            ci[k] = i; val[k++] = 4.0 * a;
            if (ix < N - 1) { ci[k] = i + 1; val[k++] = -a + 0.2; }
            if (iy < N - 1) { ci[k] = i + N; val[k++] = -a + 0.3; }
            b[i] = 1.0 + 0.01 * (i % 7);
        }
    rp[n] = k;
    *rp_o = rp; *ci_o = ci; *val_o = val; *b_o = b;
    return n;
}

#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); return 1; } } while (0)

int main(void) {
    int *rp, *ci;
    double *val, *b;
    const double eps = orc_default_breakdown_eps();
    for (int N = 1; N <= 24; N += 23) {
        int n = build(N, 1e3, &rp, &ci, &val, &b);
        CHECK(n == N * N);
        int nnz = rp[n];
        double* vs = malloc(sizeof(double) * nnz);
        double* bs = malloc(sizeof(double) * n);
        double* nrm = malloc(sizeof(double) * n);
        double* w = malloc(sizeof(double) * n);
        double* x = calloc(n, sizeof(double));
        double* y = malloc(sizeof(double) * n);
        double* lu = malloc(sizeof(double) * nnz);
        double* hist = malloc(sizeof(double) * 10000);
        int m = n < 8 ? n : 8;
        double* V = malloc(sizeof(double) * (size_t)n * (m + 1));
        double* H = malloc(sizeof(double) * (size_t)m * (m + 1));
        int ii[7];
        double dd[2];
        for (int p = 1; p <= 3; ++p) CHECK(orc_gs_scale(n, rp, ci, val, b, p, vs, bs, nrm, w) == 0);
        CHECK(orc_gs_scale(n, rp, ci, val, b, 2, vs, bs, nrm, w) == 0);
        orc_spmv(n, rp, ci, vs, bs, y);
        CHECK(orc_ilu0(n, rp, ci, vs, lu) == 0);
        CHECK(orc_arnoldi(n, rp, ci, vs, bs, m, V, H, eps) >= 1);
        CHECK(orc_gmres(n, rp, ci, vs, bs, x, 10, 1e-10, 10000, eps, NULL, NULL, hist, ii, dd) == 0);
        CHECK(ii[2] == 0 || ii[2] == 1);
        memset(x, 0, sizeof(double) * n);
        CHECK(orc_gmres(n, rp, ci, vs, bs, x, 10, 1e-10, 2000, eps, w, lu, hist, ii, dd) == 0);
        memset(x, 0, sizeof(double) * n);
        CHECK(orc_bicgstab(n, rp, ci, vs, bs, x, 1e-10, 10000, eps, NULL, NULL, hist, ii, dd) == 0);
        CHECK(ii[2] == 0);
        memset(x, 0, sizeof(double) * n);
        CHECK(orc_bicgstab(n, rp, ci, vs, bs, x, 1e-10, 10000, eps, w, lu, hist, ii, dd) == 0);
        memset(x, 0, sizeof(double) * n);
        CHECK(orc_gmres_ir(n, rp, ci, vs, bs, x, 10, 1e-10, 10000, eps, NULL, ii, dd) == 0);
        for (int fb = 0; fb <= 1; ++fb) {
            memset(x, 0, sizeof(double) * n);
            CHECK(orc_bicgstab_ir(n, rp, ci, vs, bs, x, 1e-10, 10000, eps, NULL, 1e-6, fb, 1000,
                                  ii, dd) == 0);
        }
        /* argument errors */
        CHECK(orc_gs_scale(n, rp, ci, val, b, 0, vs, bs, nrm, w) != 0);
        CHECK(orc_bicgstab_ir(n, rp, ci, vs, bs, x, 1e-10, 10000, eps, NULL, 1.5, 1, 1000, ii,
                              dd) != 0);
        free(vs); free(bs); free(nrm); free(w); free(x); free(y); free(lu); free(hist); free(V);
        free(H); free(rp); free(ci); free(val); free(b);
    }
    printf("oracle driver: ok\n");
    return 0;
}
