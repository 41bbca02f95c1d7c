/*
 * Plain FP64 CPU oracle for geometric scaling + restarted GMRES(m) + Bi-CGSTAB.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may link, load or call this file:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg use it. It shares no
 * code, header or constant with the HIP library.
 *
 * Everything here is sequential scalar C, summed left to right in storage order, compiled
 * without FP contraction, so that a reader can check each routine against the paper by eye.
 *
 * Paper: D. Gordon, R. Gordon, "Geometric scaling: a simple preconditioner for certain
 * linear systems with discontinuous coefficients" (2009).
 *   - GS(p): section 1 (definition), section 2 eq. (2) (the scaled system D A x = D b,
 *     D = diag(1/||a_i||_p)); the Lp-norm definition at the start of section 2.
 *   - Solvers: section 2 names restarted GMRES [Saad-Schultz] with a double classical
 *     Gram-Schmidt orthogonalisation step, and Bi-CGSTAB [van der Vorst]; x0 = 0 (section
 *     2.1); stopping test ||b-Ax||/||b-Ax0|| < eps on the GS(2)-scaled system, at most
 *     10,000 iterations, breakdown tolerance DBL_EPSILON relaxed by 1e-16 (section 2.2).
 *   - ILU(0): section 2 (ILUT with drop tolerance 0 and fill-in 1 acted like ILU(0)); used
 *     only as a convergence cross-check.
 *
 * Readings where the paper is silent (the same readings are listed with the design notes):
 *   R1  ||x||_p = (sum |x_i|^p)^(1/p): the printed formula lacks the absolute values.
 *   R2  The Krylov steps themselves are the textbook ones (the paper cites, does not print):
 *       GMRES with Givens rotations on the Hessenberg matrix and a back-substitution at the
 *       end of each cycle; Bi-CGSTAB with shadow residual r^ = r0.
 *   R3  Stop test: strict '<', denominator fixed at the residual of the initial guess. When
 *       the system was scaled by GS(p) with p != 2, the test still measures the GS(2)-scaled
 *       residual: entry i is multiplied by w_i = ||a_i||_p / ||a_i||_2 (weights argument).
 *   R4  A recursive estimate below tol is verified with the true residual b - A x. GMRES
 *       restarts if the check fails; Bi-CGSTAB restarts its recurrence from the true
 *       residual (r^ := r). Three failed checks in a row end the solve as STAGNATED.
 *   R5  GMRES counts Arnoldi steps; Bi-CGSTAB counts iterations, a half-step exit counting
 *       as one. Inside a GMRES cycle the estimate |g_{j+1}| of the cycle's own norm is
 *       converted to the GS(2) metric by the ratio ||W r|| / ||r|| of the cycle's start
 *       residual.
 *   R6  Breakdown: GMRES happy breakdown when h_{j+1,j} <= eps_b ||A v_j||; Bi-CGSTAB
 *       breakdown when |(r^,v)| <= eps_b ||r^|| ||v||, |(t,s)| <= eps_b ||t|| ||s|| or
 *       |(r^,r)| <= eps_b ||r^|| ||r||, with eps_b = 1e-16 * DBL_EPSILON by default.
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Built with -ffp-contract=off: every product is rounded before it is added. */

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_ZERO_ROW (-2)
#define ORC_ERR_NONFINITE (-3)
#define ORC_ERR_ALLOC (-7)

#define ORC_CONVERGED 0
#define ORC_MAXIT 1
#define ORC_BREAKDOWN 2
#define ORC_STAGNATED 3

/* info_i layout: [iters, restarts, status, half_step, verify_failures, breakdown_test]
 * breakdown_test: 0 none, 1 (r^,v), 2 (t,s), 3 (r^,r), 4 zero Hessenberg column
 * info_d layout: [relres_recursive, relres_true]                                     */

/* ---------------------------------------------------------------------------------------
 * Vector helpers: the plain definitions.
 * ------------------------------------------------------------------------------------- */
static double dot(int n, const double* x, const double* y) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

static double nrm2(int n, const double* x) { return sqrt(dot(n, x, x)); }

/* ||W x||_2 with W = diag(w); w == NULL means the identity. */
static double wnrm2(int n, const double* w, const double* x) {
    if (!w) return nrm2(n, x);
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        double t = w[i] * x[i];
        s += t * t;
    }
    return sqrt(s);
}

/* y = A x, each row summed in storage order. */
void orc_spmv(int n, const int* rp, const int* ci, const double* val, const double* x,
              double* y) {
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) s += val[k] * x[ci[k]];
        y[i] = s;
    }
}

/* r = b - A x */
static void residual(int n, const int* rp, const int* ci, const double* val, const double* b,
                     const double* x, double* r) {
    orc_spmv(n, rp, ci, val, x, r);
    for (int i = 0; i < n; ++i) r[i] = b[i] - r[i];
}

/* ---------------------------------------------------------------------------------------
 * GS(p): divide row i of A and b_i by ||a_i||_p (section 2, eq. (2)).
 * Optional outputs: norm_out[i] = ||a_i||_p; weight_out[i] = ||a_i||_p / ||a_i||_2, the factor
 * that turns a residual of the GS(p)-scaled system into one of the GS(2)-scaled system.
 * val_out/b_out may alias val_in/b_in. A row of zeros violates the paper's assumption that
 * no row of A is zero and is reported; so is any non-finite input.
 * ------------------------------------------------------------------------------------- */
int orc_gs_scale(int n, const int* rp, const int* ci, const double* val_in, const double* b_in,
                 int p, double* val_out, double* b_out, double* norm_out, double* weight_out) {
    (void)ci;
    if (n < 0 || p < 1 || (n > 0 && (!rp || !val_in || !b_in || !val_out || !b_out)))
        return ORC_ERR_ARG;
    int zero_row = 0, nonfinite = 0;
    for (int i = 0; i < n; ++i) {
        double sp = 0.0, s2 = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            double a = val_in[k];
            if (!isfinite(a)) nonfinite = 1;
            double ab = fabs(a);
            if (p == 1) sp += ab;
            else if (p == 2) sp += a * a;
            else sp += pow(ab, (double)p);
            s2 += a * a;
        }
        if (!isfinite(b_in[i])) nonfinite = 1;
        if (sp == 0.0) zero_row = 1;
        if (nonfinite || zero_row) continue;
        double nrm;
        if (p == 1) nrm = sp;
        else if (p == 2) nrm = sqrt(sp);
        else nrm = pow(sp, 1.0 / (double)p);
        if (!isfinite(nrm) || !isfinite(s2)) { nonfinite = 1; continue; }
        for (int k = rp[i]; k < rp[i + 1]; ++k) val_out[k] = val_in[k] / nrm;
        b_out[i] = b_in[i] / nrm;
        if (norm_out) norm_out[i] = nrm;
        if (weight_out) weight_out[i] = nrm / sqrt(s2);
    }
    if (nonfinite) return ORC_ERR_NONFINITE;
    if (zero_row) return ORC_ERR_ZERO_ROW;
    return ORC_OK;
}

/* ---------------------------------------------------------------------------------------
 * ILU(0) (cross-check only): L U restricted to the pattern of A, L unit lower triangular.
 * lu has A's pattern; rows must have sorted columns and a diagonal entry.
 * ------------------------------------------------------------------------------------- */
int orc_ilu0(int n, const int* rp, const int* ci, const double* val, double* lu) {
    int* diag = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int* pos = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!diag || !pos) { free(diag); free(pos); return ORC_ERR_ALLOC; }
    memcpy(lu, val, sizeof(double) * (size_t)(n > 0 ? rp[n] : 0));
    for (int i = 0; i < n; ++i) {
        diag[i] = -1;
        for (int k = rp[i]; k < rp[i + 1]; ++k) if (ci[k] == i) diag[i] = k;
        if (diag[i] < 0) { free(diag); free(pos); return ORC_ERR_ARG; }
        pos[i] = -1;
    }
    for (int i = 0; i < n; ++i) {
        for (int k = rp[i]; k < rp[i + 1]; ++k) pos[ci[k]] = k;
        for (int k = rp[i]; k < rp[i + 1] && ci[k] < i; ++k) {
            int c = ci[k];
            double piv = lu[diag[c]];
            if (piv == 0.0) { free(diag); free(pos); return ORC_ERR_ZERO_ROW; }
            lu[k] = lu[k] / piv;                       /* l_{i,c} */
            for (int kk = diag[c] + 1; kk < rp[c + 1]; ++kk) {
                int jpos = pos[ci[kk]];
                if (jpos >= 0) lu[jpos] = lu[jpos] - lu[k] * lu[kk];
            }
        }
        for (int k = rp[i]; k < rp[i + 1]; ++k) pos[ci[k]] = -1;
    }
    free(diag);
    free(pos);
    return ORC_OK;
}

/* z = (LU)^{-1} y: forward substitution with unit L, then backward with U. */
static void ilu0_apply(int n, const int* rp, const int* ci, const double* lu, const double* y,
                       double* z) {
    for (int i = 0; i < n; ++i) {
        double s = y[i];
        for (int k = rp[i]; k < rp[i + 1] && ci[k] < i; ++k) s -= lu[k] * z[ci[k]];
        z[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = z[i];
        double d = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            if (ci[k] > i) s -= lu[k] * z[ci[k]];
            else if (ci[k] == i) d = lu[k];
        }
        z[i] = s / d;
    }
}

/* ---------------------------------------------------------------------------------------
 * Arnoldi with double classical Gram-Schmidt (section 2: GMRES in AZTEC orthogonalises with
 * a double classical Gram-Schmidt step). Builds V (n x (m+1), column-major, ld n) and the
 * Hessenberg matrix H ((m+1) x m, column-major, ld m+1) from r0. Returns the number of
 * steps taken (fewer than m after a happy breakdown). Used by the GMRES oracle below and
 * exported so tests can check orthogonality and the Arnoldi relation directly.
 * ------------------------------------------------------------------------------------- */
static int arnoldi_step(int n, const int* rp, const int* ci, const double* val,
                        const double* lu, double* V, double* H, int ldh, int j, double eps_b,
                        double* w, double* z, double* c, int* happy) {
    /* w = A M^{-1} v_j (M = I without the ILU cross-check) */
    const double* vj = V + (size_t)j * n;
    if (lu) { ilu0_apply(n, rp, ci, lu, vj, z); orc_spmv(n, rp, ci, val, z, w); }
    else orc_spmv(n, rp, ci, val, vj, w);
    double nw = nrm2(n, w);
    double* h = H + (size_t)j * ldh;
    for (int i = 0; i <= j + 1; ++i) h[i] = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        /* classical: all projections against the same w, then one update */
        for (int i = 0; i <= j; ++i) c[i] = dot(n, V + (size_t)i * n, w);
        for (int i = 0; i <= j; ++i) {
            const double* vi = V + (size_t)i * n;
            for (int r = 0; r < n; ++r) w[r] = w[r] - c[i] * vi[r];
            h[i] += c[i];
        }
    }
    h[j + 1] = nrm2(n, w);
    *happy = h[j + 1] <= eps_b * nw;
    if (!*happy) {
        double* vn = V + (size_t)(j + 1) * n;
        for (int r = 0; r < n; ++r) vn[r] = w[r] / h[j + 1];
    }
    return 0;
}

int orc_arnoldi(int n, const int* rp, const int* ci, const double* val, const double* r0,
                int m, double* V, double* H, double eps_b) {
    if (n <= 0 || m <= 0) return ORC_ERR_ARG;
    double* w = (double*)malloc(sizeof(double) * (size_t)n);
    double* c = (double*)malloc(sizeof(double) * (size_t)(m + 1));
    if (!w || !c) { free(w); free(c); return ORC_ERR_ALLOC; }
    memset(H, 0, sizeof(double) * (size_t)(m + 1) * (size_t)m);
    double beta = nrm2(n, r0);
    for (int r = 0; r < n; ++r) V[r] = r0[r] / beta;
    int steps = 0;
    for (int j = 0; j < m; ++j) {
        int happy = 0;
        arnoldi_step(n, rp, ci, val, NULL, V, H, m + 1, j, eps_b, w, NULL, c, &happy);
        steps = j + 1;
        if (happy) break;
    }
    free(w);
    free(c);
    return steps;
}

/* ---------------------------------------------------------------------------------------
 * Restarted GMRES(m) on A x = b (or A M^{-1} u = b, x = M^{-1} u with the ILU cross-check).
 * x holds x0 on entry and the result on return. hist (nullable, capacity maxit) receives
 * the recursive relative-residual estimate after every Arnoldi step.
 * ------------------------------------------------------------------------------------- */
int orc_gmres(int n, const int* rp, const int* ci, const double* val, const double* b,
              double* x, int m, double tol, int maxit, double eps_b, const double* wts,
              const double* lu, double* hist, int* info_i, double* info_d) {
    if (n <= 0 || m <= 0 || maxit < 0 || !(tol > 0.0)) return ORC_ERR_ARG;
    size_t nn = (size_t)n;
    double* V = (double*)malloc(sizeof(double) * nn * (size_t)(m + 1));
    double* H = (double*)malloc(sizeof(double) * (size_t)(m + 1) * (size_t)m);
    double* r = (double*)malloc(sizeof(double) * nn);
    double* w = (double*)malloc(sizeof(double) * nn);
    double* z = (double*)malloc(sizeof(double) * nn);
    double* c = (double*)malloc(sizeof(double) * (size_t)(m + 1));
    double* cs = (double*)malloc(sizeof(double) * (size_t)m);
    double* sn = (double*)malloc(sizeof(double) * (size_t)m);
    double* g = (double*)malloc(sizeof(double) * (size_t)(m + 1));
    double* y = (double*)malloc(sizeof(double) * (size_t)m);
    if (!V || !H || !r || !w || !z || !c || !cs || !sn || !g || !y) {
        free(V); free(H); free(r); free(w); free(z); free(c); free(cs); free(sn); free(g); free(y);
        return ORC_ERR_ALLOC;
    }
    int iters = 0, restarts = 0, status = ORC_MAXIT, fails = 0, brk = 0;
    double est = 1.0, relres_true = 1.0;
    const int ldh = m + 1;

    residual(n, rp, ci, val, b, x, r);
    double ref = wnrm2(n, wts, r);
    if (ref == 0.0) {
        status = ORC_CONVERGED;
        est = 0.0;
        relres_true = 0.0;
        goto done;
    }
    if (maxit == 0) goto done;
    for (;;) {
        /* start of a cycle */
        double beta = nrm2(n, r);
        double ratio = wnrm2(n, wts, r) / beta;   /* own norm -> GS(2) metric (R5) */
        for (int i = 0; i < n; ++i) V[i] = r[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int k = 0, claimed = 0;
        for (int j = 0; j < m; ++j) {
            int happy = 0;
            arnoldi_step(n, rp, ci, val, lu, V, H, ldh, j, eps_b, w, z, c, &happy);
            ++iters;
            double* h = H + (size_t)j * ldh;
            /* apply the previous rotations to the new column */
            for (int i = 0; i < j; ++i) {
                double t = cs[i] * h[i] + sn[i] * h[i + 1];
                h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
                h[i] = t;
            }
            /* new rotation annihilating h_{j+1,j} */
            double d = hypot(h[j], h[j + 1]);
            if (d == 0.0) { status = ORC_BREAKDOWN; brk = 4; k = j; goto update; }
            cs[j] = h[j] / d;
            sn[j] = h[j + 1] / d;
            h[j] = d;
            h[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            est = fabs(g[j + 1]) * ratio / ref;
            if (hist && iters <= maxit) hist[iters - 1] = est;
            k = j + 1;
            if (est < tol) { claimed = 1; break; }
            if (happy) { claimed = 1; break; }
            if (iters >= maxit) break;
        }
    update:
        /* back-substitution H(1:k,1:k) y = g(1:k), then x += M^{-1} V_k y */
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int l = i + 1; l < k; ++l) s -= H[(size_t)l * ldh + i] * y[l];
            y[i] = s / H[(size_t)i * ldh + i];
        }
        for (int r_ = 0; r_ < n; ++r_) w[r_] = 0.0;
        for (int l = 0; l < k; ++l) {
            const double* vl = V + (size_t)l * n;
            for (int r_ = 0; r_ < n; ++r_) w[r_] = w[r_] + y[l] * vl[r_];
        }
        if (lu) {
            ilu0_apply(n, rp, ci, lu, w, z);
            for (int r_ = 0; r_ < n; ++r_) x[r_] = x[r_] + z[r_];
        } else {
            for (int r_ = 0; r_ < n; ++r_) x[r_] = x[r_] + w[r_];
        }
        residual(n, rp, ci, val, b, x, r);
        relres_true = wnrm2(n, wts, r) / ref;
        if (status == ORC_BREAKDOWN) goto done;
        if (relres_true < tol) { status = ORC_CONVERGED; goto done; }
        if (iters >= maxit) { status = ORC_MAXIT; goto done; }
        if (claimed) {
            ++fails;
            if (fails >= 3) { status = ORC_STAGNATED; goto done; }
        } else {
            fails = 0;
        }
        ++restarts;
    }
done:
    if (info_i) {
        info_i[0] = iters; info_i[1] = restarts; info_i[2] = status; info_i[3] = 0;
        info_i[4] = fails; info_i[5] = brk;
    }
    if (info_d) { info_d[0] = est; info_d[1] = relres_true; }
    free(V); free(H); free(r); free(w); free(z); free(c); free(cs); free(sn); free(g); free(y);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------------------
 * Mixed-precision restarted GMRES(m): classical iterative refinement (not in the paper,
 * which solves in FP64 throughout) in which every correction is one GMRES(m) cycle whose
 * data are stored in single precision.
 *   1. r = b - A x in double with the double matrix; stop if ||W r|| / ||W r0|| < tol.
 *   2. One GMRES(m) cycle on A d = r (started from d = 0) in which the matrix values, the
 *      basis vectors and the work vector are stored as float: every stored value is rounded
 *      to float, and each product, dot product and update is computed in double from the
 *      stored floats. The Hessenberg matrix, the Givens rotations, g and y stay double. The
 *      cycle ends early when its estimate |g_{j+1}| (in the norm of the stored r) times
 *      ||W r|| / ||r_stored|| / ||W r0|| drops below tol, on a happy breakdown, or at maxit.
 *   3. x = x + V_k y in double, and back to 1.
 * Stagnation: a cycle that claimed convergence which step 1 does not confirm counts as a
 * failure only if it did not halve the relative true residual; three failures in a row end
 * the solve as STAGNATED.
 * ------------------------------------------------------------------------------------- */
static double fdot(int n, const float* x, const float* y) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += (double)x[i] * (double)y[i];
    return s;
}

int orc_gmres_ir(int n, const int* rp, const int* ci, const double* val, const double* b,
                 double* x, int m, double tol, int maxit, double eps_b, const double* wts,
                 int* info_i, double* info_d) {
    if (n <= 0 || m <= 0 || maxit < 0 || !(tol > 0.0)) return ORC_ERR_ARG;
    size_t nn = (size_t)n;
    int nnz = rp[n];
    float* fval = (float*)malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
    float* V = (float*)malloc(sizeof(float) * nn * (size_t)(m + 1));
    float* w = (float*)malloc(sizeof(float) * nn);
    double* H = (double*)malloc(sizeof(double) * (size_t)(m + 1) * (size_t)m);
    double* r = (double*)malloc(sizeof(double) * nn);
    double* c = (double*)malloc(sizeof(double) * (size_t)(m + 1));
    double* cs = (double*)malloc(sizeof(double) * (size_t)m);
    double* sn = (double*)malloc(sizeof(double) * (size_t)m);
    double* g = (double*)malloc(sizeof(double) * (size_t)(m + 1));
    double* y = (double*)malloc(sizeof(double) * (size_t)m);
    if (!fval || !V || !w || !H || !r || !c || !cs || !sn || !g || !y) {
        free(fval); free(V); free(w); free(H); free(r); free(c); free(cs); free(sn); free(g);
        free(y);
        return ORC_ERR_ALLOC;
    }
    for (int k = 0; k < nnz; ++k) fval[k] = (float)val[k];
    int iters = 0, restarts = 0, status = ORC_MAXIT, fails = 0, brk = 0;
    double est = 1.0, relres_true = 1.0, last = 1.0;
    const int ldh = m + 1;

    residual(n, rp, ci, val, b, x, r);
    double ref = wnrm2(n, wts, r);
    if (ref == 0.0) {
        status = ORC_CONVERGED;
        est = 0.0;
        relres_true = 0.0;
        goto done;
    }
    if (maxit == 0) goto done;
    for (;;) {
        /* step 2: one cycle on A d = r with float storage */
        for (int i = 0; i < n; ++i) w[i] = (float)r[i];            /* stored right-hand side */
        double beta = sqrt(fdot(n, w, w));
        double ratio = wnrm2(n, wts, r) / beta;
        last = wnrm2(n, wts, r) / ref;
        for (int i = 0; i < n; ++i) V[i] = (float)((double)w[i] / beta);
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int k = 0, claimed = 0;
        for (int j = 0; j < m; ++j) {
            /* w = A v_j with the float matrix, sums in double, stored as float */
            const float* vj = V + (size_t)j * n;
            for (int row = 0; row < n; ++row) {
                double s = 0.0;
                for (int q = rp[row]; q < rp[row + 1]; ++q)
                    s += (double)fval[q] * (double)vj[ci[q]];
                w[row] = (float)s;
            }
            double nw = sqrt(fdot(n, w, w));
            double* h = H + (size_t)j * ldh;
            for (int i = 0; i <= j + 1; ++i) h[i] = 0.0;
            for (int pass = 0; pass < 2; ++pass) {
                for (int i = 0; i <= j; ++i) c[i] = fdot(n, V + (size_t)i * n, w);
                for (int row = 0; row < n; ++row) {
                    double t = (double)w[row];
                    for (int i = 0; i <= j; ++i) t -= c[i] * (double)V[(size_t)i * n + row];
                    w[row] = (float)t;
                }
                for (int i = 0; i <= j; ++i) h[i] += c[i];
            }
            h[j + 1] = sqrt(fdot(n, w, w));
            int happy = h[j + 1] <= eps_b * nw;
            if (!happy) {
                float* vn = V + (size_t)(j + 1) * n;
                for (int row = 0; row < n; ++row) vn[row] = (float)((double)w[row] / h[j + 1]);
            }
            ++iters;
            for (int i = 0; i < j; ++i) {
                double t = cs[i] * h[i] + sn[i] * h[i + 1];
                h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
                h[i] = t;
            }
            double d = hypot(h[j], h[j + 1]);
            if (d == 0.0) { status = ORC_BREAKDOWN; brk = 4; k = j; goto update; }
            cs[j] = h[j] / d;
            sn[j] = h[j + 1] / d;
            h[j] = d;
            h[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            est = fabs(g[j + 1]) * ratio / ref;
            k = j + 1;
            if (est < tol) { claimed = 1; break; }
            if (happy) { claimed = 1; break; }
            if (iters >= maxit) break;
        }
    update:
        /* step 3: x = x + V_k y in double */
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int l = i + 1; l < k; ++l) s -= H[(size_t)l * ldh + i] * y[l];
            y[i] = s / H[(size_t)i * ldh + i];
        }
        for (int row = 0; row < n; ++row) {
            double d = 0.0;
            for (int l = 0; l < k; ++l) d += y[l] * (double)V[(size_t)l * n + row];
            x[row] = x[row] + d;
        }
        /* step 1 of the next refinement step */
        residual(n, rp, ci, val, b, x, r);
        relres_true = wnrm2(n, wts, r) / ref;
        if (status == ORC_BREAKDOWN) goto done;
        if (relres_true < tol) { status = ORC_CONVERGED; goto done; }
        if (iters >= maxit) { status = ORC_MAXIT; goto done; }
        if (claimed && !(relres_true < 0.5 * last)) {
            ++fails;
            if (fails >= 3) { status = ORC_STAGNATED; goto done; }
        } else {
            fails = 0;
        }
        ++restarts;
    }
done:
    if (info_i) {
        info_i[0] = iters; info_i[1] = restarts; info_i[2] = status; info_i[3] = 0;
        info_i[4] = fails; info_i[5] = brk;
    }
    if (info_d) { info_d[0] = est; info_d[1] = relres_true; }
    free(fval); free(V); free(w); free(H); free(r); free(c); free(cs); free(sn); free(g); free(y);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------------------
 * Bi-CGSTAB on A x = b (van der Vorst), optionally right-preconditioned by ILU(0).
 * x holds x0 on entry and the result on return. hist (nullable, capacity maxit) receives
 * ||W r||/ref (or ||W s||/ref at a half-step exit) after every iteration.
 * ------------------------------------------------------------------------------------- */
typedef struct {
    int iters, restarts, status, fails, half, brk;
    double est, relres_true;
} bicg_state;

typedef struct {
    double *r, *rh, *p, *v, *s, *t, *ph, *sh;
} bicg_work;

static void bicg_work_free(bicg_work* w) {
    free(w->r); free(w->rh); free(w->p); free(w->v); free(w->s); free(w->t); free(w->ph);
    free(w->sh);
}

static int bicg_work_alloc(bicg_work* w, size_t nn) {
    w->r = (double*)malloc(sizeof(double) * nn);
    w->rh = (double*)malloc(sizeof(double) * nn);
    w->p = (double*)malloc(sizeof(double) * nn);
    w->v = (double*)malloc(sizeof(double) * nn);
    w->s = (double*)malloc(sizeof(double) * nn);
    w->t = (double*)malloc(sizeof(double) * nn);
    w->ph = (double*)malloc(sizeof(double) * nn);
    w->sh = (double*)malloc(sizeof(double) * nn);
    if (!w->r || !w->rh || !w->p || !w->v || !w->s || !w->t || !w->ph || !w->sh) {
        bicg_work_free(w);
        return 0;
    }
    return 1;
}

/* The FP64 iteration from the current x, with r = b - A x in w->r and the reference norm
 * ref of the stop test: the recurrence (re)starts from r (r^ = r), stops on its estimate,
 * is verified with the true residual (R4) and restarts from it after a failed check; three
 * failed checks in a row end the solve as STAGNATED. The counters in *st continue from their
 * values on entry (iters counts towards maxit); on return st->status is final and x, est and
 * relres_true belong to it. */
static void bicg64_run(int n, const int* rp, const int* ci, const double* val, const double* b,
                       double* x, double tol, int maxit, double eps_b, const double* wts,
                       const double* lu, double* hist, double ref, bicg_work* w,
                       bicg_state* st) {
    size_t nn = (size_t)n;
    double *r = w->r, *rh = w->rh, *p = w->p, *v = w->v, *s = w->s, *t = w->t, *ph = w->ph,
           *sh = w->sh;
    for (;;) {
        /* (re)start the recurrence from the current residual r */
        memcpy(rh, r, sizeof(double) * nn);
        double rh_norm = nrm2(n, rh);
        double rho = dot(n, rh, r);
        double rho_old = 1.0, alpha = 1.0, omega = 1.0;
        int first = 1;
        int verify = 0;
        st->half = 0;
        while (!verify) {
            if (fabs(rho) <= eps_b * rh_norm * nrm2(n, r)) { st->status = ORC_BREAKDOWN; st->brk = 3; goto final_check; }
            if (first) {
                memcpy(p, r, sizeof(double) * nn);
            } else {
                double beta = (rho / rho_old) * (alpha / omega);
                for (int i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
            }
            first = 0;
            /* v = A M^{-1} p */
            if (lu) { ilu0_apply(n, rp, ci, lu, p, ph); orc_spmv(n, rp, ci, val, ph, v); }
            else { memcpy(ph, p, sizeof(double) * nn); orc_spmv(n, rp, ci, val, p, v); }
            double sigma = dot(n, rh, v);
            if (fabs(sigma) <= eps_b * rh_norm * nrm2(n, v)) { st->status = ORC_BREAKDOWN; st->brk = 1; goto final_check; }
            alpha = rho / sigma;
            for (int i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
            ++st->iters;
            st->est = wnrm2(n, wts, s) / ref;
            if (st->est < tol) {
                /* half-step exit: x += alpha p^ */
                for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * ph[i];
                if (hist && st->iters <= maxit) hist[st->iters - 1] = st->est;
                st->half = 1;
                verify = 1;
                break;
            }
            /* t = A M^{-1} s */
            if (lu) { ilu0_apply(n, rp, ci, lu, s, sh); orc_spmv(n, rp, ci, val, sh, t); }
            else { memcpy(sh, s, sizeof(double) * nn); orc_spmv(n, rp, ci, val, s, t); }
            double ts = dot(n, t, s);
            double tt = dot(n, t, t);
            if (fabs(ts) <= eps_b * sqrt(tt) * nrm2(n, s)) { st->status = ORC_BREAKDOWN; st->brk = 2; goto final_check; }
            omega = ts / tt;
            for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * ph[i] + omega * sh[i];
            for (int i = 0; i < n; ++i) r[i] = s[i] - omega * t[i];
            st->est = wnrm2(n, wts, r) / ref;
            if (hist && st->iters <= maxit) hist[st->iters - 1] = st->est;
            if (st->est < tol || st->iters >= maxit) { verify = 1; break; }
            rho_old = rho;
            rho = dot(n, rh, r);
        }
        /* verification with the true residual (R4) */
        residual(n, rp, ci, val, b, x, r);
        st->relres_true = wnrm2(n, wts, r) / ref;
        if (st->relres_true < tol) { st->status = ORC_CONVERGED; return; }
        if (st->iters >= maxit) { st->status = ORC_MAXIT; return; }
        ++st->fails;
        if (st->fails >= 3) { st->status = ORC_STAGNATED; return; }
        ++st->restarts;
    }
final_check:
    residual(n, rp, ci, val, b, x, r);
    st->relres_true = wnrm2(n, wts, r) / ref;
}

int orc_bicgstab(int n, const int* rp, const int* ci, const double* val, const double* b,
                 double* x, double tol, int maxit, double eps_b, const double* wts,
                 const double* lu, double* hist, int* info_i, double* info_d) {
    if (n <= 0 || maxit < 0 || !(tol > 0.0)) return ORC_ERR_ARG;
    bicg_work w;
    if (!bicg_work_alloc(&w, (size_t)n)) return ORC_ERR_ALLOC;
    bicg_state st = {0, 0, ORC_MAXIT, 0, 0, 0, 1.0, 1.0};
    residual(n, rp, ci, val, b, x, w.r);
    double ref = wnrm2(n, wts, w.r);
    if (ref == 0.0) {
        st.status = ORC_CONVERGED;
        st.est = st.relres_true = 0.0;
    } else if (maxit > 0) {
        bicg64_run(n, rp, ci, val, b, x, tol, maxit, eps_b, wts, lu, hist, ref, &w, &st);
    }
    if (info_i) {
        info_i[0] = st.iters; info_i[1] = st.restarts; info_i[2] = st.status;
        info_i[3] = st.half; info_i[4] = st.fails; info_i[5] = st.brk;
    }
    if (info_d) { info_d[0] = st.est; info_d[1] = st.relres_true; }
    bicg_work_free(&w);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------------------
 * Mixed-precision Bi-CGSTAB: classical iterative refinement (not in the paper, which solves
 * in FP64 throughout) whose corrections are Bi-CGSTAB runs with single-precision storage.
 *   1. r = b - A x in double with the double matrix; rt = ||W r|| / ||W r0||; stop if
 *      rt < tol.
 *   2. Restart the Bi-CGSTAB recurrence from r: the stored residual r~ and the shadow
 *      residual r^ are r rounded to float. The matrix values, r~, r^, p, v and t are stored
 *      as float; every product, dot product and update is computed in double from the stored
 *      floats, and a value is rounded to float when it is stored. s = r~ - alpha v is not
 *      stored and stays double; x stays double.
 *   3. The run ends (and goes back to 1) when its estimate ||W s|| / ||W r0|| (half step) or
 *      ||W r~|| / ||W r0|| drops below max(tol, delta * rt): a reduction by delta of the
 *      residual it started from is as far as float storage is trusted to go. It also ends
 *      when the estimate ||W r~|| / ||W r0|| exceeds rt / delta or is not finite: the float
 *      recurrences have diverged, and the refinement step decides (a choice the paper leaves
 *      open: float-storage Bi-CGSTAB can diverge to overflow on the jump problems); and,
 *      with run_cap > 0, after run_cap iterations (a run that wanders without reaching its
 *      target would otherwise spend the whole iteration budget before any refinement step).
 * Stagnation: a refinement step that does not halve rt counts as a failure; three failures
 * in a row end the refinement. Breakdown tests as in Bi-CGSTAB (R6), on the stored vectors.
 * FP64 continuation (fallback != 0; a design choice, not in the paper): the solve is
 * handed to FP64 Bi-CGSTAB (the algorithm of orc_bicgstab) when the refinement stops paying:
 *   - a run leaves the true residual above the one it started from (float recurrences that
 *     diverged move x away from the solution before the divergence test ends them): the run
 *     is undone (x is restored to its value at the run's start), then handed over;
 *   - three refinement steps in a row do not halve the true residual;
 *   - a float-storage run breaks down (after the same undo test).
 * The continuation starts from x with r = b - A x, keeps the reference norm and the
 * iteration count towards maxit, counts as one more restart, and decides the status.
 * info_i[6] = the iteration count at the hand-over (0 if it never happened). With
 * fallback == 0 the refinement ends as STAGNATED or BREAKDOWN, without any undo.
 * ------------------------------------------------------------------------------------- */
int orc_bicgstab_ir(int n, const int* rp, const int* ci, const double* val, const double* b,
                    double* x, double tol, int maxit, double eps_b, const double* wts,
                    double delta, int fallback, int run_cap, int* info_i, double* info_d) {
    if (n <= 0 || maxit < 0 || !(tol > 0.0) || !(delta > 0.0) || !(delta < 1.0) ||
        run_cap < 0)
        return ORC_ERR_ARG;
    size_t nn = (size_t)n;
    int nnz = rp[n];
    float* fval = (float*)malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
    float* rs = (float*)malloc(sizeof(float) * nn);    /* stored residual r~ */
    float* rh = (float*)malloc(sizeof(float) * nn);
    float* p = (float*)malloc(sizeof(float) * nn);
    float* v = (float*)malloc(sizeof(float) * nn);
    float* t = (float*)malloc(sizeof(float) * nn);
    double* r = (double*)malloc(sizeof(double) * nn);  /* true residual, double */
    double* s = (double*)malloc(sizeof(double) * nn);
    double* xs = (double*)malloc(sizeof(double) * nn); /* x at the start of the run */
    if (!fval || !rs || !rh || !p || !v || !t || !r || !s || !xs) {
        free(fval); free(rs); free(rh); free(p); free(v); free(t); free(r); free(s); free(xs);
        return ORC_ERR_ALLOC;
    }
    for (int k = 0; k < nnz; ++k) fval[k] = (float)val[k];
    int iters = 0, restarts = 0, status = ORC_MAXIT, fails = 0, half = 0, brk = 0;
    int fp64_from = 0;
    double est = 1.0, relres_true = 1.0;

    residual(n, rp, ci, val, b, x, r);
    double ref = wnrm2(n, wts, r);
    if (ref == 0.0) {
        status = ORC_CONVERGED;
        est = relres_true = 0.0;
        goto done;
    }
    if (maxit == 0) goto done;
    double rt = 1.0;
    for (;;) {
        /* step 2: restart from the true residual */
        double target = delta * rt > tol ? delta * rt : tol;
        memcpy(xs, x, sizeof(double) * nn);
        const int run_start = iters;
        for (int i = 0; i < n; ++i) rs[i] = (float)r[i];
        memcpy(rh, rs, sizeof(float) * nn);
        double rh_norm = sqrt(fdot(n, rh, rh));
        double rho = fdot(n, rh, rs);
        double rho_old = 1.0, alpha = 1.0, omega = 1.0;
        int first = 1;
        half = 0;
        for (;;) {
            if (fabs(rho) <= eps_b * rh_norm * sqrt(fdot(n, rs, rs))) {
                status = ORC_BREAKDOWN; brk = 3; goto float_breakdown;
            }
            if (first) {
                memcpy(p, rs, sizeof(float) * nn);
            } else {
                double beta = (rho / rho_old) * (alpha / omega);
                for (int i = 0; i < n; ++i)
                    p[i] = (float)((double)rs[i] + beta * ((double)p[i] - omega * (double)v[i]));
            }
            first = 0;
            for (int row = 0; row < n; ++row) {          /* v = A p, float matrix */
                double acc = 0.0;
                for (int q = rp[row]; q < rp[row + 1]; ++q)
                    acc += (double)fval[q] * (double)p[ci[q]];
                v[row] = (float)acc;
            }
            double sigma = fdot(n, rh, v);
            if (fabs(sigma) <= eps_b * rh_norm * sqrt(fdot(n, v, v))) {
                status = ORC_BREAKDOWN; brk = 1; goto float_breakdown;
            }
            alpha = rho / sigma;
            for (int i = 0; i < n; ++i) s[i] = (double)rs[i] - alpha * (double)v[i];
            ++iters;
            est = wnrm2(n, wts, s) / ref;
            if (est < target) {                            /* half-step exit */
                for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * (double)p[i];
                half = 1;
                break;
            }
            for (int row = 0; row < n; ++row) {          /* t = A s, float matrix */
                double acc = 0.0;
                for (int q = rp[row]; q < rp[row + 1]; ++q) acc += (double)fval[q] * s[ci[q]];
                t[row] = (float)acc;
            }
            double ts = 0.0;
            for (int i = 0; i < n; ++i) ts += (double)t[i] * s[i];
            double tt = fdot(n, t, t);
            if (fabs(ts) <= eps_b * sqrt(tt) * nrm2(n, s)) {
                status = ORC_BREAKDOWN; brk = 2; goto float_breakdown;
            }
            omega = ts / tt;
            for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * (double)p[i] + omega * s[i];
            for (int i = 0; i < n; ++i) rs[i] = (float)(s[i] - omega * (double)t[i]);
            double ws = 0.0;
            for (int i = 0; i < n; ++i) {
                double e = wts ? wts[i] * (double)rs[i] : (double)rs[i];
                ws += e * e;
            }
            est = sqrt(ws) / ref;
            if (est < target || iters >= maxit || !(est <= rt / delta) ||
                (run_cap > 0 && iters - run_start >= run_cap))
                break;
            rho_old = rho;
            rho = fdot(n, rh, rs);
        }
        /* step 1 of the next refinement step */
        residual(n, rp, ci, val, b, x, r);
        relres_true = wnrm2(n, wts, r) / ref;
        if (relres_true < tol) { status = ORC_CONVERGED; goto done; }
        if (fallback && !(relres_true <= rt)) {   /* the run made x worse: undo, hand over */
            memcpy(x, xs, sizeof(double) * nn);
            goto fp64;
        }
        if (iters >= maxit) { status = ORC_MAXIT; goto done; }
        if (!(relres_true < 0.5 * rt)) {
            ++fails;
            if (fails >= 3) {
                if (fallback) goto fp64;
                status = ORC_STAGNATED;
                goto done;
            }
        } else {
            fails = 0;
        }
        rt = relres_true;
        ++restarts;
    }
float_breakdown:
    residual(n, rp, ci, val, b, x, r);
    relres_true = wnrm2(n, wts, r) / ref;
    if (!fallback) goto done;
    if (!(relres_true <= rt)) memcpy(x, xs, sizeof(double) * nn);   /* undo the run */
fp64:
    {
        /* FP64 continuation from x: r = b - A x, then orc_bicgstab's iteration */
        bicg_work w;
        if (!bicg_work_alloc(&w, nn)) {
            free(fval); free(rs); free(rh); free(p); free(v); free(t); free(r); free(s);
            free(xs);
            return ORC_ERR_ALLOC;
        }
        residual(n, rp, ci, val, b, x, w.r);
        fp64_from = iters;
        bicg_state st = {iters, restarts + 1, ORC_MAXIT, 0, 0, 0, est,
                         wnrm2(n, wts, w.r) / ref};
        if (st.relres_true < tol) st.status = ORC_CONVERGED;
        else if (iters < maxit)
            bicg64_run(n, rp, ci, val, b, x, tol, maxit, eps_b, wts, NULL, NULL, ref, &w, &st);
        iters = st.iters; restarts = st.restarts; status = st.status; fails = st.fails;
        half = st.half; brk = st.brk; est = st.est; relres_true = st.relres_true;
        bicg_work_free(&w);
    }
done:
    if (info_i) {
        info_i[0] = iters; info_i[1] = restarts; info_i[2] = status; info_i[3] = half;
        info_i[4] = fails; info_i[5] = brk; info_i[6] = fp64_from;
    }
    if (info_d) { info_d[0] = est; info_d[1] = relres_true; }
    free(fval); free(rs); free(rh); free(p); free(v); free(t); free(r); free(s); free(xs);
    return ORC_OK;
}

/* Default breakdown tolerance: DBL_EPSILON relaxed by 1e-16 (section 2.2). */
double orc_default_breakdown_eps(void) { return 1e-16 * DBL_EPSILON; }
