/*
 * FP64 CPU oracle for the ADMM collision-avoidance path of
 * "GPU-Accelerated Optimization-Based Collision Avoidance" (arXiv 2406.07048).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may include, link or
 * call this file; only the test-suite, the smoke check and the CPU baseline of
 * the benchmark do. It shares no code with the HIP library.
 *
 * It computes, plainly and slowly, in double precision:
 *   - the scale-based detection LP (Sec. III-A, eq. scale_opt) through its
 *     dual (Sec. III-B, eq. scale_opt_dual) with a textbook two-phase dense
 *     tableau simplex (Bland's rule);
 *   - one dual-update sub-problem (Sec. IV-C, eq. const_least_square) with the
 *     Jacobi-scaled proximal term (reading: prox weight eps * ||row_l K||^2
 *     around the previous iterate), by a primal active-set method;
 *   - the state/input update (Sec. IV-B, eq. ADMM_state_updates) as one QP per
 *     ADMM iteration (Sec. IV-B, SQP remark) with R(s), rho(s) linearised at the
 *     current iterate, solved by condensing the dynamics and a Cholesky
 *     factorisation of the input Hessian;
 *   - the multiplier update (Sec. IV-B, eq. ADMM_residue_updates) with the exact
 *     nonlinear T and R, and the stopping test (Sec. IV-B, stopping criteria).
 *
 * Layout conventions (shared documentation with the C ABI, not shared code):
 * pair blocks enumerate (scenario, robot part i, obstacle j); a block holds
 * the N pairs t = 1..N; its dual rows (lambda, mu, gamma) are stored row-major
 * [row][t]; zeta[block*N + t-1]; xi[(block*dim + c)*N + t-1].
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXD 3
#define MAXROWS 64
#define MAXS 16

/* ------------------------------------------------------------------ */
/* dense helpers                                                       */
/* ------------------------------------------------------------------ */

/* Solve M z = r in place (M n x n row-major, destroyed), Gaussian elimination
   with partial pivoting. Returns 0 on success, 1 if a pivot vanishes. */
static int gauss_solve(int n, double *M, double *r)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(M[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabs(M[i * n + k]) > best) { best = fabs(M[i * n + k]); p = i; }
        if (best == 0.0) return 1;
        if (p != k) {
            for (int j = 0; j < n; ++j) { double t = M[k * n + j]; M[k * n + j] = M[p * n + j]; M[p * n + j] = t; }
            double t = r[k]; r[k] = r[p]; r[p] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            double f = M[i * n + k] / M[k * n + k];
            if (f == 0.0) continue;
            for (int j = k; j < n; ++j) M[i * n + j] -= f * M[k * n + j];
            r[i] -= f * r[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = r[k];
        for (int j = k + 1; j < n; ++j) s -= M[k * n + j] * r[j];
        r[k] = s / M[k * n + k];
    }
    return 0;
}

/* Cholesky factor L (lower triangle, in place) of an SPD matrix. Returns 1
   if not SPD. */
static int chol_factor(int n, double *M)
{
    for (int j = 0; j < n; ++j) {
        double s = M[j * n + j];
        for (int k = 0; k < j; ++k) s -= M[j * n + k] * M[j * n + k];
        if (s <= 0.0) return 1;
        double L = sqrt(s);
        M[j * n + j] = L;
        for (int i = j + 1; i < n; ++i) {
            double t = M[i * n + j];
            for (int k = 0; k < j; ++k) t -= M[i * n + k] * M[j * n + k];
            M[i * n + j] = t / L;
        }
    }
    return 0;
}

/* Solve L L^T z = r in place with the factor of chol_factor. */
static void chol_apply(int n, const double *M, double *r)
{
    for (int i = 0; i < n; ++i) {
        double s = r[i];
        for (int k = 0; k < i; ++k) s -= M[i * n + k] * r[k];
        r[i] = s / M[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = r[i];
        for (int k = i + 1; k < n; ++k) s -= M[k * n + i] * r[k];
        r[i] = s / M[i * n + i];
    }
}

/* Cholesky solve of an SPD system (M destroyed). Returns 1 if not SPD. */
static int chol_solve(int n, double *M, double *r)
{
    if (chol_factor(n, M)) return 1;
    chol_apply(n, M, r);
    return 0;
}

/* ------------------------------------------------------------------ */
/* scale LP (Sec. III-A eq. scale_opt, Sec. III-B eq. scale_opt_dual)  */
/* ------------------------------------------------------------------ */

/*
 * min c^T z  s.t.  E z = f (f >= 0), z >= 0, with m rows and n columns,
 * by the two-phase tableau simplex with Bland's anti-cycling rule.
 * Outputs z (n) and the simplex multipliers pi (m) of the optimal basis.
 * Returns 0 optimal, 1 infeasible, 2 unbounded, 3 iteration cap.
 */
static int simplex_std(int m, int n, const double *E, const double *f, const double *c,
                       double *z, double *pi)
{
    const int W = n + m + 1;           /* columns: structural, artificial, rhs */
    double *T = (double *)calloc((size_t)(m + 1) * W, sizeof(double));
    int *basis = (int *)malloc(sizeof(int) * m);
    int status = 0;
    double scale = 1.0;
    for (int i = 0; i < m * n; ++i) if (fabs(E[i]) > scale) scale = fabs(E[i]);
    for (int j = 0; j < n; ++j) if (fabs(c[j]) > scale) scale = fabs(c[j]);
    const double tol = 1e-12 * scale;

    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < n; ++j) T[i * W + j] = E[i * n + j];
        T[i * W + n + i] = 1.0;
        T[i * W + W - 1] = f[i];
        basis[i] = n + i;
    }
    for (int phase = 1; phase <= 2; ++phase) {
        double *obj = T + (size_t)m * W;
        /* reduced costs of the current basis for this phase's cost vector */
        for (int j = 0; j < W; ++j) {
            double cj = (j == W - 1) ? 0.0 : (phase == 1 ? (j >= n ? 1.0 : 0.0) : (j < n ? c[j] : 0.0));
            double s = cj;
            for (int i = 0; i < m; ++i) {
                int bj = basis[i];
                double cb = phase == 1 ? (bj >= n ? 1.0 : 0.0) : (bj < n ? c[bj] : 0.0);
                s -= cb * T[i * W + j];
            }
            obj[j] = s;   /* obj[W-1] = -objective value */
        }
        int it;
        for (it = 0; it < 1000; ++it) {
            /* phase 1 only seeks feasibility: stop once the artificial sum is 0 */
            if (phase == 1 && -obj[W - 1] <= 1e-12 * (1.0 + scale)) break;
            /* reduced-cost tolerance grows with the tableau entries, so that
               rounding noise of large intermediate entries never drives a pivot */
            double growth = 1.0;
            for (int i = 0; i < m * W; ++i) if (fabs(T[i]) > growth) growth = fabs(T[i]);
            const double rtol = tol * growth;
            int enter = -1;
            int ncols = (phase == 1) ? n + m : n;   /* artificials never re-enter in phase 2 */
            for (int j = 0; j < ncols; ++j)
                if (obj[j] < -rtol) { enter = j; break; }          /* Bland: lowest index */
            if (enter < 0) break;
            /* Harris two-pass ratio test: the minimum ratio with the right-hand
               side relaxed by a small tolerance, then, among the rows within
               it, the largest pivot element (never a pivot that is rounding
               noise of a cancelled entry) */
            int leave = -1;
            double cmaxv = 0.0;
            for (int i = 0; i < m; ++i) if (fabs(T[i * W + enter]) > cmaxv) cmaxv = fabs(T[i * W + enter]);
            const double ptol = tol > 1e-9 * cmaxv ? tol : 1e-9 * cmaxv;
            double theta = INFINITY;
            for (int i = 0; i < m; ++i) {
                double a = T[i * W + enter];
                if (a > ptol) {
                    double r = (T[i * W + W - 1] + tol) / a;
                    if (r < theta) theta = r;
                }
            }
            double bestpiv = 0.0;
            for (int i = 0; i < m; ++i) {
                double a = T[i * W + enter];
                if (a > ptol && T[i * W + W - 1] / a <= theta && a > bestpiv) {
                    bestpiv = a;
                    leave = i;
                }
            }
            if (leave < 0) { status = 2; goto done; }
            double pv = T[leave * W + enter];
            for (int j = 0; j < W; ++j) T[leave * W + j] /= pv;
            for (int i = 0; i <= m; ++i) {
                if (i == leave) continue;
                double fct = T[i * W + enter];
                if (fct == 0.0) continue;
                for (int j = 0; j < W; ++j) T[i * W + j] -= fct * T[leave * W + j];
            }
            basis[leave] = enter;
            for (int i = 0; i < m; ++i) if (T[i * W + W - 1] < 0.0) T[i * W + W - 1] = 0.0;
        }
        if (it >= 1000) { status = 3; goto done; }
        if (phase == 1) {
            if (-obj[W - 1] > 1e-9 * (1.0 + scale)) { status = 1; goto done; }
            /* drive remaining (zero-level) artificials out of the basis */
            for (int i = 0; i < m; ++i) {
                if (basis[i] < n) continue;
                int piv = -1;
                double best = 1e-9;
                for (int j = 0; j < n; ++j)
                    if (fabs(T[i * W + j]) > best) { best = fabs(T[i * W + j]); piv = j; }
                if (piv < 0) continue;   /* redundant row: artificial stays at zero */
                double pv = T[i * W + piv];
                for (int j = 0; j < W; ++j) T[i * W + j] /= pv;
                for (int r = 0; r <= m; ++r) {
                    if (r == i) continue;
                    double fct = T[r * W + piv];
                    if (fct == 0.0) continue;
                    for (int j = 0; j < W; ++j) T[r * W + j] -= fct * T[i * W + j];
                }
                basis[i] = piv;
            }
        }
    }
    for (int j = 0; j < n; ++j) z[j] = 0.0;
    for (int i = 0; i < m; ++i) if (basis[i] < n) z[basis[i]] = T[i * W + W - 1];
    /* multipliers: the artificial column k holds B^{-1} e_k, and its phase-2
       reduced cost is 0 - pi_k */
    for (int k = 0; k < m; ++k) pi[k] = -T[(size_t)m * W + n + k];
done:
    free(T);
    free(basis);
    return status;
}

/*
 * Scale LP of one robot part against one obstacle, both expressed in the
 * part's body frame (obstacle faces Cp = C R, offsets dp = d - C pos):
 *     alpha* = min alpha  s.t.  A x <= alpha b,  Cp x <= dp.
 * Solved through the dual max -dp^T mu s.t. b^T lam = 1,
 * A^T lam + Cp^T mu = 0, lam, mu >= 0 (Sec. III-B). Returns alpha*, the primal
 * point x* (from the simplex multipliers), the dual certificate and the
 * duality gap (primal objective alpha* minus dual objective -dp^T mu*).
 */
int orc_scale_lp(int dim, int nr, const double *A, const double *b,
                 int no, const double *Cp, const double *dp,
                 double *alpha, double *x, double *lam, double *mu, double *gap)
{
    int m = dim + 1, n = nr + no;
    double *E = (double *)calloc((size_t)m * n, sizeof(double));
    double *cc = (double *)calloc(n, sizeof(double));
    double *z = (double *)calloc(n, sizeof(double));
    double f[MAXD + 1] = {0}, pi[MAXD + 1] = {0};
    f[0] = 1.0;
    for (int k = 0; k < nr; ++k) {
        E[0 * n + k] = b[k];
        for (int r = 0; r < dim; ++r) E[(1 + r) * n + k] = A[k * dim + r];
    }
    for (int l = 0; l < no; ++l) {
        for (int r = 0; r < dim; ++r) E[(1 + r) * n + nr + l] = Cp[l * dim + r];
        cc[nr + l] = dp[l];
    }
    int st = simplex_std(m, n, E, f, cc, z, pi);
    double dual_obj = 0.0;
    for (int k = 0; k < nr; ++k) lam[k] = z[k];
    for (int l = 0; l < no; ++l) { mu[l] = z[nr + l]; dual_obj -= dp[l] * z[nr + l]; }
    *alpha = -pi[0];
    for (int r = 0; r < dim; ++r) x[r] = pi[1 + r];
    if (gap) *gap = *alpha - dual_obj;
    free(E); free(cc); free(z);
    return st;
}

/* ------------------------------------------------------------------ */
/* pair QP (Sec. IV-C eq. const_least_square, with proximal term)      */
/* ------------------------------------------------------------------ */

/* Rows of K (Sec. IV-C): lambda rows (0, A_k), mu rows (dp_l, Cp_l),
   gamma row (1, 0). Fills K (n x (dim+1)) and returns n. */
static int build_K(int dim, int nr, const double *A, int no, const double *Cp, const double *dp, double *K)
{
    int c = dim + 1, n = nr + no + 1;
    memset(K, 0, sizeof(double) * n * c);
    for (int k = 0; k < nr; ++k)
        for (int r = 0; r < dim; ++r) K[k * c + 1 + r] = A[k * dim + r];
    for (int l = 0; l < no; ++l) {
        K[(nr + l) * c] = dp[l];
        for (int r = 0; r < dim; ++r) K[(nr + l) * c + 1 + r] = Cp[l * dim + r];
    }
    K[(nr + no) * c] = 1.0;
    return n;
}

/*
 * One dual-update sub-problem:
 *   min_y 1/2 ||K^T y + bhat||^2 + eps/2 sum_l D_l (y_l - yhat_l)^2
 *   s.t.  b^T lam = 1,  y >= 0,
 * with y = (lam, mu, gamma), bhat = (1 + zeta, xi), D_l = ||row_l K||^2.
 * Primal active-set method (equality-constrained sub-QPs solved by Gaussian
 * elimination). Output y (n); returns the number of active-set iterations,
 * or -1 on failure.
 */
int orc_pair_qp(int dim, int nr, const double *A, const double *b,
                int no, const double *Cp, const double *dp,
                double zeta, const double *xi, const double *yhat, double eps,
                double *y)
{
    const int c = dim + 1;
    double K[MAXROWS * (MAXD + 1)];
    int n = build_K(dim, nr, A, no, Cp, dp, K);
    double bh[MAXD + 1];
    bh[0] = 1.0 + zeta;
    for (int r = 0; r < dim; ++r) bh[1 + r] = xi[r];
    double G[MAXROWS * MAXROWS], g[MAXROWS], D[MAXROWS], kap[MAXROWS];
    for (int l = 0; l < n; ++l) {
        double s = 0.0;
        for (int q = 0; q < c; ++q) s += K[l * c + q] * K[l * c + q];
        D[l] = s;
        kap[l] = (l < nr) ? b[l] : 0.0;
    }
    for (int l = 0; l < n; ++l) {
        for (int m = 0; m < n; ++m) {
            double s = 0.0;
            for (int q = 0; q < c; ++q) s += K[l * c + q] * K[m * c + q];
            G[l * n + m] = s + (l == m ? eps * D[l] : 0.0);
        }
        double s = 0.0;
        for (int q = 0; q < c; ++q) s += K[l * c + q] * bh[q];
        g[l] = s - eps * D[l] * yhat[l];
    }
    /* feasible start: yhat if feasible, else 1/b_k on the largest b_k */
    int feasible = 1;
    double ky = 0.0;
    for (int l = 0; l < n; ++l) { if (!(yhat[l] >= 0.0)) feasible = 0; ky += kap[l] * yhat[l]; }
    if (fabs(ky - 1.0) > 1e-12) feasible = 0;
    int inW[MAXROWS];
    if (feasible) {
        for (int l = 0; l < n; ++l) { y[l] = yhat[l]; }
        /* re-normalise the equality exactly onto the lambda part */
        if (ky != 1.0) for (int k = 0; k < nr; ++k) y[k] /= ky;
    } else {
        int kb = 0;
        for (int k = 1; k < nr; ++k) if (b[k] > b[kb]) kb = k;
        for (int l = 0; l < n; ++l) y[l] = 0.0;
        y[kb] = 1.0 / b[kb];
    }
    for (int l = 0; l < n; ++l) inW[l] = (y[l] == 0.0);

    double gscale = 1.0;
    for (int l = 0; l < n * n; ++l) if (fabs(G[l]) > gscale) gscale = fabs(G[l]);
    /* After a full (unblocked) step the iterate is the minimiser of the
       equality-constrained sub-problem on the current working set, so the
       bound multipliers are checked directly instead of re-solving. */
    int at_eqp_min = 0;
    double nu = 0.0;
    for (int iter = 0; iter < 50 * n; ++iter) {
        int F[MAXROWS], nf = 0;
        for (int l = 0; l < n; ++l) if (!inW[l]) F[nf++] = l;
        double grad[MAXROWS];
        for (int l = 0; l < n; ++l) {
            double s = g[l];
            for (int m = 0; m < n; ++m) s += G[l * n + m] * y[m];
            grad[l] = s;
        }
        double p[MAXROWS] = {0};
        double ymax = 1.0;
        for (int l = 0; l < n; ++l) if (fabs(y[l]) > ymax) ymax = fabs(y[l]);
        if (!at_eqp_min) {
            int sz = nf + 1;
            double M[(MAXROWS + 1) * (MAXROWS + 1)], rhs[MAXROWS + 1];
            for (int a = 0; a < nf; ++a) {
                for (int bq = 0; bq < nf; ++bq) M[a * sz + bq] = G[F[a] * n + F[bq]];
                M[a * sz + nf] = -kap[F[a]];
                M[nf * sz + a] = kap[F[a]];
                rhs[a] = -grad[F[a]];
            }
            M[nf * sz + nf] = 0.0;
            rhs[nf] = 0.0;
            if (gauss_solve(sz, M, rhs)) return -1;
            double pmax = 0.0;
            for (int a = 0; a < nf; ++a) { p[F[a]] = rhs[a]; if (fabs(rhs[a]) > pmax) pmax = fabs(rhs[a]); }
            nu = rhs[nf];
            if (pmax <= 1e-13 * ymax) at_eqp_min = 1;
        }
        if (at_eqp_min) {
            /* bound multipliers w = grad - kappa nu on the working set */
            int drop = -1;
            double wmin = -1e-12 * gscale * ymax;
            for (int l = 0; l < n; ++l) {
                if (!inW[l]) continue;
                double w = grad[l] - kap[l] * nu;
                if (w < wmin) { wmin = w; drop = l; }
            }
            if (drop < 0) return iter;
            inW[drop] = 0;
            at_eqp_min = 0;
            continue;
        }
        double step = 1.0;
        int block = -1;
        for (int a = 0; a < nf; ++a) {
            int l = F[a];
            if (p[l] < 0.0) {
                double s = -y[l] / p[l];
                if (s < step) { step = s; block = l; }
            }
        }
        for (int l = 0; l < n; ++l) y[l] += step * p[l];
        if (block >= 0) { y[block] = 0.0; inW[block] = 1; }
        else at_eqp_min = 1;
    }
    return -1;
}

/* ------------------------------------------------------------------ */
/* the paper's route for the dual-update QP (Sec. IV-C): elimination   */
/* of the equality, the KKT conditions as an LCP, Lemke's method       */
/* ------------------------------------------------------------------ */

/*
 * Lemke's complementary pivoting for the LCP  w = M z + q, w, z >= 0,
 * w^T z = 0  (n unknowns, M row-major). With q >= 0, z = 0. Otherwise an
 * artificial variable z0 with covering vector e = 1 enters; each pivot
 * brings in the complement of the variable that just left, with the
 * lexicographic minimum-ratio rule (rows of the basis inverse break ties),
 * until z0 leaves. Returns 0 (z written), 1 (secondary ray) or 2 (pivot
 * limit).
 */
static int lemke(int n, const double *M, const double *q, double *z)
{
    int cols = 2 * n + 2;      /* w_1..w_n, z_1..z_n, z0, rhs */
    double *T = (double *)calloc((size_t)n * cols, sizeof(double));
    int *basis = (int *)malloc(sizeof(int) * n);
    int st = 0;
    /* rows: I w - M z - e z0 = q */
    for (int i = 0; i < n; ++i) {
        T[i * cols + i] = 1.0;
        for (int j = 0; j < n; ++j) T[i * cols + n + j] = -M[i * n + j];
        T[i * cols + 2 * n] = -1.0;
        T[i * cols + 2 * n + 1] = q[i];
        basis[i] = i;
    }
    int qmin = 0;
    for (int i = 1; i < n; ++i) if (q[i] < q[qmin]) qmin = i;
    for (int i = 0; i < n; ++i) z[i] = 0.0;
    if (n == 0 || q[qmin] >= 0.0) { free(T); free(basis); return 0; }
    int enter = 2 * n, leave_row = qmin;
    for (int piv = 0; piv < 50 * n + 50; ++piv) {
        /* pivot on (leave_row, enter) */
        double pv = T[leave_row * cols + enter];
        for (int j = 0; j < cols; ++j) T[leave_row * cols + j] /= pv;
        for (int i = 0; i < n; ++i) {
            if (i == leave_row) continue;
            double f = T[i * cols + enter];
            if (f != 0.0)
                for (int j = 0; j < cols; ++j) T[i * cols + j] -= f * T[leave_row * cols + j];
        }
        int left = basis[leave_row];
        basis[leave_row] = enter;
        if (left == 2 * n) goto done;                    /* z0 left: solution */
        enter = left < n ? n + left : left - n;           /* complement of the leaving variable */
        /* lexicographic ratio test over rows with a positive entry */
        leave_row = -1;
        for (int i = 0; i < n; ++i) {
            double a = T[i * cols + enter];
            if (a <= 1e-12) continue;
            if (leave_row < 0) { leave_row = i; continue; }
            double ai = T[leave_row * cols + enter];
            double r1 = T[i * cols + 2 * n + 1] / a, r0 = T[leave_row * cols + 2 * n + 1] / ai;
            if (r1 < r0 - 1e-12 * (1.0 + fabs(r0))) { leave_row = i; continue; }
            if (r1 > r0 + 1e-12 * (1.0 + fabs(r0))) continue;
            for (int k = 0; k < n; ++k) {
                double l1 = T[i * cols + k] / a, l0 = T[leave_row * cols + k] / ai;
                if (l1 < l0 - 1e-14) { leave_row = i; break; }
                if (l1 > l0 + 1e-14) break;
            }
        }
        if (leave_row < 0) { st = 1; goto out; }
    }
    st = 2;
    goto out;
done:
    for (int i = 0; i < n; ++i)
        if (basis[i] >= n && basis[i] < 2 * n) z[basis[i] - n] = T[i * cols + 2 * n + 1];
out:
    free(T);
    free(basis);
    return st;
}

/*
 * The dual-update QP of orc_pair_qp solved the paper's way (Sec. IV-C):
 * (1) one equality variable y_e with kappa_e > 0 (reading: the largest b_k)
 *     is eliminated, y_e = (eta - kappa_u^T y_u) / kappa_e, eta = 1, and its
 *     sign condition becomes the inequality kappa~^T y_u <= eta~ with
 *     kappa~ = kappa_u / kappa_e, eta~ = eta / kappa_e (eq.
 *     const_least_square_ineq);
 * (2) the KKT conditions of that QP (eq. kkt_conditions) are the LCP with
 *     z = (y_u, phi), M = [[Q, kappa~], [-kappa~^T, 0]], q = (c, eta~)
 *     (eq. linear_complementarity_problem), where Q and c are the Hessian
 *     and gradient at y_u = 0 of the reduced objective: K~ K~^T and K~ b~
 *     of the paper plus the proximal term eps/2 sum_l D_l (y_l - yhat_l)^2
 *     carried through the elimination;
 * (3) Lemke's method solves the LCP.
 * Output y (n); returns 0, or a Lemke status (1 ray, 2 pivot limit) + 1.
 */
int orc_pair_qp_lemke(int dim, int nr, const double *A, const double *b,
                      int no, const double *Cp, const double *dp,
                      double zeta, const double *xi, const double *yhat, double eps,
                      double *y)
{
    const int c = dim + 1;
    double K[MAXROWS * (MAXD + 1)];
    int n = build_K(dim, nr, A, no, Cp, dp, K);
    double bh[MAXD + 1];
    bh[0] = 1.0 + zeta;
    for (int r = 0; r < dim; ++r) bh[1 + r] = xi[r];
    double D[MAXROWS];
    for (int l = 0; l < n; ++l) {
        double s = 0.0;
        for (int q = 0; q < c; ++q) s += K[l * c + q] * K[l * c + q];
        D[l] = s;
    }
    int e = 0;
    for (int k = 1; k < nr; ++k) if (b[k] > b[e]) e = k;
    const double eta = 1.0, ke = b[e];
    /* y = E y_u + f: y_e = eta~ - kappa~^T y_u, the others copy y_u */
    int m = n - 1, map[MAXROWS];
    for (int l = 0, u = 0; l < n; ++l) if (l != e) map[u++] = l;
    double kt[MAXROWS];
    for (int u = 0; u < m; ++u) kt[u] = map[u] < nr ? b[map[u]] / ke : 0.0;
    const double etat = eta / ke;
    /* Kt rows = K_u - kappa~ K_e; bt = bhat + K_e^T eta~ */
    double Kt[MAXROWS * (MAXD + 1)], bt[MAXD + 1];
    for (int u = 0; u < m; ++u)
        for (int q = 0; q < c; ++q) Kt[u * c + q] = K[map[u] * c + q] - kt[u] * K[e * c + q];
    for (int q = 0; q < c; ++q) bt[q] = bh[q] + K[e * c + q] * etat;
    int nz = m + 1;
    double *Mm = (double *)calloc((size_t)nz * nz, sizeof(double));
    double qv[MAXROWS + 1], zz[MAXROWS + 1];
    for (int u = 0; u < m; ++u) {
        for (int v = 0; v < m; ++v) {
            double s = 0.0;
            for (int q = 0; q < c; ++q) s += Kt[u * c + q] * Kt[v * c + q];
            s += eps * D[e] * kt[u] * kt[v];
            if (u == v) s += eps * D[map[u]];
            Mm[u * nz + v] = s;
        }
        Mm[u * nz + m] = kt[u];
        Mm[m * nz + u] = -kt[u];
        double s = 0.0;
        for (int q = 0; q < c; ++q) s += Kt[u * c + q] * bt[q];
        /* proximal gradient at y_u = 0: y_e = eta~, y_u = 0 */
        s += eps * (-kt[u] * D[e] * (etat - yhat[e]) - D[map[u]] * yhat[map[u]]);
        qv[u] = s;
    }
    qv[m] = etat;
    int st = lemke(nz, Mm, qv, zz);
    free(Mm);
    if (st) return st + 1;
    double ye = etat;
    for (int u = 0; u < m; ++u) { y[map[u]] = zz[u]; ye -= kt[u] * zz[u]; }
    y[e] = ye;
    return 0;
}

/* ------------------------------------------------------------------ */
/* pose R(s), rho(s) and their derivatives                             */
/* ------------------------------------------------------------------ */

typedef struct {
    int dim, n_s, n_u, N, n_parts, n_scen;
    const int *part_face_ptr;
    const double *part_A, *part_b, *part_off;
    const int *obs_ptr, *obs_face_ptr;
    const double *obs_C, *obs_d;
    const double *A_dyn, *B_dyn, *c_dyn;
    const int *pos_idx, *att_idx;
    int att_kind;                   /* 0: planar yaw, 1: ZYX Euler (phi, theta, psi) */
    const double *Q_s, *Q_u, *x_ref, *x0;
    double sigma, eps_prox, eps_pri, eps_dual;
    /* dynamics x_{t+1} = A x_t + B u_t + c (Sec. IV-A eq. system_eqn, given
       linearised): the model of (scenario s, step t) is number
       s * dyn_ss + t * dyn_ts of the arrays A_dyn, B_dyn, c_dyn (0, 0: one
       time-invariant model). model != 0 names a nonlinear f that every ADMM
       iteration linearises about its current iterate instead (the SQP step of
       Sec. IV-B); the given model then only sets the initial trajectory. */
    int dyn_ts, dyn_ss;
    int model;                      /* 0: the given linear model, 1: kinematic bicycle, 2: quadrotor */
    double model_par[8];
    /* state and input bounds (Sec. IV-A eq. MPC_opt_origin, its state and
       control rows) on x_t, t = 1..N, and u_t, t = 0..N-1: s_lo, s_hi [n_s],
       u_lo, u_hi [n_u]; NULL or infinite entries: no bound */
    const double *s_lo, *s_hi, *u_lo, *u_hi;
} orc_problem;

static const double *dyn_A(const orc_problem *P, int s) { return P->A_dyn + (size_t)s * P->dyn_ss * P->n_s * P->n_s; }
static const double *dyn_B(const orc_problem *P, int s) { return P->B_dyn + (size_t)s * P->dyn_ss * P->n_s * P->n_u; }
static const double *dyn_c(const orc_problem *P, int s) { return P->c_dyn + (size_t)s * P->dyn_ss * P->n_s; }

static int n_att(const orc_problem *P) { return P->att_kind == 0 ? 1 : 3; }

/* R(s) and dR/d(att_a) for a = 0..n_att-1 (dim x dim row-major each). */
static void rotation(const orc_problem *P, const double *s, double *R, double *dR)
{
    if (P->att_kind == 0) {
        double th = s[P->att_idx[0]], c = cos(th), sn = sin(th);
        R[0] = c; R[1] = -sn; R[2] = sn; R[3] = c;
        if (dR) { dR[0] = -sn; dR[1] = -c; dR[2] = c; dR[3] = -sn; }
        return;
    }
    double ph = s[P->att_idx[0]], th = s[P->att_idx[1]], ps = s[P->att_idx[2]];
    double cf = cos(ph), sf = sin(ph), ct = cos(th), st = sin(th), cp = cos(ps), sp = sin(ps);
    double Rx[9] = {1, 0, 0, 0, cf, -sf, 0, sf, cf};
    double Ry[9] = {ct, 0, st, 0, 1, 0, -st, 0, ct};
    double Rz[9] = {cp, -sp, 0, sp, cp, 0, 0, 0, 1};
    double dRx[9] = {0, 0, 0, 0, -sf, -cf, 0, cf, -sf};
    double dRy[9] = {-st, 0, ct, 0, 0, 0, -ct, 0, -st};
    double dRz[9] = {-sp, -cp, 0, cp, -sp, 0, 0, 0, 0};
    const double *F1[4] = {Rz, Rz, dRz, Rz};
    const double *F2[4] = {Ry, dRy, Ry, Ry};
    const double *F3[4] = {Rx, Rx, Rx, dRx};
    /* index 0: R; 1: d/dtheta; 2: d/dpsi; 3: d/dphi */
    double out[4][9];
    for (int v = 0; v < 4; ++v) {
        double T1[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0;
                for (int k = 0; k < 3; ++k) acc += F1[v][i * 3 + k] * F2[v][k * 3 + j];
                T1[i * 3 + j] = acc;
            }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0;
                for (int k = 0; k < 3; ++k) acc += T1[i * 3 + k] * F3[v][k * 3 + j];
                out[v][i * 3 + j] = acc;
            }
    }
    memcpy(R, out[0], sizeof(double) * 9);
    if (dR) {
        memcpy(dR + 0, out[3], sizeof(double) * 9);   /* d/dphi */
        memcpy(dR + 9, out[1], sizeof(double) * 9);   /* d/dtheta */
        memcpy(dR + 18, out[2], sizeof(double) * 9);  /* d/dpsi */
    }
}

/* Part frame quantities at state s: R, pos_i = rho(s) + R o_i, the obstacle
   faces in the part frame Cp = C R and offsets dp = d - C pos_i. */
static void part_frame(const orc_problem *P, const double *s, int i, int j,
                       double *R, double *pos, double *Cp, double *dp)
{
    int dim = P->dim;
    rotation(P, s, R, NULL);
    for (int r = 0; r < dim; ++r) {
        double acc = s[P->pos_idx[r]];
        for (int q = 0; q < dim; ++q) acc += R[r * dim + q] * P->part_off[i * dim + q];
        pos[r] = acc;
    }
    int f0 = P->obs_face_ptr[j], f1 = P->obs_face_ptr[j + 1];
    for (int l = 0; l < f1 - f0; ++l) {
        const double *cl = P->obs_C + (size_t)(f0 + l) * dim;
        double acc = P->obs_d[f0 + l];
        for (int r = 0; r < dim; ++r) acc -= cl[r] * pos[r];
        dp[l] = acc;
        for (int q = 0; q < dim; ++q) {
            double a = 0;
            for (int r = 0; r < dim; ++r) a += cl[r] * R[r * dim + q];
            Cp[l * dim + q] = a;
        }
    }
}

/* ------------------------------------------------------------------ */
/* block enumeration                                                   */
/* ------------------------------------------------------------------ */

typedef struct { int s, i, j, nr, no, n; long yoff; } orc_block;

static int count_blocks(const orc_problem *P)
{
    return P->n_parts * P->obs_ptr[P->n_scen];
}

static void enumerate_blocks(const orc_problem *P, orc_block *B)
{
    int b = 0;
    long off = 0;
    for (int s = 0; s < P->n_scen; ++s)
        for (int i = 0; i < P->n_parts; ++i)
            for (int j = P->obs_ptr[s]; j < P->obs_ptr[s + 1]; ++j) {
                orc_block *q = &B[b++];
                q->s = s; q->i = i; q->j = j;
                q->nr = P->part_face_ptr[i + 1] - P->part_face_ptr[i];
                q->no = P->obs_face_ptr[j + 1] - P->obs_face_ptr[j];
                q->n = q->nr + q->no + 1;
                q->yoff = off;
                off += (long)q->n * P->N;
            }
}

long orc_y_size(const orc_problem *P)
{
    int nb = count_blocks(P);
    orc_block *B = (orc_block *)malloc(sizeof(orc_block) * (nb > 0 ? nb : 1));
    enumerate_blocks(P, B);
    long tot = nb ? B[nb - 1].yoff + (long)B[nb - 1].n * P->N : 0;
    free(B);
    return tot;
}

static const double *state_at(const orc_problem *P, const double *x, int s, int t)
{
    return x + ((size_t)s * (P->N + 1) + t) * P->n_s;
}

/* ------------------------------------------------------------------ */
/* trajectory QP (Sec. IV-B eq. ADMM_state_updates, one SQP QP)         */
/* ------------------------------------------------------------------ */

/*
 * min sum_{t=1..N} (1/2 x_t^T H_t x_t + h_t^T x_t) + sum_{t=0..N-1} u_t^T Q_u u_t
 * s.t. x_{t+1} = A_t x_t + B_t u_t + c_t, x_0 given, where the model of step
 * t is A + t ts n_s n_s (B, c likewise; ts = 0: time-invariant).
 * Condensed: x_t = z_t + sum_{k<t} A_{t-1} ... A_{k+1} B_k u_k with the free
 * response z_t = A_{t-1} z_{t-1} + c_{t-1}, then a dense Cholesky solve in the
 * stacked inputs.  H: N blocks (t = 1..N) of n_s x n_s.
 */

/* The condensed form: free response z (t = 0..N), the maps M_t = dx_t/du
 * (t = 1..N, n_s x nU each, nU = N n_u), and the input Hessian Hs and the
 * gradient gr at u = 0 of 1/2 u^T Hs u + gr^T u. */
static void condense(int n_s, int n_u, int N, const double *A0, const double *B0, const double *c0, int ts,
                     const double *x0, const double *H, const double *h, const double *Q_u,
                     double *Mt, double *z, double *Hs, double *gr)
{
    int nU = N * n_u;
    double *HM = (double *)calloc((size_t)n_s * nU, sizeof(double));
    memcpy(z, x0, sizeof(double) * n_s);
    for (int t = 1; t <= N; ++t) {
        double *Mc = Mt + (size_t)(t - 1) * n_s * nU;
        const double *Mp = (t >= 2) ? Mt + (size_t)(t - 2) * n_s * nU : NULL;
        const double *A = A0 + (size_t)(t - 1) * ts * n_s * n_s, *B = B0 + (size_t)(t - 1) * ts * n_s * n_u;
        const double *c = c0 + (size_t)(t - 1) * ts * n_s;
        for (int r = 0; r < n_s; ++r) {
            double acc = c[r];
            for (int q = 0; q < n_s; ++q) acc += A[r * n_s + q] * z[(t - 1) * n_s + q];
            z[t * n_s + r] = acc;
            for (int col = 0; col < nU; ++col) {
                double a = 0.0;
                if (Mp) for (int q = 0; q < n_s; ++q) a += A[r * n_s + q] * Mp[q * nU + col];
                Mc[r * nU + col] = a;
            }
            for (int k = 0; k < n_u; ++k) Mc[r * nU + (t - 1) * n_u + k] += B[r * n_u + k];
        }
    }
    for (int k = 0; k < N; ++k)
        for (int a = 0; a < n_u; ++a)
            for (int bq = 0; bq < n_u; ++bq)
                Hs[(k * n_u + a) * nU + k * n_u + bq] = 2.0 * Q_u[a * n_u + bq];
    for (int t = 1; t <= N; ++t) {
        const double *Mc = Mt + (size_t)(t - 1) * n_s * nU;
        const double *Ht = H + (size_t)(t - 1) * n_s * n_s;
        const double *ht = h + (size_t)(t - 1) * n_s;
        for (int r = 0; r < n_s; ++r)
            for (int col = 0; col < nU; ++col) {
                double a = 0.0;
                for (int q = 0; q < n_s; ++q) a += Ht[r * n_s + q] * Mc[q * nU + col];
                HM[r * nU + col] = a;
            }
        for (int a = 0; a < nU; ++a) {
            for (int bq = 0; bq < nU; ++bq) {
                double acc = 0.0;
                for (int r = 0; r < n_s; ++r) acc += Mc[r * nU + a] * HM[r * nU + bq];
                Hs[a * nU + bq] += acc;
            }
            double acc = 0.0;
            for (int r = 0; r < n_s; ++r) {
                double Hz = ht[r];
                for (int q = 0; q < n_s; ++q) Hz += Ht[r * n_s + q] * z[t * n_s + q];
                acc += Mc[r * nU + a] * Hz;
            }
            gr[a] += acc;
        }
    }
    free(HM);
}

/* x_{t+1} = A_t x_t + B_t u_t + c_t for t = 0..N-1 from the x_0 in x. */
static void rollout(int n_s, int n_u, int N, const double *A0, const double *B0, const double *c0, int ts,
                    const double *u, double *x)
{
    for (int t = 0; t < N; ++t) {
        const double *A = A0 + (size_t)t * ts * n_s * n_s, *B = B0 + (size_t)t * ts * n_s * n_u;
        const double *c = c0 + (size_t)t * ts * n_s;
        for (int r = 0; r < n_s; ++r) {
            double acc = c[r];
            for (int q = 0; q < n_s; ++q) acc += A[r * n_s + q] * x[t * n_s + q];
            for (int k = 0; k < n_u; ++k) acc += B[r * n_u + k] * u[t * n_u + k];
            x[(t + 1) * n_s + r] = acc;
        }
    }
}

int orc_traj_qp(int n_s, int n_u, int N, const double *A0, const double *B0, const double *c0, int ts,
                const double *x0, const double *H, const double *h, const double *Q_u,
                double *x, double *u)
{
    int nU = N * n_u;
    double *Mt = (double *)calloc((size_t)N * n_s * nU, sizeof(double));   /* dx_t/du, t=1..N */
    double *z = (double *)calloc((size_t)(N + 1) * n_s, sizeof(double));
    double *Hs = (double *)calloc((size_t)nU * nU, sizeof(double));
    double *gr = (double *)calloc(nU, sizeof(double));
    condense(n_s, n_u, N, A0, B0, c0, ts, x0, H, h, Q_u, Mt, z, Hs, gr);
    for (int a = 0; a < nU; ++a) gr[a] = -gr[a];
    int st = chol_solve(nU, Hs, gr);
    if (!st) {
        memcpy(u, gr, sizeof(double) * nU);
        memcpy(x, x0, sizeof(double) * n_s);
        rollout(n_s, n_u, N, A0, B0, c0, ts, u, x);
    }
    free(Mt); free(z); free(Hs); free(gr);
    return st;
}

/* ------------------------------------------------------------------ */
/* trajectory QP with state and input bounds (Sec. IV-A eq.            */
/* MPC_opt_origin, state and control rows; the indicator IC_0 of eq.   */
/* ADMM_Lagrangian in full)                                            */
/* ------------------------------------------------------------------ */

/* Bound c of the condensed QP as n_c^T u >= b_c over the stacked inputs u
 * (length nU = N n_u). Bounds are numbered: input lower (t, k) at
 * 2 (t n_u + k), input upper at 2 (t n_u + k) + 1, then state lower (t, r),
 * t = 1..N, at 2 nU + 2 ((t-1) n_s + r), state upper one after it. The state
 * rows come from x_t = z_t + M_t u (z the free response, M_t = dx_t/du). */
typedef struct {
    int n_s, n_u, N, nU;
    const double *Mt, *z;                  /* as in orc_traj_qp */
    const double *xlo, *xhi, *ulo, *uhi;   /* NULL: no bound of that kind */
} bqp;

static int bqp_count(const bqp *Q) { return 2 * Q->nU + 2 * Q->N * Q->n_s; }

/* Normal (dense, nU) and right-hand side of bound c; returns 0 if the bound
 * is absent (infinite). */
static int bqp_row(const bqp *Q, int c, double *n, double *b)
{
    int up = c & 1, v = c >> 1;
    memset(n, 0, sizeof(double) * Q->nU);
    if (v < Q->nU) {
        int k = v % Q->n_u;
        const double *lim = up ? Q->uhi : Q->ulo;
        if (!lim || !isfinite(lim[k])) return 0;
        n[v] = up ? -1.0 : 1.0;
        *b = up ? -lim[k] : lim[k];
        return 1;
    }
    v -= Q->nU;
    int t = v / Q->n_s + 1, r = v % Q->n_s;
    const double *lim = up ? Q->xhi : Q->xlo;
    if (!lim || !isfinite(lim[r])) return 0;
    const double *row = Q->Mt + ((size_t)(t - 1) * Q->n_s + r) * Q->nU;
    for (int a = 0; a < Q->nU; ++a) n[a] = up ? -row[a] : row[a];
    double zt = Q->z[t * Q->n_s + r];
    *b = up ? zt - lim[r] : lim[r] - zt;
    return 1;
}

/*
 * min sum_{t=1..N} (1/2 x_t^T H_t x_t + h_t^T x_t) + sum_{t=0..N-1} u_t^T Q_u u_t
 * s.t. x_{t+1} = A_t x_t + B_t u_t + c_t, x_0 given,
 *      xlo <= x_t <= xhi (t = 1..N), ulo <= u_t <= uhi (t = 0..N-1),
 * any bound array NULL or any entry infinite meaning no bound. Condensed as
 * orc_traj_qp, then the dual active-set method of Goldfarb and Idnani (Math.
 * Programming 27, 1983) on the strictly convex QP 1/2 u^T G u + g^T u in the
 * stacked inputs, with G^{-1} formed explicitly: from the unconstrained
 * minimiser, repeatedly take the most violated bound p and move the primal
 * point along the direction that keeps the active bounds satisfied while
 * p's multiplier grows; a bound whose multiplier reaches zero first is
 * dropped (partial step), else p joins the active set (full step). Every step
 * raises the dual objective, so no active set repeats.
 * Returns 0, 1 (G not positive definite), 2 (bounds infeasible), 3 (step cap).
 * n_active (may be NULL) receives the bounds active at the solution.
 */
int orc_traj_qp_bounded(int n_s, int n_u, int N, const double *A0, const double *B0, const double *c0, int ts,
                        const double *x0, const double *H, const double *h, const double *Q_u,
                        const double *xlo, const double *xhi, const double *ulo, const double *uhi,
                        double *x, double *u, int *n_active)
{
    int nU = N * n_u;
    double *Mt = (double *)calloc((size_t)N * n_s * nU, sizeof(double));
    double *z = (double *)calloc((size_t)(N + 1) * n_s, sizeof(double));
    double *G = (double *)calloc((size_t)nU * nU, sizeof(double));
    double *g = (double *)calloc(nU, sizeof(double));
    condense(n_s, n_u, N, A0, B0, c0, ts, x0, H, h, Q_u, Mt, z, G, g);
    bqp Q = {n_s, n_u, N, nU, Mt, z, xlo, xhi, ulo, uhi};
    int nC = bqp_count(&Q), st = 0, nA = 0;
    double *Gi = (double *)calloc((size_t)nU * nU, sizeof(double));
    double *L = (double *)malloc(sizeof(double) * nU * nU);
    /* G^{-1} column by column from one Cholesky factor */
    memcpy(L, G, sizeof(double) * nU * nU);
    if (chol_factor(nU, L)) st = 1;
    for (int col = 0; col < nU && !st; ++col) {
        double *e = Gi + (size_t)col * nU;     /* G symmetric: column = row */
        e[col] = 1.0;
        chol_apply(nU, L, e);
    }
    int *act = (int *)malloc(sizeof(int) * (nU + 1));
    double *lam = (double *)malloc(sizeof(double) * (nU + 1));
    double *NA = (double *)malloc(sizeof(double) * (size_t)(nU + 1) * nU);    /* active normals */
    double *WA = (double *)malloc(sizeof(double) * (size_t)(nU + 1) * nU);    /* G^{-1} n_i */
    double *np_ = (double *)malloc(sizeof(double) * nU), *wp = (double *)malloc(sizeof(double) * nU);
    double *d = (double *)malloc(sizeof(double) * nU);
    double *M = (double *)malloc(sizeof(double) * (nU + 1) * (nU + 1));
    double *r = (double *)malloc(sizeof(double) * (nU + 1));
    unsigned char *in = (unsigned char *)calloc(nC, 1);
    double *nrow = (double *)malloc(sizeof(double) * nU);
    if (!st) {
        for (int a = 0; a < nU; ++a) {
            double acc = 0.0;
            for (int b2 = 0; b2 < nU; ++b2) acc -= Gi[(size_t)a * nU + b2] * g[b2];
            u[a] = acc;
        }
    }
    int steps = 0, cap = 20 * (nC + nU) + 100;
    while (!st) {
        /* the most violated bound not in the active set (scaled by its normal) */
        int p = -1;
        double worst = 0.0, bp = 0.0;
        for (int c = 0; c < nC; ++c) {
            double b;
            if (in[c] || !bqp_row(&Q, c, nrow, &b)) continue;
            double s = -b, nn = 0.0;
            for (int a = 0; a < nU; ++a) { s += nrow[a] * u[a]; nn += nrow[a] * nrow[a]; }
            double tol = 1e-11 * (1.0 + fabs(b));
            if (s < -tol && s / sqrt(nn) < worst) { worst = s / sqrt(nn); p = c; bp = b; }
        }
        if (p < 0) break;
        bqp_row(&Q, p, np_, &bp);
        double lp = 0.0;
        for (;;) {
            if (++steps > cap) { st = 3; break; }
            for (int a = 0; a < nU; ++a) {
                double acc = 0.0;
                for (int b2 = 0; b2 < nU; ++b2) acc += Gi[(size_t)a * nU + b2] * np_[b2];
                wp[a] = acc;
            }
            /* r = (N_A^T G^{-1} N_A)^{-1} N_A^T G^{-1} n_p */
            for (int i = 0; i < nA; ++i) {
                double acc = 0.0;
                for (int a = 0; a < nU; ++a) acc += NA[(size_t)i * nU + a] * wp[a];
                r[i] = acc;
                for (int j = 0; j < nA; ++j) {
                    double m = 0.0;
                    for (int a = 0; a < nU; ++a) m += NA[(size_t)i * nU + a] * WA[(size_t)j * nU + a];
                    M[i * nA + j] = m;
                }
            }
            if (nA && gauss_solve(nA, M, r)) { st = 2; break; }
            double dn = 0.0, pp = 0.0;
            for (int a = 0; a < nU; ++a) {
                double acc = wp[a];
                for (int i = 0; i < nA; ++i) acc -= r[i] * WA[(size_t)i * nU + a];
                d[a] = acc;
                dn += np_[a] * acc;
                pp += np_[a] * wp[a];
            }
            /* partial step: the first active multiplier to reach zero */
            int k = -1;
            double t2 = INFINITY;
            for (int i = 0; i < nA; ++i)
                if (r[i] > 0.0 && lam[i] / r[i] < t2) { t2 = lam[i] / r[i]; k = i; }
            double s = -bp;
            for (int a = 0; a < nU; ++a) s += np_[a] * u[a];
            int dependent = dn <= 1e-12 * pp;
            if (dependent && k < 0) { st = 2; break; }
            double t1 = dependent ? INFINITY : -s / dn;
            double t = t1 < t2 ? t1 : t2;
            if (!dependent)
                for (int a = 0; a < nU; ++a) u[a] += t * d[a];
            for (int i = 0; i < nA; ++i) lam[i] -= t * r[i];
            lp += t;
            if (t1 <= t2) {
                /* full step: p joins the active set */
                memcpy(NA + (size_t)nA * nU, np_, sizeof(double) * nU);
                memcpy(WA + (size_t)nA * nU, wp, sizeof(double) * nU);
                act[nA] = p;
                lam[nA] = lp;
                in[p] = 1;
                ++nA;
                break;
            }
            /* partial step: drop bound k and try p again */
            in[act[k]] = 0;
            for (int i = k; i + 1 < nA; ++i) {
                act[i] = act[i + 1];
                lam[i] = lam[i + 1];
                memcpy(NA + (size_t)i * nU, NA + (size_t)(i + 1) * nU, sizeof(double) * nU);
                memcpy(WA + (size_t)i * nU, WA + (size_t)(i + 1) * nU, sizeof(double) * nU);
            }
            --nA;
        }
    }
    if (st != 1) {
        memcpy(x, x0, sizeof(double) * n_s);
        rollout(n_s, n_u, N, A0, B0, c0, ts, u, x);
    }
    if (n_active) *n_active = nA;
    free(Mt); free(z); free(G); free(g); free(Gi); free(L); free(act); free(lam); free(NA); free(WA);
    free(np_); free(wp); free(d); free(M); free(r); free(in); free(nrow);
    return st;
}

/* ------------------------------------------------------------------ */
/* ADMM pieces                                                         */
/* ------------------------------------------------------------------ */

/* T and R of one pair (Sec. IV-A): T = 1 + dp^T mu + gamma,
   R = A^T lam + Cp^T mu, where y holds block rows for one t with stride N. */
static void pair_TR(const orc_problem *P, const orc_block *q, const double *s,
                    const double *yb, int stride, double *Tout, double *Rout)
{
    int dim = P->dim;
    double R[9], pos[3], Cp[MAXROWS * MAXD], dp[MAXROWS];
    part_frame(P, s, q->i, q->j, R, pos, Cp, dp);
    const double *A = P->part_A + (size_t)P->part_face_ptr[q->i] * dim;
    double T = 1.0 + yb[(q->n - 1) * stride];
    for (int l = 0; l < q->no; ++l) T += dp[l] * yb[(q->nr + l) * stride];
    for (int r = 0; r < dim; ++r) {
        double acc = 0.0;
        for (int k = 0; k < q->nr; ++k) acc += A[k * dim + r] * yb[k * stride];
        for (int l = 0; l < q->no; ++l) acc += Cp[l * dim + r] * yb[(q->nr + l) * stride];
        Rout[r] = acc;
    }
    *Tout = T;
}

/* s^0: obstacle-free LQ solution (stage Hessian 2 Q_s, gradient -2 Q_s xref). */
static int lq_stage_base(const orc_problem *P, int s, double *H, double *h)
{
    int n_s = P->n_s, N = P->N;
    for (int t = 1; t <= N; ++t) {
        const double *xr = P->x_ref + ((size_t)s * (N + 1) + t) * n_s;
        for (int r = 0; r < n_s; ++r) {
            double acc = 0.0;
            for (int q = 0; q < n_s; ++q) {
                H[((size_t)(t - 1) * n_s + r) * n_s + q] = 2.0 * P->Q_s[r * n_s + q];
                acc += 2.0 * P->Q_s[r * n_s + q] * xr[q];
            }
            h[(size_t)(t - 1) * n_s + r] = -acc;
        }
    }
    return 0;
}

static int any_finite(const double *v, int n)
{
    if (!v) return 0;
    for (int i = 0; i < n; ++i)
        if (isfinite(v[i])) return 1;
    return 0;
}

/* The trajectory QP of scenario s for the models (A, B, c, ts), with the
   problem's state and input bounds when it has any (the indicator IC_0 of
   Sec. IV-B eq. ADMM_Lagrangian covers them). Nonzero on failure. */
static int traj_solve(const orc_problem *P, int s, const double *A, const double *B, const double *c, int ts,
                      const double *H, const double *h, double *x, double *u)
{
    const double *x0 = P->x0 + (size_t)s * P->n_s;
    if (any_finite(P->s_lo, P->n_s) || any_finite(P->s_hi, P->n_s) || any_finite(P->u_lo, P->n_u) ||
        any_finite(P->u_hi, P->n_u))
        return orc_traj_qp_bounded(P->n_s, P->n_u, P->N, A, B, c, ts, x0, H, h, P->Q_u, P->s_lo, P->s_hi,
                                   P->u_lo, P->u_hi, x, u, NULL) != 0;
    return orc_traj_qp(P->n_s, P->n_u, P->N, A, B, c, ts, x0, H, h, P->Q_u, x, u);
}

/* Initial iterate: s^0 = obstacle-free LQ, zeta = xi = 0,
   y^0 = (lam*, mu*, max(alpha* - 1, 0)) from the scale LP at s^0. */
int orc_admm_init(const orc_problem *P, double *x, double *u, double *y, double *zeta, double *xi)
{
    int n_s = P->n_s, N = P->N, dim = P->dim;
    double *H = (double *)malloc(sizeof(double) * N * n_s * n_s);
    double *h = (double *)malloc(sizeof(double) * N * n_s);
    int bad = 0;
    for (int s = 0; s < P->n_scen; ++s) {
        lq_stage_base(P, s, H, h);
        bad |= traj_solve(P, s, dyn_A(P, s), dyn_B(P, s), dyn_c(P, s), P->dyn_ts, H, h,
                          x + (size_t)s * (N + 1) * n_s, u + (size_t)s * N * P->n_u);
    }
    free(H); free(h);
    int nb = count_blocks(P);
    orc_block *B = (orc_block *)malloc(sizeof(orc_block) * (nb > 0 ? nb : 1));
    enumerate_blocks(P, B);
    int npairs = nb * N;
    #pragma omp parallel for schedule(dynamic, 16) reduction(|:bad)
    for (int pidx = 0; pidx < npairs; ++pidx) {
        const orc_block *q = &B[pidx / N];
        int t = pidx % N + 1;
        const double *st = state_at(P, x, q->s, t);
        double R[9], pos[3], Cp[MAXROWS * MAXD], dp[MAXROWS], xs[3], alpha, lam[MAXROWS], mu[MAXROWS];
        part_frame(P, st, q->i, q->j, R, pos, Cp, dp);
        const double *A = P->part_A + (size_t)P->part_face_ptr[q->i] * dim;
        const double *b = P->part_b + P->part_face_ptr[q->i];
        bad |= (orc_scale_lp(dim, q->nr, A, b, q->no, Cp, dp, &alpha, xs, lam, mu, NULL) != 0);
        double *yb = y + q->yoff + (t - 1);
        for (int k = 0; k < q->nr; ++k) yb[k * N] = lam[k];
        for (int l = 0; l < q->no; ++l) yb[(q->nr + l) * N] = mu[l];
        yb[(q->n - 1) * N] = alpha > 1.0 ? alpha - 1.0 : 0.0;
        zeta[(size_t)(pidx / N) * N + t - 1] = 0.0;
        for (int r = 0; r < dim; ++r) xi[((size_t)(pidx / N) * dim + r) * N + t - 1] = 0.0;
    }
    free(B);
    return bad;
}

/* Scale alpha* of every pair at the trajectory x (certificate check), and,
   when y_out is not NULL, the LP certificates (lam*, mu*, max(alpha* - 1, 0))
   in the layout of y. */
int orc_scale_all(const orc_problem *P, const double *x, double *alpha_out, double *y_out)
{
    int N = P->N, dim = P->dim, nb = count_blocks(P), bad = 0;
    orc_block *B = (orc_block *)malloc(sizeof(orc_block) * (nb > 0 ? nb : 1));
    enumerate_blocks(P, B);
    #pragma omp parallel for schedule(dynamic, 16) reduction(|:bad)
    for (int pidx = 0; pidx < nb * N; ++pidx) {
        const orc_block *q = &B[pidx / N];
        int t = pidx % N + 1;
        double R[9], pos[3], Cp[MAXROWS * MAXD], dp[MAXROWS], xs[3], lam[MAXROWS], mu[MAXROWS];
        part_frame(P, state_at(P, x, q->s, t), q->i, q->j, R, pos, Cp, dp);
        bad |= (orc_scale_lp(dim, q->nr, P->part_A + (size_t)P->part_face_ptr[q->i] * dim,
                             P->part_b + P->part_face_ptr[q->i], q->no, Cp, dp,
                             &alpha_out[pidx], xs, lam, mu, NULL) != 0);
        if (y_out) {
            double *yb = y_out + q->yoff + (t - 1);
            for (int k = 0; k < q->nr; ++k) yb[k * N] = lam[k];
            for (int l = 0; l < q->no; ++l) yb[(q->nr + l) * N] = mu[l];
            yb[(q->n - 1) * N] = alpha_out[pidx] > 1.0 ? alpha_out[pidx] - 1.0 : 0.0;
        }
    }
    free(B);
    return bad;
}

/* Step 1 (Sec. IV-B eq. ADMM_dual_updates): every pair QP at (s^k, zeta^k,
   xi^k) with proximal centre y^k.  y_in -> y_out. active: per-scenario mask
   (NULL = all). Returns number of failed pair solves. */
int orc_pair_phase(const orc_problem *P, const double *x, const double *y_in,
                   const double *zeta, const double *xi, const unsigned char *active,
                   double *y_out)
{
    int N = P->N, dim = P->dim, nb = count_blocks(P), bad = 0;
    orc_block *B = (orc_block *)malloc(sizeof(orc_block) * (nb > 0 ? nb : 1));
    enumerate_blocks(P, B);
    #pragma omp parallel for schedule(dynamic, 16) reduction(+:bad)
    for (int pidx = 0; pidx < nb * N; ++pidx) {
        const orc_block *q = &B[pidx / N];
        int t = pidx % N + 1;
        if (active && !active[q->s]) continue;
        double R[9], pos[3], Cp[MAXROWS * MAXD], dp[MAXROWS], yh[MAXROWS], yo[MAXROWS], xr[3];
        part_frame(P, state_at(P, x, q->s, t), q->i, q->j, R, pos, Cp, dp);
        for (int l = 0; l < q->n; ++l) yh[l] = y_in[q->yoff + (long)l * N + t - 1];
        for (int r = 0; r < dim; ++r) xr[r] = xi[((size_t)(pidx / N) * dim + r) * N + t - 1];
        int it = orc_pair_qp(dim, q->nr, P->part_A + (size_t)P->part_face_ptr[q->i] * dim,
                             P->part_b + P->part_face_ptr[q->i], q->no, Cp, dp,
                             zeta[(size_t)(pidx / N) * N + t - 1], xr, yh, P->eps_prox, yo);
        if (it < 0) { bad += 1; if (getenv("ORC_DEBUG")) fprintf(stderr, "pair fail block %d t %d\n", pidx / N, t); }
        for (int l = 0; l < q->n; ++l) y_out[q->yoff + (long)l * N + t - 1] = yo[l];
    }
    free(B);
    return bad;
}

/* ------------------------------------------------------------------ */
/* nonlinear dynamics s_{t+1} = s_t + f(s_t, u_t) (Sec. IV-A eq.       */
/* system_eqn) with f = dt f_c, f_c a continuous-time model, and its   */
/* Jacobians by the complex-step derivative                            */
/* ------------------------------------------------------------------ */

/* F(s, u) = s + dt f_c(s, u) in complex arithmetic.
   model 1, kinematic bicycle: s = (p_x, p_y, theta, v), u = (a, delta),
     f_c = (v cos theta, v sin theta, v tan(delta) / L, a); par = (dt, L).
   model 2, quadrotor: s = (p, v, phi theta psi, omega), u = (dF, tau),
     p' = v, v' = (m g + dF) / m R e_3 - g e_3 with R = R_z(psi) R_y(theta) R_x(phi),
     Euler-angle rates from the body rates omega (ZYX), omega' = J^{-1} (tau - omega x J omega);
     par = (dt, m, J_x, J_y, J_z, g). */
static void model_F(const orc_problem *P, const double complex *s, const double complex *u, double complex *F)
{
    const double *par = P->model_par;
    double dt = par[0];
    int n_s = P->n_s;
    double complex f[12];
    if (P->model == 1) {
        f[0] = s[3] * ccos(s[2]);
        f[1] = s[3] * csin(s[2]);
        f[2] = s[3] * ctan(u[1]) / par[1];
        f[3] = u[0];
    } else {
        double m = par[1], Jx = par[2], Jy = par[3], Jz = par[4], g = par[5];
        double complex cph = ccos(s[6]), sph = csin(s[6]), cth = ccos(s[7]), sth = csin(s[7]);
        double complex cps = ccos(s[8]), sps = csin(s[8]);
        double complex thrust = (m * g + u[0]) / m;
        for (int i = 0; i < 3; ++i) f[i] = s[3 + i];
        f[3] = thrust * (cps * sth * cph + sps * sph);
        f[4] = thrust * (sps * sth * cph - cps * sph);
        f[5] = thrust * (cth * cph) - g;
        double complex wx = s[9], wy = s[10], wz = s[11];
        f[6] = wx + (sph * wy + cph * wz) * sth / cth;
        f[7] = cph * wy - sph * wz;
        f[8] = (sph * wy + cph * wz) / cth;
        f[9] = (u[1] - (wy * Jz * wz - wz * Jy * wy)) / Jx;
        f[10] = (u[2] - (wz * Jx * wx - wx * Jz * wz)) / Jy;
        f[11] = (u[3] - (wx * Jy * wy - wy * Jx * wx)) / Jz;
    }
    for (int i = 0; i < n_s; ++i) F[i] = s[i] + dt * f[i];
}

/* F(s, u), A = dF/ds (n_s x n_s) and B = dF/du (n_s x n_u), row-major.
   Derivatives by the complex step: d/dx_j F = Im F(x + i h e_j) / h with
   h = 1e-30, exact to rounding for these analytic f (no difference is
   formed, so no cancellation). */
static void model_linearize(const orc_problem *P, const double *s, const double *u, double *F, double *A, double *B)
{
    int n_s = P->n_s, n_u = P->n_u;
    const double h = 1e-30;
    double complex sc[16] = {0}, uc[8] = {0}, Fc[16];
    for (int i = 0; i < n_s; ++i) sc[i] = s[i];
    for (int j = 0; j < n_u; ++j) uc[j] = u[j];
    model_F(P, sc, uc, Fc);
    for (int i = 0; i < n_s; ++i) F[i] = creal(Fc[i]);
    for (int j = 0; j < n_s + n_u; ++j) {
        if (j < n_s) sc[j] += I * h; else uc[j - n_s] += I * h;
        model_F(P, sc, uc, Fc);
        for (int i = 0; i < n_s; ++i) {
            double d = cimag(Fc[i]) / h;
            if (j < n_s) A[i * n_s + j] = d; else B[i * n_u + (j - n_s)] = d;
        }
        if (j < n_s) sc[j] = s[j]; else uc[j - n_s] = u[j - n_s];
    }
}

/* Test hook: one step of the nonlinear model and its Jacobians. */
int orc_model_step(const orc_problem *P, const double *s, const double *u, double *F, double *A, double *B)
{
    if (P->model != 1 && P->model != 2) return 1;
    model_linearize(P, s, u, F, A, B);
    return 0;
}

/* The model of every step of scenario s linearised about the current
   iterate (x^k_t, u^k_t), t = 0..N-1 (the SQP step): A_t, B_t and
   c_t = F(x^k_t, u^k_t) - A_t x^k_t - B_t u^k_t. */
static void sqp_models(const orc_problem *P, int s, const double *x_in, const double *u_in, double *Al, double *Bl,
                       double *cl)
{
    int n_s = P->n_s, n_u = P->n_u, N = P->N;
    for (int t = 0; t < N; ++t) {
        const double *xt = x_in + ((size_t)s * (N + 1) + t) * n_s;
        const double *ut = u_in + ((size_t)s * N + t) * n_u;
        double *A = Al + (size_t)t * n_s * n_s, *B = Bl + (size_t)t * n_s * n_u, *c = cl + (size_t)t * n_s;
        double F[16];
        model_linearize(P, xt, ut, F, A, B);
        for (int i = 0; i < n_s; ++i) {
            double acc = F[i];
            for (int j = 0; j < n_s; ++j) acc -= A[i * n_s + j] * xt[j];
            for (int j = 0; j < n_u; ++j) acc -= B[i * n_u + j] * ut[j];
            c[i] = acc;
        }
    }
}

/*
 * Step 2 (Sec. IV-B eq. ADMM_state_updates): T and R linearised in the pose
 * coordinates at s^k with y^{k+1}; the penalty sigma/2 ||r + J (q - q^k)||^2
 * is added to the tracking cost and the LQ problem is solved.
 * x_in/u_in = s^k; writes x_out/u_out = s^{k+1}.
 */
int orc_traj_phase(const orc_problem *P, const double *x_in, const double *y,
                   const double *zeta, const double *xi, const unsigned char *active,
                   double *x_out, double *u_out)
{
    int n_s = P->n_s, N = P->N, dim = P->dim, na = n_att(P), nq = dim + na;
    int nb = count_blocks(P), bad = 0;
    orc_block *B = (orc_block *)malloc(sizeof(orc_block) * (nb > 0 ? nb : 1));
    enumerate_blocks(P, B);
    int qidx[6];
    for (int r = 0; r < dim; ++r) qidx[r] = P->pos_idx[r];
    for (int a = 0; a < na; ++a) qidx[dim + a] = P->att_idx[a];
    #pragma omp parallel for schedule(dynamic, 1) reduction(|:bad)
    for (int s = 0; s < P->n_scen; ++s) {
        if (active && !active[s]) {
            memcpy(x_out + (size_t)s * (N + 1) * n_s, x_in + (size_t)s * (N + 1) * n_s, sizeof(double) * (N + 1) * n_s);
            continue;
        }
        double *H = (double *)malloc(sizeof(double) * N * n_s * n_s);
        double *h = (double *)malloc(sizeof(double) * N * n_s);
        double *uo = u_out + (size_t)s * N * P->n_u;
        lq_stage_base(P, s, H, h);
        for (int b = 0; b < nb; ++b) {
            const orc_block *q = &B[b];
            if (q->s != s) continue;
            const double *A = P->part_A + (size_t)P->part_face_ptr[q->i] * dim;
            const double *Cw = P->obs_C + (size_t)P->obs_face_ptr[q->j] * dim;
            const double *o = P->part_off + (size_t)q->i * dim;
            for (int t = 1; t <= N; ++t) {
                const double *st = state_at(P, x_in, s, t);
                const double *yb = y + q->yoff + (t - 1);
                double Rm[9], dR[27];
                rotation(P, st, Rm, dR);
                double T, Rr[3];
                pair_TR(P, q, st, yb, N, &T, Rr);
                double r[4];
                r[0] = T + zeta[(size_t)b * N + t - 1];
                for (int c = 0; c < dim; ++c) r[1 + c] = Rr[c] + xi[((size_t)b * dim + c) * N + t - 1];
                /* cbar = C^T mu (world frame) */
                double cbar[3] = {0, 0, 0};
                for (int l = 0; l < q->no; ++l)
                    for (int c = 0; c < dim; ++c) cbar[c] += Cw[l * dim + c] * yb[(q->nr + l) * N];
                (void)A;
                /* J: (dim+1) x nq in pose coordinates (position, attitude) */
                double J[4 * 6];
                memset(J, 0, sizeof(J));
                for (int c = 0; c < dim; ++c) J[0 * nq + c] = -cbar[c];
                for (int a = 0; a < na; ++a) {
                    const double *dRa = dR + a * dim * dim;
                    double acc = 0.0;
                    for (int r1 = 0; r1 < dim; ++r1)
                        for (int q1 = 0; q1 < dim; ++q1) acc += cbar[r1] * dRa[r1 * dim + q1] * o[q1];
                    J[0 * nq + dim + a] = -acc;
                    for (int c = 0; c < dim; ++c) {
                        double v = 0.0;
                        for (int r1 = 0; r1 < dim; ++r1) v += dRa[r1 * dim + c] * cbar[r1];
                        J[(1 + c) * nq + dim + a] = v;
                    }
                }
                double qk[6];
                for (int a = 0; a < nq; ++a) qk[a] = st[qidx[a]];
                double e[4];
                for (int m = 0; m <= dim; ++m) {
                    double acc = r[m];
                    for (int a = 0; a < nq; ++a) acc -= J[m * nq + a] * qk[a];
                    e[m] = acc;
                }
                double *Ht = H + (size_t)(t - 1) * n_s * n_s;
                double *ht = h + (size_t)(t - 1) * n_s;
                for (int a = 0; a < nq; ++a) {
                    for (int c = 0; c < nq; ++c) {
                        double acc = 0.0;
                        for (int m = 0; m <= dim; ++m) acc += J[m * nq + a] * J[m * nq + c];
                        Ht[qidx[a] * n_s + qidx[c]] += P->sigma * acc;
                    }
                    double acc = 0.0;
                    for (int m = 0; m <= dim; ++m) acc += J[m * nq + a] * e[m];
                    ht[qidx[a]] += P->sigma * acc;
                }
            }
        }
        if (P->model) {
            /* the SQP step: f linearised about the current iterate (u_out
               holds u^k on entry) */
            double *Al = (double *)malloc(sizeof(double) * N * n_s * n_s);
            double *Bl = (double *)malloc(sizeof(double) * N * n_s * P->n_u);
            double *cl = (double *)malloc(sizeof(double) * N * n_s);
            sqp_models(P, s, x_in, u_out, Al, Bl, cl);
            bad |= traj_solve(P, s, Al, Bl, cl, 1, H, h, x_out + (size_t)s * (N + 1) * n_s, uo);
            free(Al); free(Bl); free(cl);
        } else {
            bad |= traj_solve(P, s, dyn_A(P, s), dyn_B(P, s), dyn_c(P, s), P->dyn_ts, H, h,
                              x_out + (size_t)s * (N + 1) * n_s, uo);
        }
        free(H); free(h);
    }
    free(B);
    return bad;
}

/* Step 3 (Sec. IV-B eq. ADMM_residue_updates): zeta += T(s^{k+1}, y^{k+1}),
   xi += R(s^{k+1}, y^{k+1}); accumulates per-scenario sum of squared
   multiplier changes into rpri (n_scen). */
void orc_mult_phase(const orc_problem *P, const double *x, const double *y,
                    const unsigned char *active, double *zeta, double *xi, double *rpri)
{
    int N = P->N, dim = P->dim, nb = count_blocks(P);
    orc_block *B = (orc_block *)malloc(sizeof(orc_block) * (nb > 0 ? nb : 1));
    enumerate_blocks(P, B);
    for (int s = 0; s < P->n_scen; ++s) rpri[s] = 0.0;
    for (int b = 0; b < nb; ++b) {
        const orc_block *q = &B[b];
        if (active && !active[q->s]) continue;
        for (int t = 1; t <= N; ++t) {
            double T, Rr[3];
            pair_TR(P, q, state_at(P, x, q->s, t), y + q->yoff + (t - 1), N, &T, Rr);
            zeta[(size_t)b * N + t - 1] += T;
            double acc = T * T;
            for (int c = 0; c < dim; ++c) {
                xi[((size_t)b * dim + c) * N + t - 1] += Rr[c];
                acc += Rr[c] * Rr[c];
            }
            rpri[q->s] += acc;
        }
    }
    free(B);
}

/* Tracking cost F (Sec. IV-A eq. navigation_cost) over x_{1..N}, u_{0..N-1}. */
double orc_cost(const orc_problem *P, int s, const double *x, const double *u)
{
    int n_s = P->n_s, n_u = P->n_u, N = P->N;
    double F = 0.0;
    for (int t = 1; t <= N; ++t) {
        const double *xt = x + ((size_t)s * (N + 1) + t) * n_s;
        const double *xr = P->x_ref + ((size_t)s * (N + 1) + t) * n_s;
        for (int r = 0; r < n_s; ++r)
            for (int q = 0; q < n_s; ++q) F += (xt[r] - xr[r]) * P->Q_s[r * n_s + q] * (xt[q] - xr[q]);
    }
    for (int t = 0; t < N; ++t) {
        const double *ut = u + ((size_t)s * N + t) * n_u;
        for (int r = 0; r < n_u; ++r)
            for (int q = 0; q < n_u; ++q) F += ut[r] * P->Q_u[r * n_u + q] * ut[q];
    }
    return F;
}

/*
 * Full ADMM run from the given iterate (x, u, y, zeta, xi) for at most
 * max_iters iterations; each scenario stops at the first iteration at which
 * both sums of squares fall below eps_pri and eps_dual (Sec. IV-B) and is
 * left unchanged afterwards.  hist_* (max_iters x n_scen, may be NULL)
 * receive r_pri, r_dual and F per iteration; iters_out (n_scen) the number of
 * iterations each scenario ran. Returns the number of failed sub-solves.
 */
int orc_admm_run(const orc_problem *P, int max_iters, double *x, double *u, double *y,
                 double *zeta, double *xi, double *hist_pri, double *hist_dual, double *hist_cost,
                 int *iters_out)
{
    int S = P->n_scen, N = P->N, dim = P->dim;
    long ny = orc_y_size(P);
    int nb = count_blocks(P);
    orc_block *B = (orc_block *)malloc(sizeof(orc_block) * (nb > 0 ? nb : 1));
    enumerate_blocks(P, B);
    double *ynew = (double *)malloc(sizeof(double) * (ny > 0 ? ny : 1));
    double *xnew = (double *)malloc(sizeof(double) * S * (N + 1) * P->n_s);
    double *rpri = (double *)calloc(S, sizeof(double));
    double *rdual = (double *)calloc(S, sizeof(double));
    unsigned char *active = (unsigned char *)malloc(S);
    int bad = 0;
    for (int s = 0; s < S; ++s) { active[s] = 1; iters_out[s] = 0; }
    for (int k = 0; k < max_iters; ++k) {
        int any = 0;
        for (int s = 0; s < S; ++s) any |= active[s];
        if (!any) break;
        memcpy(ynew, y, sizeof(double) * ny);
        bad += orc_pair_phase(P, x, y, zeta, xi, active, ynew);
        bad += orc_traj_phase(P, x, ynew, zeta, xi, active, xnew, u);
        for (int s = 0; s < S; ++s) rdual[s] = 0.0;
        for (int b = 0; b < nb; ++b) {
            const orc_block *q = &B[b];
            if (!active[q->s]) continue;
            for (int l = 0; l < q->n - 1; ++l)      /* lambda and mu rows only */
                for (int t = 0; t < N; ++t) {
                    double dlt = ynew[q->yoff + (long)l * N + t] - y[q->yoff + (long)l * N + t];
                    rdual[q->s] += dlt * dlt;
                }
        }
        memcpy(y, ynew, sizeof(double) * ny);
        memcpy(x, xnew, sizeof(double) * S * (N + 1) * P->n_s);
        orc_mult_phase(P, x, y, active, zeta, xi, rpri);
        for (int s = 0; s < S; ++s) {
            if (!active[s]) {
                if (hist_pri) { hist_pri[k * S + s] = NAN; hist_dual[k * S + s] = NAN; hist_cost[k * S + s] = NAN; }
                continue;
            }
            iters_out[s] = k + 1;
            if (hist_pri) {
                hist_pri[k * S + s] = rpri[s];
                hist_dual[k * S + s] = rdual[s];
                hist_cost[k * S + s] = orc_cost(P, s, x, u);
            }
            if (rpri[s] <= P->eps_pri && rdual[s] <= P->eps_dual) active[s] = 0;
        }
    }
    (void)dim;
    free(B); free(ynew); free(xnew); free(rpri); free(rdual); free(active);
    return bad;
}

int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* reverse-mode gradient through the unrolled iteration                */
/* ------------------------------------------------------------------ */

/*
 * Second derivatives d2R/d(att_a)d(att_b), a, b < n_att, stored [a][b][dim*dim].
 * Planar: d2R/dtheta2 = -R. ZYX Euler R = Rz(psi) Ry(theta) Rx(phi): products
 * of the factor matrices and their first and second derivatives.
 */
static void rotation_dd(const orc_problem *P, const double *s, double *ddR)
{
    if (P->att_kind == 0) {
        double th = s[P->att_idx[0]], c = cos(th), sn = sin(th);
        ddR[0] = -c; ddR[1] = sn; ddR[2] = -sn; ddR[3] = -c;
        return;
    }
    double ph = s[P->att_idx[0]], th = s[P->att_idx[1]], ps = s[P->att_idx[2]];
    double cf = cos(ph), sf = sin(ph), ct = cos(th), st = sin(th), cp = cos(ps), sp = sin(ps);
    double X[3][9] = {{1, 0, 0, 0, cf, -sf, 0, sf, cf},
                      {0, 0, 0, 0, -sf, -cf, 0, cf, -sf},
                      {0, 0, 0, 0, -cf, sf, 0, -sf, -cf}};
    double Y[3][9] = {{ct, 0, st, 0, 1, 0, -st, 0, ct},
                      {-st, 0, ct, 0, 0, 0, -ct, 0, -st},
                      {-ct, 0, -st, 0, 0, 0, st, 0, -ct}};
    double Z[3][9] = {{cp, -sp, 0, sp, cp, 0, 0, 0, 1},
                      {-sp, -cp, 0, cp, -sp, 0, 0, 0, 0},
                      {-cp, sp, 0, -sp, -cp, 0, 0, 0, 0}};
    /* derivative orders of (phi, theta, psi) for each (a, b) */
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            int o[3] = {0, 0, 0};
            o[a] += 1;
            o[b] += 1;
            const double *F1 = Z[o[2]], *F2 = Y[o[1]], *F3 = X[o[0]];
            double T1[9];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double acc = 0;
                    for (int k = 0; k < 3; ++k) acc += F1[i * 3 + k] * F2[k * 3 + j];
                    T1[i * 3 + j] = acc;
                }
            double *out = ddR + (a * 3 + b) * 9;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double acc = 0;
                    for (int k = 0; k < 3; ++k) acc += T1[i * 3 + k] * F3[k * 3 + j];
                    out[i * 3 + j] = acc;
                }
        }
}

/* T, R and their Jacobian J ((dim+1) x nq, pose coordinates) of one pair at
   state st with dual rows yb (stride between rows); also cbar = C^T mu. */
static void pair_lin(const orc_problem *P, const orc_block *q, const double *st, const double *yb, int stride,
                     double *T, double *Rr, double *J, double *cbar)
{
    int dim = P->dim, na = n_att(P), nq = dim + na;
    double Rm[9], dR[27];
    rotation(P, st, Rm, dR);
    pair_TR(P, q, st, yb, stride, T, Rr);
    const double *Cw = P->obs_C + (size_t)P->obs_face_ptr[q->j] * dim;
    const double *o = P->part_off + (size_t)q->i * dim;
    for (int c = 0; c < dim; ++c) cbar[c] = 0.0;
    for (int l = 0; l < q->no; ++l)
        for (int c = 0; c < dim; ++c) cbar[c] += Cw[l * dim + c] * yb[(q->nr + l) * stride];
    for (int i = 0; i < (dim + 1) * nq; ++i) J[i] = 0.0;
    for (int c = 0; c < dim; ++c) J[c] = -cbar[c];
    for (int a = 0; a < na; ++a) {
        const double *dRa = dR + a * dim * dim;
        double acc = 0.0;
        for (int r = 0; r < dim; ++r)
            for (int c = 0; c < dim; ++c) acc += cbar[r] * dRa[r * dim + c] * o[c];
        J[dim + a] = -acc;
        for (int c = 0; c < dim; ++c) {
            double v = 0.0;
            for (int r = 0; r < dim; ++r) v += dRa[r * dim + c] * cbar[r];
            J[(1 + c) * nq + dim + a] = v;
        }
    }
}

/* Adjoint of J through cbar (dual rows mu) and through the attitude
   (second derivatives of R). Adds into ybar (rows, stride) and qbar (nq). */
static void jac_adjoint(const orc_problem *P, const orc_block *q, const double *st, const double *yb, int stride,
                        const double *Jbar, double *ybar, int ystride, double *qbar)
{
    int dim = P->dim, na = n_att(P), nq = dim + na;
    double Rm[9], dR[27], ddR[81];
    rotation(P, st, Rm, dR);
    rotation_dd(P, st, ddR);
    const double *Cw = P->obs_C + (size_t)P->obs_face_ptr[q->j] * dim;
    const double *o = P->part_off + (size_t)q->i * dim;
    double cbar[3] = {0, 0, 0};
    for (int l = 0; l < q->no; ++l)
        for (int c = 0; c < dim; ++c) cbar[c] += Cw[l * dim + c] * yb[(q->nr + l) * stride];
    double cbb[3] = {0, 0, 0};
    for (int c = 0; c < dim; ++c) cbb[c] -= Jbar[c];
    for (int a = 0; a < na; ++a) {
        const double *dRa = dR + a * dim * dim;
        for (int r = 0; r < dim; ++r) {
            double dro = 0.0;
            for (int c = 0; c < dim; ++c) dro += dRa[r * dim + c] * o[c];
            cbb[r] -= Jbar[dim + a] * dro;
            for (int c = 0; c < dim; ++c) cbb[r] += Jbar[(1 + c) * nq + dim + a] * dRa[r * dim + c];
        }
    }
    for (int l = 0; l < q->no; ++l) {
        double acc = 0.0;
        for (int c = 0; c < dim; ++c) acc += Cw[l * dim + c] * cbb[c];
        ybar[(q->nr + l) * ystride] += acc;
    }
    for (int b = 0; b < na; ++b) {
        double acc = 0.0;
        for (int a = 0; a < na; ++a) {
            const double *dd = ddR + (a * na + b) * dim * dim;
            double t0 = 0.0;
            for (int r = 0; r < dim; ++r)
                for (int c = 0; c < dim; ++c) t0 += cbar[r] * dd[r * dim + c] * o[c];
            acc -= Jbar[dim + a] * t0;
            for (int c = 0; c < dim; ++c) {
                double v = 0.0;
                for (int r = 0; r < dim; ++r) v += dd[r * dim + c] * cbar[r];
                acc += Jbar[(1 + c) * nq + dim + a] * v;
            }
        }
        qbar[dim + b] += acc;
    }
    (void)Rm;
}

/* Adjoint of (T, R) at (st, y) for the row weights (tb, rb[dim]): adds into
   ybar rows, qbar and the obstacle-offset gradient dbar (faces of q->j). */
static void TR_adjoint(const orc_problem *P, const orc_block *q, const double *st, const double *yb, int stride,
                       double tb, const double *rb, double *ybar, int ystride, double *qbar, double *dbar)
{
    int dim = P->dim, nq = dim + n_att(P);
    double R[9], pos[3], Cp[MAXROWS * MAXD], dp[MAXROWS], T, Rr[3], J[4 * 6], cbar[3];
    part_frame(P, st, q->i, q->j, R, pos, Cp, dp);
    const double *A = P->part_A + (size_t)P->part_face_ptr[q->i] * dim;
    for (int k = 0; k < q->nr; ++k) {
        double acc = 0.0;
        for (int r = 0; r < dim; ++r) acc += A[k * dim + r] * rb[r];
        ybar[k * ystride] += acc;
    }
    for (int l = 0; l < q->no; ++l) {
        double acc = dp[l] * tb;
        for (int r = 0; r < dim; ++r) acc += Cp[l * dim + r] * rb[r];
        ybar[(q->nr + l) * ystride] += acc;
        dbar[P->obs_face_ptr[q->j] + l] += yb[(q->nr + l) * stride] * tb;
    }
    ybar[(q->n - 1) * ystride] += tb;
    pair_lin(P, q, st, yb, stride, &T, Rr, J, cbar);
    for (int a = 0; a < nq; ++a) {
        double acc = J[a] * tb;
        for (int r = 0; r < dim; ++r) acc += J[(1 + r) * nq + a] * rb[r];
        qbar[a] += acc;
    }
}

/* Adjoint of one proximal pair QP on its active set (dense KKT transpose).
   ybar_new (rows of y^{k+1}) -> adds into ybar_old (rows of yhat = y^k),
   zb (zeta^k), xib[dim] (xi^k), qbar (pose at s^k) and dbar. */
static int pairqp_adjoint(const orc_problem *P, const orc_block *q, const double *st, const double *yhat,
                          const double *ynew, int stride, double zeta, const double *xi, const double *ybar_new,
                          double *ybar_old, int ystride, double *zb, double *xib, double *qbar, double *dbar)
{
    int dim = P->dim, na = n_att(P), c = dim + 1, n = q->n;
    double R[9], dR[27], pos[3], Cp[MAXROWS * MAXD], dp[MAXROWS];
    part_frame(P, st, q->i, q->j, R, pos, Cp, dp);
    rotation(P, st, R, dR);
    const double *A = P->part_A + (size_t)P->part_face_ptr[q->i] * dim;
    const double *b = P->part_b + P->part_face_ptr[q->i];
    double K[MAXROWS * (MAXD + 1)];
    build_K(dim, q->nr, A, q->no, Cp, dp, K);
    double bh[MAXD + 1], D[MAXROWS], kap[MAXROWS], y[MAXROWS], yh[MAXROWS], yb[MAXROWS];
    bh[0] = 1.0 + zeta;
    for (int r = 0; r < dim; ++r) bh[1 + r] = xi[r];
    for (int l = 0; l < n; ++l) {
        double s = 0.0;
        for (int m = 0; m < c; ++m) s += K[l * c + m] * K[l * c + m];
        D[l] = s;
        kap[l] = l < q->nr ? b[l] : 0.0;
        y[l] = ynew[l * stride];
        yh[l] = yhat[l * stride];
        yb[l] = ybar_new[l * ystride];
    }
    int F[MAXROWS], nf = 0;
    for (int l = 0; l < n; ++l) if (y[l] > 0.0) F[nf++] = l;
    /* transposed KKT on the free set: [G_FF kap_F; -kap_F^T 0] [a; beta] = [ybar_F; 0] */
    int sz = nf + 1;
    double M[(MAXROWS + 1) * (MAXROWS + 1)], rhs[MAXROWS + 1];
    for (int i2 = 0; i2 < nf; ++i2) {
        for (int j2 = 0; j2 < nf; ++j2) {
            double s = 0.0;
            for (int m = 0; m < c; ++m) s += K[F[i2] * c + m] * K[F[j2] * c + m];
            M[i2 * sz + j2] = s + (i2 == j2 ? P->eps_prox * D[F[i2]] : 0.0);
        }
        M[i2 * sz + nf] = kap[F[i2]];
        M[nf * sz + i2] = -kap[F[i2]];
        rhs[i2] = yb[F[i2]];
    }
    M[nf * sz + nf] = 0.0;
    rhs[nf] = 0.0;
    if (gauss_solve(sz, M, rhs)) return 1;
    double gbar[MAXROWS] = {0}, Kbar[MAXROWS * (MAXD + 1)] = {0}, Dbar[MAXROWS] = {0};
    for (int i2 = 0; i2 < nf; ++i2) gbar[F[i2]] = -rhs[i2];
    /* Gbar = -a y^T on F x F:  K^bar += (Gbar + Gbar^T) K, Dbar_l += eps Gbar_ll */
    for (int i2 = 0; i2 < nf; ++i2) {
        int l = F[i2];
        double al = rhs[i2];
        /* (Gbar K)_l = -a_l (y^T K) ; (Gbar^T K)_l = -y_l (a^T K) */
        for (int m = 0; m < c; ++m) {
            double yK = 0.0, aK = 0.0;
            for (int j2 = 0; j2 < nf; ++j2) {
                yK += y[F[j2]] * K[F[j2] * c + m];
                aK += rhs[j2] * K[F[j2] * c + m];
            }
            Kbar[l * c + m] += -al * yK - y[l] * aK;
        }
        Dbar[l] += P->eps_prox * (-al * y[l]);
    }
    /* g = K bh - eps D yhat */
    double bhbar[MAXD + 1] = {0};
    for (int l = 0; l < n; ++l) {
        if (gbar[l] == 0.0) continue;
        for (int m = 0; m < c; ++m) {
            Kbar[l * c + m] += gbar[l] * bh[m];
            bhbar[m] += K[l * c + m] * gbar[l];
        }
        Dbar[l] += -P->eps_prox * gbar[l] * yh[l];
        ybar_old[l * ystride] += -P->eps_prox * D[l] * gbar[l];
    }
    for (int l = 0; l < n; ++l)
        for (int m = 0; m < c; ++m) Kbar[l * c + m] += 2.0 * Dbar[l] * K[l * c + m];
    *zb += bhbar[0];
    for (int r = 0; r < dim; ++r) xib[r] += bhbar[1 + r];
    /* K rows of the obstacle: (dp_l, Cp_l) with dp = d - C pos, Cp_l = c_l^T R */
    const double *Cw = P->obs_C + (size_t)P->obs_face_ptr[q->j] * dim;
    const double *o = P->part_off + (size_t)q->i * dim;
    double posbar[3] = {0, 0, 0}, Rbar[9] = {0};
    for (int l = 0; l < q->no; ++l) {
        const double *Kb = Kbar + (q->nr + l) * c;
        dbar[P->obs_face_ptr[q->j] + l] += Kb[0];
        for (int r = 0; r < dim; ++r) posbar[r] -= Kb[0] * Cw[l * dim + r];
        /* Cp_lq = sum_r c_lr R_rq */
        for (int r = 0; r < dim; ++r)
            for (int m = 0; m < dim; ++m) Rbar[r * dim + m] += Cw[l * dim + r] * Kb[1 + m];
    }
    /* pos = rho + R o */
    for (int r = 0; r < dim; ++r) {
        qbar[r] += posbar[r];
        for (int m = 0; m < dim; ++m) Rbar[r * dim + m] += posbar[r] * o[m];
    }
    for (int a = 0; a < na; ++a) {
        double acc = 0.0;
        for (int i2 = 0; i2 < dim * dim; ++i2) acc += Rbar[i2] * dR[a * dim * dim + i2];
        qbar[dim + a] += acc;
    }
    return 0;
}

/* Adjoint of the condensed LQ solve. Inputs: stage H (N blocks), the
   solution (x, u), and the adjoint (xbar over t = 1..N, ubar). Outputs: w
   (N x n_s, = M abar), and adds x0bar. Hbar_t = -1/2 (w_t x_t^T + x_t w_t^T),
   hbar_t = -w_t are formed by the caller from w. */
static int lq_adjoint(int n_s, int n_u, int N, const double *A0, const double *B0, int ts, const double *H,
                      const double *Q_u, const double *xbar, const double *ubar, double *w, double *x0bar)
{
    int nU = N * n_u;
    double *Mt = (double *)calloc((size_t)N * n_s * nU, sizeof(double));
    double *Hs = (double *)calloc((size_t)nU * nU, sizeof(double));
    double *HM = (double *)calloc((size_t)n_s * nU, sizeof(double));
    double *ab = (double *)calloc(nU, sizeof(double));
    double *zb = (double *)calloc((size_t)(N + 1) * n_s, sizeof(double));
    for (int t = 1; t <= N; ++t) {
        double *Mc = Mt + (size_t)(t - 1) * n_s * nU;
        const double *Mp = (t >= 2) ? Mt + (size_t)(t - 2) * n_s * nU : NULL;
        const double *A = A0 + (size_t)(t - 1) * ts * n_s * n_s, *B = B0 + (size_t)(t - 1) * ts * n_s * n_u;
        for (int r = 0; r < n_s; ++r) {
            for (int col = 0; col < nU; ++col) {
                double a = 0.0;
                if (Mp) for (int q2 = 0; q2 < n_s; ++q2) a += A[r * n_s + q2] * Mp[q2 * nU + col];
                Mc[r * nU + col] = a;
            }
            for (int k = 0; k < n_u; ++k) Mc[r * nU + (t - 1) * n_u + k] += B[r * n_u + k];
        }
    }
    for (int k = 0; k < N; ++k)
        for (int a = 0; a < n_u; ++a)
            for (int b2 = 0; b2 < n_u; ++b2) Hs[(k * n_u + a) * nU + k * n_u + b2] = 2.0 * Q_u[a * n_u + b2];
    for (int a = 0; a < nU; ++a) ab[a] = ubar ? ubar[a] : 0.0;
    for (int t = 1; t <= N; ++t) {
        const double *Mc = Mt + (size_t)(t - 1) * n_s * nU;
        const double *Ht = H + (size_t)(t - 1) * n_s * n_s;
        for (int r = 0; r < n_s; ++r)
            for (int col = 0; col < nU; ++col) {
                double a = 0.0;
                for (int q2 = 0; q2 < n_s; ++q2) a += Ht[r * n_s + q2] * Mc[q2 * nU + col];
                HM[r * nU + col] = a;
            }
        for (int a = 0; a < nU; ++a) {
            for (int b2 = 0; b2 < nU; ++b2) {
                double acc = 0.0;
                for (int r = 0; r < n_s; ++r) acc += Mc[r * nU + a] * HM[r * nU + b2];
                Hs[a * nU + b2] += acc;
            }
            double acc = 0.0;
            for (int r = 0; r < n_s; ++r) acc += Mc[r * nU + a] * xbar[(size_t)(t - 1) * n_s + r];
            ab[a] += acc;
        }
    }
    int st = chol_solve(nU, Hs, ab);   /* abar = Hs^{-1} (ubar + sum M^T xbar) */
    if (!st) {
        for (int t = 1; t <= N; ++t) {
            const double *Mc = Mt + (size_t)(t - 1) * n_s * nU;
            const double *Ht = H + (size_t)(t - 1) * n_s * n_s;
            double *wt = w + (size_t)(t - 1) * n_s;
            for (int r = 0; r < n_s; ++r) {
                double acc = 0.0;
                for (int a = 0; a < nU; ++a) acc += Mc[r * nU + a] * ab[a];
                wt[r] = acc;
            }
            /* zbar_t = xbar_t - H_t w_t */
            for (int r = 0; r < n_s; ++r) {
                double acc = xbar[(size_t)(t - 1) * n_s + r];
                for (int q2 = 0; q2 < n_s; ++q2) acc -= Ht[r * n_s + q2] * wt[q2];
                zb[t * n_s + r] = acc;
            }
        }
        /* z_t = A_{t-1} z_{t-1} + c_{t-1}, z_0 = x0: backpropagate zbar to x0 */
        for (int t = N; t >= 1; --t) {
            const double *A = A0 + (size_t)(t - 1) * ts * n_s * n_s;
            for (int q2 = 0; q2 < n_s; ++q2) {
                double acc = 0.0;
                for (int r = 0; r < n_s; ++r) acc += A[r * n_s + q2] * zb[t * n_s + r];
                zb[(t - 1) * n_s + q2] += acc;
            }
        }
        for (int r = 0; r < n_s; ++r) x0bar[r] += zb[r];
    }
    free(Mt); free(Hs); free(HM); free(ab); free(zb);
    return st;
}

/* Stage terms of the trajectory QP of iteration k for scenario s (as in
   orc_traj_phase): H (N blocks), h (N x n_s). */
static void traj_stage(const orc_problem *P, const orc_block *B, int nb, int s, const double *x_in,
                       const double *y, const double *zeta, const double *xi, double *H, double *h)
{
    int n_s = P->n_s, N = P->N, dim = P->dim, nq = dim + n_att(P);
    int qidx[6];
    for (int r = 0; r < dim; ++r) qidx[r] = P->pos_idx[r];
    for (int a = 0; a < n_att(P); ++a) qidx[dim + a] = P->att_idx[a];
    lq_stage_base(P, s, H, h);
    for (int b = 0; b < nb; ++b) {
        const orc_block *q = &B[b];
        if (q->s != s) continue;
        for (int t = 1; t <= N; ++t) {
            const double *st = state_at(P, x_in, s, t);
            double T, Rr[3], J[24], cbar[3], r[4], e[4], qk[6];
            pair_lin(P, q, st, y + q->yoff + (t - 1), N, &T, Rr, J, cbar);
            r[0] = T + zeta[(size_t)b * N + t - 1];
            for (int c = 0; c < dim; ++c) r[1 + c] = Rr[c] + xi[((size_t)b * dim + c) * N + t - 1];
            for (int a = 0; a < nq; ++a) qk[a] = st[qidx[a]];
            for (int m = 0; m <= dim; ++m) {
                double acc = r[m];
                for (int a = 0; a < nq; ++a) acc -= J[m * nq + a] * qk[a];
                e[m] = acc;
            }
            double *Ht = H + (size_t)(t - 1) * n_s * n_s, *ht = h + (size_t)(t - 1) * n_s;
            for (int a = 0; a < nq; ++a) {
                for (int c2 = 0; c2 < nq; ++c2) {
                    double acc = 0.0;
                    for (int m = 0; m <= dim; ++m) acc += J[m * nq + a] * J[m * nq + c2];
                    Ht[qidx[a] * n_s + qidx[c2]] += P->sigma * acc;
                }
                double acc = 0.0;
                for (int m = 0; m <= dim; ++m) acc += J[m * nq + a] * e[m];
                ht[qidx[a]] += P->sigma * acc;
            }
        }
    }
}


/* Adjoint of the trajectory phase (x^k, y^{k+1}, zeta^k, xi^k) -> (x^{k+1},
   u^{k+1}). Consumes xb (adjoint of x^{k+1}, zeroed on return) and ub
   (adjoint of u^{k+1}, zeroed); adds into yb (y^{k+1}), zbar, xibar
   (zeta^k, xi^k), qbar (pose coordinates of x^k, per pair), dbar and x0bar. */
static int traj_adjoint(const orc_problem *P, const orc_block *B, int nb, const double *Xk, const double *Xn,
                        const double *Yn, const double *Zk, const double *XIk, double *xb, double *ub, double *yb,
                        double *zbar, double *xibar, double *qbar, double *grad_d, double *grad_x0)
{
    int S = P->n_scen, N = P->N, n_s = P->n_s, n_u = P->n_u, dim = P->dim, nq = dim + n_att(P), bad = 0;
    int qidx[6];
    for (int r = 0; r < dim; ++r) qidx[r] = P->pos_idx[r];
    for (int a = 0; a < n_att(P); ++a) qidx[dim + a] = P->att_idx[a];
    double *H = (double *)malloc(sizeof(double) * N * n_s * n_s), *h = (double *)malloc(sizeof(double) * N * n_s);
    double *w = (double *)malloc(sizeof(double) * N * n_s), *xbt = (double *)malloc(sizeof(double) * N * n_s);
        for (int s = 0; s < S; ++s) {
        traj_stage(P, B, nb, s, Xk, Yn, Zk, XIk, H, h);
        for (int t = 1; t <= N; ++t)
            for (int r = 0; r < n_s; ++r) xbt[(t - 1) * n_s + r] = xb[((size_t)s * (N + 1) + t) * n_s + r];
        bad += lq_adjoint(n_s, n_u, N, dyn_A(P, s), dyn_B(P, s), P->dyn_ts, H, P->Q_u, xbt, ub + (size_t)s * N * n_u, w,
                          grad_x0 + (size_t)s * n_s);
        /* x^{k+1} and u^{k+1} do not depend on x^k, u^k except through the stage terms */
        for (int t = 0; t <= N; ++t)
            for (int r = 0; r < n_s; ++r) xb[((size_t)s * (N + 1) + t) * n_s + r] = 0.0;
        for (int i = 0; i < N * n_u; ++i) ub[(size_t)s * N * n_u + i] = 0.0;
        for (int b = 0; b < nb; ++b) {
            const orc_block *q = &B[b];
            if (q->s != s) continue;
            for (int t = 1; t <= N; ++t) {
                const double *st = state_at(P, Xk, s, t);
                const double *xt1 = state_at(P, Xn, s, t);
                const double *wt = w + (size_t)(t - 1) * n_s;
                double T, Rr[3], J[24], cbar[3], r[4], ep[4], qk[6], wq[6], xq[6];
                pair_lin(P, q, st, Yn + q->yoff + t - 1, N, &T, Rr, J, cbar);
                r[0] = T + Zk[(size_t)b * N + t - 1];
                for (int c2 = 0; c2 < dim; ++c2) r[1 + c2] = Rr[c2] + XIk[((size_t)b * dim + c2) * N + t - 1];
                for (int a = 0; a < nq; ++a) { qk[a] = st[qidx[a]]; wq[a] = wt[qidx[a]]; xq[a] = xt1[qidx[a]]; }
                for (int m = 0; m <= dim; ++m) {
                    double acc = r[m];
                    for (int a = 0; a < nq; ++a) acc -= J[m * nq + a] * qk[a];
                    ep[m] = acc;
                }
                /* Hbar (pose block) = -1/2 (w x^T + x w^T), hbar = -w */
                double Hb[36], hb[6];
                for (int a = 0; a < nq; ++a) {
                    hb[a] = -wq[a];
                    for (int c2 = 0; c2 < nq; ++c2) Hb[a * nq + c2] = -0.5 * (wq[a] * xq[c2] + xq[a] * wq[c2]);
                }
                /* H += sigma J^T J ; h += sigma J^T (e - J q^k), e = r */
                double Jb[24] = {0}, eb[4] = {0}, qb[6] = {0};
                for (int m = 0; m <= dim; ++m)
                    for (int a = 0; a < nq; ++a) {
                        double acc = 0.0;
                        for (int c2 = 0; c2 < nq; ++c2) acc += J[m * nq + c2] * (Hb[c2 * nq + a] + Hb[a * nq + c2]);
                        Jb[m * nq + a] += P->sigma * acc;
                    }
                double Jh[4] = {0};
                for (int m = 0; m <= dim; ++m)
                    for (int a = 0; a < nq; ++a) Jh[m] += J[m * nq + a] * hb[a];
                for (int m = 0; m <= dim; ++m) {
                    for (int a = 0; a < nq; ++a) Jb[m * nq + a] += P->sigma * (ep[m] * hb[a] - Jh[m] * qk[a]);
                    eb[m] += P->sigma * Jh[m];
                }
                for (int a = 0; a < nq; ++a) {
                    double acc = 0.0;
                    for (int m = 0; m <= dim; ++m) acc += J[m * nq + a] * Jh[m];
                    qb[a] -= P->sigma * acc;
                }
                /* e = (T + zeta, R + xi) at (s^k, y^{k+1}) */
                zbar[(size_t)b * N + t - 1] += eb[0];
                for (int c2 = 0; c2 < dim; ++c2) xibar[((size_t)b * dim + c2) * N + t - 1] += eb[1 + c2];
                TR_adjoint(P, q, st, Yn + q->yoff + t - 1, N, eb[0], eb + 1, yb + q->yoff + t - 1, N, qb, grad_d);
                jac_adjoint(P, q, st, Yn + q->yoff + t - 1, N, Jb, yb + q->yoff + t - 1, N, qb);
                for (int a = 0; a < nq; ++a) qbar[((size_t)b * N + t - 1) * nq + a] += qb[a];
            }
        }
    }
    free(H); free(h); free(w); free(xbt);
    return bad;
}

/* The reverse pass of orc_admm_grad over stored iterates: X, U, Y, Zt, XI
 * hold the iterates k = 0..K (x^k, u^k, y^k, zeta^k, xi^k) back to back.
 * Writes L = sum_s F_s(x^K, u^K) and the gradients; returns the number of
 * failed solves. */
static int admm_reverse(const orc_problem *P, int K, const double *X, const double *U, const double *Y,
                        const double *Zt, const double *XI, double *L_out, double *grad_d, double *grad_x0)
{
    int S = P->n_scen, N = P->N, n_s = P->n_s, n_u = P->n_u, dim = P->dim, nq = dim + n_att(P);
    int nb = count_blocks(P), bad = 0;
    long ny = orc_y_size(P), npair = (long)nb * N;
    size_t nx = (size_t)S * (N + 1) * n_s, nu_ = (size_t)S * N * n_u;
    orc_block *B = (orc_block *)malloc(sizeof(orc_block) * (nb > 0 ? nb : 1));
    enumerate_blocks(P, B);
    double L = 0.0;
    for (int s = 0; s < S; ++s) L += orc_cost(P, s, X + nx * K, U + nu_ * K);
    *L_out = L;
    /* adjoints */
    double *xb = (double *)calloc(nx, sizeof(double)), *ub = (double *)calloc(nu_, sizeof(double));
    double *yb = (double *)calloc(ny > 0 ? ny : 1, sizeof(double)), *yb_old = (double *)calloc(ny > 0 ? ny : 1, sizeof(double));
    double *zbar = (double *)calloc(npair > 0 ? npair : 1, sizeof(double));
    double *xibar = (double *)calloc((npair > 0 ? npair : 1) * dim, sizeof(double));
    double *qbar = (double *)calloc((size_t)(npair > 0 ? npair : 1) * nq, sizeof(double));
    int Fo = P->obs_face_ptr[P->obs_ptr[S]];
    for (int i = 0; i < Fo; ++i) grad_d[i] = 0.0;
    for (int i = 0; i < S * n_s; ++i) grad_x0[i] = 0.0;
    int qidx[6];
    for (int r = 0; r < dim; ++r) qidx[r] = P->pos_idx[r];
    for (int a = 0; a < n_att(P); ++a) qidx[dim + a] = P->att_idx[a];
    /* dL/dx^K, dL/du^K of F = sum (x - xref)^T Q_s (x - xref) + u^T Q_u u */
    for (int s = 0; s < S; ++s) {
        for (int t = 1; t <= N; ++t) {
            const double *xt = X + nx * K + ((size_t)s * (N + 1) + t) * n_s;
            const double *xr = P->x_ref + ((size_t)s * (N + 1) + t) * n_s;
            for (int r = 0; r < n_s; ++r) {
                double acc = 0.0;
                for (int q2 = 0; q2 < n_s; ++q2) acc += 2.0 * P->Q_s[r * n_s + q2] * (xt[q2] - xr[q2]);
                xb[((size_t)s * (N + 1) + t) * n_s + r] = acc;
            }
        }
        for (int t = 0; t < N; ++t) {
            const double *ut = U + nu_ * K + ((size_t)s * N + t) * n_u;
            for (int r = 0; r < n_u; ++r) {
                double acc = 0.0;
                for (int q2 = 0; q2 < n_u; ++q2) acc += 2.0 * P->Q_u[r * n_u + q2] * ut[q2];
                ub[((size_t)s * N + t) * n_u + r] = acc;
            }
        }
    }
    double *H = (double *)malloc(sizeof(double) * N * n_s * n_s), *h = (double *)malloc(sizeof(double) * N * n_s);
    double *w = (double *)malloc(sizeof(double) * N * n_s), *xbt = (double *)malloc(sizeof(double) * N * n_s);
    for (int k = K - 1; k >= 0; --k) {
        const double *Xk = X + nx * k, *Yk = Y + (size_t)ny * k, *Zk = Zt + (size_t)npair * k, *XIk = XI + (size_t)npair * dim * k;
        const double *Xn = X + nx * (k + 1), *Un = U + nu_ * (k + 1), *Yn = Y + (size_t)ny * (k + 1);
        /* (3) multiplier update adjoint at (s^{k+1}, y^{k+1}) */
        memset(qbar, 0, sizeof(double) * npair * nq);
        for (int b = 0; b < nb; ++b)
            for (int t = 1; t <= N; ++t) {
                const orc_block *q = &B[b];
                double rbv[3];
                for (int r = 0; r < dim; ++r) rbv[r] = xibar[((size_t)b * dim + r) * N + t - 1];
                TR_adjoint(P, q, state_at(P, Xn, q->s, t), Yn + q->yoff + t - 1, N, zbar[(size_t)b * N + t - 1], rbv,
                           yb + q->yoff + t - 1, N, qbar + ((size_t)b * N + t - 1) * nq,
                           grad_d);
            }
        for (int b = 0; b < nb; ++b)
            for (int t = 1; t <= N; ++t)
                for (int a = 0; a < nq; ++a)
                    xb[((size_t)B[b].s * (N + 1) + t) * n_s + qidx[a]] += qbar[((size_t)b * N + t - 1) * nq + a];
        /* zeta^k, xi^k receive the identity part of the update: zbar, xibar unchanged */
        /* (2) trajectory QP adjoint */
        memset(qbar, 0, sizeof(double) * npair * nq);
        bad += traj_adjoint(P, B, nb, Xk, Xn, Yn, Zk, XIk, xb, ub, yb, zbar, xibar, qbar, grad_d, grad_x0);
        /* (1) pair QP adjoint: y^{k+1} <- (s^k, y^k, zeta^k, xi^k) */
        memset(yb_old, 0, sizeof(double) * ny);
        for (int b = 0; b < nb; ++b)
            for (int t = 1; t <= N; ++t) {
                const orc_block *q = &B[b];
                double xr[3], xib[3] = {0, 0, 0};
                for (int r = 0; r < dim; ++r) xr[r] = XIk[((size_t)b * dim + r) * N + t - 1];
                bad += pairqp_adjoint(P, q, state_at(P, Xk, q->s, t), Yk + q->yoff + t - 1, Yn + q->yoff + t - 1, N,
                                      Zk[(size_t)b * N + t - 1], xr, yb + q->yoff + t - 1, yb_old + q->yoff + t - 1, N,
                                      &zbar[(size_t)b * N + t - 1], xib, qbar + ((size_t)b * N + t - 1) * nq, grad_d);
                for (int r = 0; r < dim; ++r) xibar[((size_t)b * dim + r) * N + t - 1] += xib[r];
            }
        memcpy(yb, yb_old, sizeof(double) * ny);
        for (int b = 0; b < nb; ++b)
            for (int t = 1; t <= N; ++t)
                for (int a = 0; a < nq; ++a)
                    xb[((size_t)B[b].s * (N + 1) + t) * n_s + qidx[a]] += qbar[((size_t)b * N + t - 1) * nq + a];
        (void)Un;
    }
    /* s^0 = obstacle-free LQ(x0): H_t = 2 Q_s; the u^0 adjoint is zero */
    for (int s = 0; s < S; ++s) {
        double *hh = (double *)malloc(sizeof(double) * N * n_s);
        lq_stage_base(P, s, H, hh);
        for (int t = 1; t <= N; ++t)
            for (int r = 0; r < n_s; ++r) xbt[(t - 1) * n_s + r] = xb[((size_t)s * (N + 1) + t) * n_s + r];
        bad += lq_adjoint(n_s, n_u, N, dyn_A(P, s), dyn_B(P, s), P->dyn_ts, H, P->Q_u, xbt, NULL, w, grad_x0 + (size_t)s * n_s);
        for (int r = 0; r < n_s; ++r) grad_x0[(size_t)s * n_s + r] += xb[((size_t)s * (N + 1)) * n_s + r];
        free(hh);
    }
    free(H); free(h); free(w); free(xbt);
    free(xb); free(ub); free(yb); free(yb_old); free(zbar); free(xibar); free(qbar);
    free(B);
    return bad;
}

/*
 * Gradient of L = sum_s F_s(x^K, u^K) after exactly K iterations (no early
 * stop) from the initial iterate s^0 = obstacle-free LQ(x0), the given y0,
 * zeta = xi = 0, with respect to every obstacle face offset d (grad_d[F_o])
 * and every initial state (grad_x0[n_scen * n_s]). y0 is held fixed.
 * Reverse mode through the stored iterates, with the dense KKT transposes of
 * each pair QP on its active set and of the condensed trajectory QP.
 * Returns 0, or the number of failed solves.
 */
int orc_admm_grad(const orc_problem *P, int K, const double *y0, double *L_out, double *grad_d, double *grad_x0)
{
    if (P->model) return 1 << 20;   /* the reverse pass covers the given linear models only */
    int S = P->n_scen, N = P->N, n_s = P->n_s, n_u = P->n_u, dim = P->dim;
    int nb = count_blocks(P), bad = 0;
    long ny = orc_y_size(P), npair = (long)nb * N;
    size_t nx = (size_t)S * (N + 1) * n_s, nu_ = (size_t)S * N * n_u;
    orc_block *B = (orc_block *)malloc(sizeof(orc_block) * (nb > 0 ? nb : 1));
    enumerate_blocks(P, B);
    double *X = (double *)malloc(sizeof(double) * nx * (K + 1));
    double *U = (double *)malloc(sizeof(double) * nu_ * (K + 1));
    double *Y = (double *)malloc(sizeof(double) * (ny > 0 ? ny : 1) * (K + 1));
    double *Zt = (double *)calloc((size_t)(npair > 0 ? npair : 1) * (K + 1), sizeof(double));
    double *XI = (double *)calloc((size_t)(npair > 0 ? npair : 1) * dim * (K + 1), sizeof(double));
    double *rp = (double *)calloc(S, sizeof(double));
    /* forward, storing every iterate */
    {
        double *H = (double *)malloc(sizeof(double) * N * n_s * n_s), *h = (double *)malloc(sizeof(double) * N * n_s);
        for (int s = 0; s < S; ++s) {
            lq_stage_base(P, s, H, h);
            bad |= orc_traj_qp(n_s, n_u, N, dyn_A(P, s), dyn_B(P, s), dyn_c(P, s), P->dyn_ts, P->x0 + (size_t)s * n_s, H, h, P->Q_u,
                               X + (size_t)s * (N + 1) * n_s, U + (size_t)s * N * n_u);
        }
        free(H); free(h);
    }
    memcpy(Y, y0, sizeof(double) * ny);
    for (int k = 0; k < K; ++k) {
        double *Xk = X + nx * k, *Yk = Y + (size_t)ny * k, *Zk = Zt + (size_t)npair * k, *XIk = XI + (size_t)npair * dim * k;
        double *Xn = X + nx * (k + 1), *Un = U + nu_ * (k + 1), *Yn = Y + (size_t)ny * (k + 1);
        double *Zn = Zt + (size_t)npair * (k + 1), *XIn = XI + (size_t)npair * dim * (k + 1);
        memcpy(Yn, Yk, sizeof(double) * ny);
        bad += orc_pair_phase(P, Xk, Yk, Zk, XIk, NULL, Yn);
        memcpy(Un, U + nu_ * k, sizeof(double) * nu_);
        bad += orc_traj_phase(P, Xk, Yn, Zk, XIk, NULL, Xn, Un);
        memcpy(Zn, Zk, sizeof(double) * npair);
        memcpy(XIn, XIk, sizeof(double) * npair * dim);
        orc_mult_phase(P, Xn, Yn, NULL, Zn, XIn, rp);
    }
    int bad2 = admm_reverse(P, K, X, U, Y, Zt, XI, L_out, grad_d, grad_x0);
    free(B); free(X); free(U); free(Y); free(Zt); free(XI); free(rp);
    return bad + bad2;
}

/* Test hook: the reverse pass of orc_admm_grad at iterates given by the
 * caller (k = 0..K back to back, canonical layouts), e.g. those of another
 * implementation, so that its reverse pass can be compared apart from the
 * rounding of its forward iterates. */
int orc_admm_grad_at(const orc_problem *P, int K, const double *X, const double *U, const double *Y,
                     const double *Zt, const double *XI, double *L_out, double *grad_d, double *grad_x0)
{
    if (P->model) return 1 << 20;
    return admm_reverse(P, K, X, U, Y, Zt, XI, L_out, grad_d, grad_x0);
}

/* Test hook: VJP of one pair QP in the part frame. Given ybar (n), returns
   the adjoints of dp (no), Cp (no x dim), zeta, xi (dim) and yhat (n) by the
   same active-set KKT transpose as the reverse pass. */
int orc_pairqp_vjp(int dim, int nr, const double *A, const double *b, int no, const double *Cp, const double *dp,
                   double zeta, const double *xi, const double *yhat, double eps, const double *ybar,
                   double *dp_bar, double *Cp_bar, double *zeta_bar, double *xi_bar, double *yhat_bar)
{
    int c = dim + 1, n = nr + no + 1;
    double y[MAXROWS];
    if (orc_pair_qp(dim, nr, A, b, no, Cp, dp, zeta, xi, yhat, eps, y) < 0) return 1;
    double K[MAXROWS * (MAXD + 1)];
    build_K(dim, nr, A, no, Cp, dp, K);
    double bh[MAXD + 1], D[MAXROWS], kap[MAXROWS];
    bh[0] = 1.0 + zeta;
    for (int r = 0; r < dim; ++r) bh[1 + r] = xi[r];
    for (int l = 0; l < n; ++l) {
        double s = 0.0;
        for (int m = 0; m < c; ++m) s += K[l * c + m] * K[l * c + m];
        D[l] = s;
        kap[l] = l < nr ? b[l] : 0.0;
        yhat_bar[l] = 0.0;
    }
    int F[MAXROWS], nf = 0;
    for (int l = 0; l < n; ++l) if (y[l] > 0.0) F[nf++] = l;
    int sz = nf + 1;
    double M[(MAXROWS + 1) * (MAXROWS + 1)], rhs[MAXROWS + 1];
    for (int i2 = 0; i2 < nf; ++i2) {
        for (int j2 = 0; j2 < nf; ++j2) {
            double s = 0.0;
            for (int m = 0; m < c; ++m) s += K[F[i2] * c + m] * K[F[j2] * c + m];
            M[i2 * sz + j2] = s + (i2 == j2 ? eps * D[F[i2]] : 0.0);
        }
        M[i2 * sz + nf] = kap[F[i2]];
        M[nf * sz + i2] = -kap[F[i2]];
        rhs[i2] = ybar[F[i2]];
    }
    M[nf * sz + nf] = 0.0;
    rhs[nf] = 0.0;
    if (gauss_solve(sz, M, rhs)) return 1;
    double gbar[MAXROWS] = {0}, Kbar[MAXROWS * (MAXD + 1)] = {0}, Dbar[MAXROWS] = {0}, bhbar[MAXD + 1] = {0};
    for (int i2 = 0; i2 < nf; ++i2) gbar[F[i2]] = -rhs[i2];
    for (int i2 = 0; i2 < nf; ++i2) {
        int l = F[i2];
        for (int m = 0; m < c; ++m) {
            double yK = 0.0, aK = 0.0;
            for (int j2 = 0; j2 < nf; ++j2) {
                yK += y[F[j2]] * K[F[j2] * c + m];
                aK += rhs[j2] * K[F[j2] * c + m];
            }
            Kbar[l * c + m] += -rhs[i2] * yK - y[l] * aK;
        }
        Dbar[l] += eps * (-rhs[i2] * y[l]);
    }
    for (int l = 0; l < n; ++l) {
        if (gbar[l] == 0.0) continue;
        for (int m = 0; m < c; ++m) {
            Kbar[l * c + m] += gbar[l] * bh[m];
            bhbar[m] += K[l * c + m] * gbar[l];
        }
        Dbar[l] += -eps * gbar[l] * yhat[l];
        yhat_bar[l] += -eps * D[l] * gbar[l];
    }
    for (int l = 0; l < n; ++l)
        for (int m = 0; m < c; ++m) Kbar[l * c + m] += 2.0 * Dbar[l] * K[l * c + m];
    for (int l = 0; l < no; ++l) {
        dp_bar[l] = Kbar[(nr + l) * c];
        for (int r = 0; r < dim; ++r) Cp_bar[l * dim + r] = Kbar[(nr + l) * c + 1 + r];
    }
    *zeta_bar = bhbar[0];
    for (int r = 0; r < dim; ++r) xi_bar[r] = bhbar[1 + r];
    return 0;
}

/* Test hook: VJP of the trajectory phase for cotangents (xbar of x^{k+1},
   ubar of u^{k+1}); writes the adjoints of y^{k+1}, zeta^k, xi^k, x^k (full
   state array), the obstacle offsets and x0. Output arrays are overwritten. */
int orc_traj_vjp(const orc_problem *P, const double *x_in, const double *y, const double *zeta, const double *xi,
                 const double *xbar_in, const double *ubar_in, double *ybar, double *zbar, double *xibar,
                 double *xkbar, double *dbar, double *x0bar)
{
    int S = P->n_scen, N = P->N, n_s = P->n_s, n_u = P->n_u, dim = P->dim, nq = dim + n_att(P);
    int nb = count_blocks(P);
    long ny = orc_y_size(P), npair = (long)nb * N;
    size_t nx = (size_t)S * (N + 1) * n_s, nu_ = (size_t)S * N * n_u;
    orc_block *B = (orc_block *)malloc(sizeof(orc_block) * (nb > 0 ? nb : 1));
    enumerate_blocks(P, B);
    double *xn = (double *)malloc(sizeof(double) * nx), *un = (double *)calloc(nu_, sizeof(double));
    int bad = orc_traj_phase(P, x_in, y, zeta, xi, NULL, xn, un);
    double *xb = (double *)malloc(sizeof(double) * nx), *ub = (double *)malloc(sizeof(double) * nu_);
    memcpy(xb, xbar_in, sizeof(double) * nx);
    memcpy(ub, ubar_in, sizeof(double) * nu_);
    double *qbar = (double *)calloc((size_t)(npair > 0 ? npair : 1) * nq, sizeof(double));
    memset(ybar, 0, sizeof(double) * ny);
    memset(zbar, 0, sizeof(double) * npair);
    memset(xibar, 0, sizeof(double) * npair * dim);
    memset(xkbar, 0, sizeof(double) * nx);
    memset(dbar, 0, sizeof(double) * P->obs_face_ptr[P->obs_ptr[S]]);
    memset(x0bar, 0, sizeof(double) * S * n_s);
    bad += traj_adjoint(P, B, nb, x_in, xn, y, zeta, xi, xb, ub, ybar, zbar, xibar, qbar, dbar, x0bar);
    int qidx[6];
    for (int r = 0; r < dim; ++r) qidx[r] = P->pos_idx[r];
    for (int a = 0; a < n_att(P); ++a) qidx[dim + a] = P->att_idx[a];
    for (int b = 0; b < nb; ++b)
        for (int t = 1; t <= N; ++t)
            for (int a = 0; a < nq; ++a)
                xkbar[((size_t)B[b].s * (N + 1) + t) * n_s + qidx[a]] += qbar[((size_t)b * N + t - 1) * nq + a];
    free(B); free(xn); free(un); free(xb); free(ub); free(qbar);
    return bad;
}
