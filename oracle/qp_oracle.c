/*
 * FP64 CPU oracle for the batched QP layer of OptNet (Amos & Kolter, 2017).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links or calls this
 * file; only the tests, the smoke check and the CPU-baseline leg of the bench
 * do.  It shares no code, header, table or helper with the HIP library.
 *
 * Problem (Section 3, eq. qp2):
 *     minimize_z  1/2 z^T Q z + q^T z   subject to  A z = b,  G z <= h
 * with z in R^n, A in R^{neq x n}, G in R^{nineq x n}.  Q is used through its
 * symmetric part Qs = (Q + Q^T)/2, which leaves the objective unchanged.
 *
 * Forward: the primal-dual interior point method of Section 3.1 (following
 * Mattingley & Boyd's CVXGEN): slack variables s on the inequalities, an affine
 * scaling direction from eq. cvxgen:affine, a centering-plus-corrector
 * direction from eq. cvxgen:cc with the same matrix K, and an update with the
 * sum of the two directions.  Every Newton system is solved on the full,
 * unreduced matrix K exactly as printed under eq. cvxgen:affine (no block
 * elimination, no symmetrization), by dense LU with partial pivoting.
 *
 * Readings where the paper is silent:
 *   - sigma = (mu_aff / mu)^3 (Mehrotra's rule as used by CVXGEN);
 *   - one step length for primal and dual variables: alpha_aff = min(1, a_max)
 *     and alpha = min(1, 0.99 a_max), a_max the largest step keeping s, lambda
 *     non-negative (+inf when no component decreases);
 *   - initial point: solve K with the D(lambda), D(s) block replaced by an
 *     identity pair, i.e. [Qs 0 G^T A^T; 0 I I 0; G I 0 0; A 0 0 0] x =
 *     [-q; 0; h; b]; then s = h - G z, lambda = -s, and each of s, lambda whose
 *     minimum is <= 0 is shifted by (1 - min) so that its minimum becomes 1;
 *   - stop when max(mu, |r_x|_inf, |r_s|_inf, |r_y|_inf) <= tol (mu = s^T
 *     lambda / nineq, the duality measure of Section 3.1), or after max_iter
 *     steps; in replay mode after exactly `replay` steps.
 *
 * Backward: eq. eq-d-def (the transposed KKT-differential matrix at the
 * solution, with the D(G z - h) block as printed) solved by LU, then the
 * gradient formulas of eq. grads.
 *
 * Plain loops, row-major arrays, compiled with -ffp-contract=off.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { OR_OPTIMAL = 0, OR_MAX_ITER = 1, OR_SINGULAR = 2, OR_NONFINITE = 3, OR_EARG = -1, OR_ENOMEM = -2 };

/* In-place LU with partial pivoting of the N x N row-major matrix M, then the
 * solution of M x = rhs (rhs overwritten with x).  Returns 0, or 1 when a zero
 * or non-finite pivot is met. */
static int lu_factor(int N, double *M, int *piv)
{
    for (int k = 0; k < N; ++k) {
        int best = k;
        double bv = fabs(M[(size_t)k * N + k]);
        for (int i = k + 1; i < N; ++i) {
            double v = fabs(M[(size_t)i * N + k]);
            if (v > bv) { bv = v; best = i; }
        }
        if (!(bv > 0.0) || !isfinite(bv)) return 1;
        piv[k] = best;
        if (best != k) {
            for (int j = 0; j < N; ++j) {
                double t = M[(size_t)k * N + j];
                M[(size_t)k * N + j] = M[(size_t)best * N + j];
                M[(size_t)best * N + j] = t;
            }
        }
        double pv = M[(size_t)k * N + k];
        for (int i = k + 1; i < N; ++i) {
            double f = M[(size_t)i * N + k] / pv;
            M[(size_t)i * N + k] = f;
            if (f != 0.0)
                for (int j = k + 1; j < N; ++j) M[(size_t)i * N + j] -= f * M[(size_t)k * N + j];
        }
    }
    return 0;
}

static void lu_solve(int N, const double *M, const int *piv, double *x)
{
    for (int k = 0; k < N; ++k) {
        if (piv[k] != k) { double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t; }
    }
    for (int i = 0; i < N; ++i) {
        double acc = x[i];
        for (int j = 0; j < i; ++j) acc -= M[(size_t)i * N + j] * x[j];
        x[i] = acc;
    }
    for (int i = N - 1; i >= 0; --i) {
        double acc = x[i];
        for (int j = i + 1; j < N; ++j) acc -= M[(size_t)i * N + j] * x[j];
        x[i] = acc / M[(size_t)i * N + i];
    }
}

#define QS(i, j) (0.5 * (Q[(size_t)(i) * n + (j)] + Q[(size_t)(j) * n + (i)]))

/* Assemble K of eq. cvxgen:affine, unknown order (dz, ds, dlambda, dnu):
 *   [ Qs   0      G^T   A^T ]
 *   [ 0    Dlam   Ds    0   ]
 *   [ G    I      0     0   ]
 *   [ A    0      0     0   ]
 * `diag_lam`, `diag_s` are the diagonals of the second block row. */
static void build_K(int n, int m, int p, const double *Q, const double *A, const double *G,
                    const double *diag_lam, const double *diag_s, double *K)
{
    const int N = n + 2 * m + p;
    const int os = n, ol = n + m, on = n + 2 * m;
    memset(K, 0, sizeof(double) * (size_t)N * N);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) K[(size_t)i * N + j] = QS(i, j);
        for (int k = 0; k < m; ++k) K[(size_t)i * N + ol + k] = G[(size_t)k * n + i];
        for (int k = 0; k < p; ++k) K[(size_t)i * N + on + k] = A[(size_t)k * n + i];
    }
    for (int k = 0; k < m; ++k) {
        K[(size_t)(os + k) * N + os + k] = diag_lam[k];
        K[(size_t)(os + k) * N + ol + k] = diag_s[k];
        for (int j = 0; j < n; ++j) K[(size_t)(ol + k) * N + j] = G[(size_t)k * n + j];
        K[(size_t)(ol + k) * N + os + k] = 1.0;
    }
    for (int k = 0; k < p; ++k)
        for (int j = 0; j < n; ++j) K[(size_t)(on + k) * N + j] = A[(size_t)k * n + j];
}

/* Largest a >= 0 with v + a*dv >= 0 componentwise (+inf if no dv_i < 0). */
static double max_step(int m, const double *v, const double *dv)
{
    double a = INFINITY;
    for (int i = 0; i < m; ++i)
        if (dv[i] < 0.0) {
            double t = -v[i] / dv[i];
            if (t < a) a = t;
        }
    return a;
}

/* Residuals of the KKT conditions (Section 3, stationarity and primal
 * feasibility), with the right-hand-side signs of eq. cvxgen:affine:
 *   rx = -(A^T nu + G^T lam + Qs z + q),  rs = -(G z + s - h),  ry = -(A z - b). */
static void residuals(int n, int m, int p, const double *Q, const double *q, const double *A,
                      const double *b, const double *G, const double *h, const double *z,
                      const double *s, const double *lam, const double *nu, double *rx,
                      double *rs, double *ry)
{
    for (int i = 0; i < n; ++i) {
        double acc = q[i];
        for (int j = 0; j < n; ++j) acc += QS(i, j) * z[j];
        for (int k = 0; k < m; ++k) acc += G[(size_t)k * n + i] * lam[k];
        for (int k = 0; k < p; ++k) acc += A[(size_t)k * n + i] * nu[k];
        rx[i] = -acc;
    }
    for (int k = 0; k < m; ++k) {
        double acc = s[k] - h[k];
        for (int j = 0; j < n; ++j) acc += G[(size_t)k * n + j] * z[j];
        rs[k] = -acc;
    }
    for (int k = 0; k < p; ++k) {
        double acc = -b[k];
        for (int j = 0; j < n; ++j) acc += A[(size_t)k * n + j] * z[j];
        ry[k] = -acc;
    }
}

static double inf_norm(int len, const double *v)
{
    double r = 0.0;
    for (int i = 0; i < len; ++i) {
        double a = fabs(v[i]);
        if (a > r || a != a) r = a; /* NaN propagates */
    }
    return r;
}

static int all_finite(size_t len, const double *v)
{
    for (size_t i = 0; i < len; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* Solve one QP.  Inputs row-major: Q[n*n], q[n], A[p*n], b[p], G[m*n], h[m]
 * (A/b and G/h may be NULL when p or m is 0).  Outputs z[n], s[m], lam[m],
 * nu[p], *iters = number of Newton steps taken.  replay < 0: stop on tol or
 * max_iter; replay >= 0: take exactly `replay` steps (status still reports
 * whether the tolerance test holds at the returned iterate).
 * Returns OR_OPTIMAL, OR_MAX_ITER, OR_SINGULAR, OR_NONFINITE or a negative
 * call error. */
int oracle_qp_solve(int n, int m, int p, const double *Q, const double *q, const double *A,
                    const double *b, const double *G, const double *h, int max_iter, double tol,
                    int replay, double *z, double *s, double *lam, double *nu, int *iters)
{
    if (n < 1 || m < 0 || p < 0 || !Q || !q || !z || !iters) return OR_EARG;
    if (m > 0 && (!G || !h || !s || !lam)) return OR_EARG;
    if (p > 0 && (!A || !b || !nu)) return OR_EARG;
    *iters = 0;
    if (!all_finite((size_t)n * n, Q) || !all_finite(n, q) || !all_finite((size_t)m * n, G) ||
        !all_finite(m, h) || !all_finite((size_t)p * n, A) || !all_finite(p, b))
        return OR_NONFINITE;

    const int N = n + 2 * m + p;
    const int os = n, ol = n + m, on = n + 2 * m;
    double *K = (double *)malloc(sizeof(double) * (size_t)N * N);
    double *rhs = (double *)malloc(sizeof(double) * N);
    double *daff = (double *)malloc(sizeof(double) * N);
    double *dcc = (double *)malloc(sizeof(double) * N);
    double *work = (double *)malloc(sizeof(double) * (size_t)(2 * m + n + p + 4));
    int *piv = (int *)malloc(sizeof(int) * N);
    if (!K || !rhs || !daff || !dcc || !work || !piv) {
        free(K); free(rhs); free(daff); free(dcc); free(work); free(piv);
        return OR_ENOMEM;
    }
    double *rx = work, *rs = work + n, *ry = work + n + m, *ones = work + n + m + p;
    int status = OR_MAX_ITER;

    /* Initial point (reading stated in the header): K with identity pair. */
    for (int k = 0; k < m; ++k) ones[k] = 1.0;
    build_K(n, m, p, Q, A, G, ones, ones, K);
    for (int i = 0; i < n; ++i) rhs[i] = -q[i];
    for (int k = 0; k < m; ++k) { rhs[os + k] = 0.0; rhs[ol + k] = h[k]; }
    for (int k = 0; k < p; ++k) rhs[on + k] = b[k];
    if (lu_factor(N, K, piv)) { status = OR_SINGULAR; goto done_zero; }
    lu_solve(N, K, piv, rhs);
    for (int i = 0; i < n; ++i) z[i] = rhs[i];
    for (int k = 0; k < p; ++k) nu[k] = rhs[on + k];
    for (int k = 0; k < m; ++k) {
        double gz = 0.0;
        for (int j = 0; j < n; ++j) gz += G[(size_t)k * n + j] * z[j];
        s[k] = h[k] - gz;
        lam[k] = -s[k];
    }
    if (m > 0) {
        double ms = s[0], ml = lam[0];
        for (int k = 1; k < m; ++k) { if (s[k] < ms) ms = s[k]; if (lam[k] < ml) ml = lam[k]; }
        if (ms <= 0.0) for (int k = 0; k < m; ++k) s[k] += 1.0 - ms;
        if (ml <= 0.0) for (int k = 0; k < m; ++k) lam[k] += 1.0 - ml;
    } else {
        /* Equality-constrained (or unconstrained) QP: the initial system is
         * the KKT system itself, so its solution is optimal. */
        status = all_finite(n, z) && all_finite(p, nu) ? OR_OPTIMAL : OR_NONFINITE;
        goto done;
    }

    for (int it = 0;; ++it) {
        residuals(n, m, p, Q, q, A, b, G, h, z, s, lam, nu, rx, rs, ry);
        double mu = 0.0;
        for (int k = 0; k < m; ++k) mu += s[k] * lam[k];
        mu /= (double)m;
        double err = mu;
        double t;
        t = inf_norm(n, rx); if (t > err || t != t) err = t;
        t = inf_norm(m, rs); if (t > err || t != t) err = t;
        t = inf_norm(p, ry); if (t > err || t != t) err = t;
        if (!isfinite(err)) { status = OR_NONFINITE; *iters = it; break; }
        int converged = err <= tol;
        if (replay >= 0 ? it >= replay : (converged || it >= max_iter)) {
            status = converged ? OR_OPTIMAL : OR_MAX_ITER;
            *iters = it;
            break;
        }

        /* Affine scaling direction, eq. cvxgen:affine. */
        build_K(n, m, p, Q, A, G, lam, s, K);
        if (lu_factor(N, K, piv)) { status = OR_SINGULAR; *iters = it; break; }
        for (int i = 0; i < n; ++i) daff[i] = rx[i];
        for (int k = 0; k < m; ++k) { daff[os + k] = -s[k] * lam[k]; daff[ol + k] = rs[k]; }
        for (int k = 0; k < p; ++k) daff[on + k] = ry[k];
        lu_solve(N, K, piv, daff);

        /* Step to the boundary along the affine direction, mu_aff, sigma. */
        double a_s = max_step(m, s, daff + os), a_l = max_step(m, lam, daff + ol);
        double a_aff = a_s < a_l ? a_s : a_l;
        if (a_aff > 1.0) a_aff = 1.0;
        double mu_aff = 0.0;
        for (int k = 0; k < m; ++k)
            mu_aff += (s[k] + a_aff * daff[os + k]) * (lam[k] + a_aff * daff[ol + k]);
        mu_aff /= (double)m;
        double ratio = mu_aff / mu;
        double sigma = ratio * ratio * ratio;

        /* Centering-plus-corrector direction, eq. cvxgen:cc (same K). */
        for (int i = 0; i < n; ++i) dcc[i] = 0.0;
        for (int k = 0; k < m; ++k) {
            dcc[os + k] = sigma * mu - daff[os + k] * daff[ol + k];
            dcc[ol + k] = 0.0;
        }
        for (int k = 0; k < p; ++k) dcc[on + k] = 0.0;
        lu_solve(N, K, piv, dcc);

        /* Combined direction and step. */
        for (int i = 0; i < N; ++i) daff[i] += dcc[i];
        a_s = max_step(m, s, daff + os);
        a_l = max_step(m, lam, daff + ol);
        double a = a_s < a_l ? a_s : a_l;
        a = 0.99 * a;
        if (a > 1.0) a = 1.0;
        for (int i = 0; i < n; ++i) z[i] += a * daff[i];
        for (int k = 0; k < m; ++k) { s[k] += a * daff[os + k]; lam[k] += a * daff[ol + k]; }
        for (int k = 0; k < p; ++k) nu[k] += a * daff[on + k];
    }
    goto done;

done_zero:
    for (int i = 0; i < n; ++i) z[i] = 0.0;
    for (int k = 0; k < m; ++k) { s[k] = 0.0; lam[k] = 0.0; }
    for (int k = 0; k < p; ++k) nu[k] = 0.0;
done:
    free(K); free(rhs); free(daff); free(dcc); free(work); free(piv);
    return status;
}

/* Backward pass (Section 3, eq. eq-d-def and eq. grads).  Given the solution
 * (z, lam, nu) and g = dl/dz, solve
 *   [ Qs  G^T D(lam)  A^T ] [d_z  ]     [ g ]
 *   [ G   D(G z - h)  0   ] [d_lam] = - [ 0 ]
 *   [ A   0           0   ] [d_nu ]     [ 0 ]
 * and write
 *   dQ = 1/2 (d_z z^T + z d_z^T),  dq = d_z,
 *   dA = d_nu z^T + nu d_z^T,      db = -d_nu,
 *   dG = D(lam) d_lam z^T + lam d_z^T,  dh = -D(lam) d_lam.
 * Any output pointer may be NULL.  Returns 0, or OR_SINGULAR. */
int oracle_qp_backward(int n, int m, int p, const double *Q, const double *A, const double *G,
                       const double *h, const double *z, const double *lam, const double *nu,
                       const double *g, double *dQ, double *dq, double *dA, double *db,
                       double *dG, double *dh, double *d_out)
{
    if (n < 1 || m < 0 || p < 0 || !Q || !z || !g) return OR_EARG;
    const int N = n + m + p;
    const int ol = n, on = n + m;
    double *M = (double *)calloc((size_t)N * N, sizeof(double));
    double *d = (double *)malloc(sizeof(double) * N);
    int *piv = (int *)malloc(sizeof(int) * N);
    if (!M || !d || !piv) { free(M); free(d); free(piv); return OR_ENOMEM; }
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) M[(size_t)i * N + j] = QS(i, j);
        for (int k = 0; k < m; ++k) M[(size_t)i * N + ol + k] = G[(size_t)k * n + i] * lam[k];
        for (int k = 0; k < p; ++k) M[(size_t)i * N + on + k] = A[(size_t)k * n + i];
    }
    for (int k = 0; k < m; ++k) {
        double gz = 0.0;
        for (int j = 0; j < n; ++j) {
            M[(size_t)(ol + k) * N + j] = G[(size_t)k * n + j];
            gz += G[(size_t)k * n + j] * z[j];
        }
        M[(size_t)(ol + k) * N + ol + k] = gz - h[k];
    }
    for (int k = 0; k < p; ++k)
        for (int j = 0; j < n; ++j) M[(size_t)(on + k) * N + j] = A[(size_t)k * n + j];
    for (int i = 0; i < N; ++i) d[i] = i < n ? -g[i] : 0.0;
    int rc = 0;
    if (lu_factor(N, M, piv)) { rc = OR_SINGULAR; goto out; }
    lu_solve(N, M, piv, d);
    {
        const double *dz = d, *dl = d + ol, *dn = d + on;
        if (dQ)
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j)
                    dQ[(size_t)i * n + j] = 0.5 * (dz[i] * z[j] + z[i] * dz[j]);
        if (dq) for (int i = 0; i < n; ++i) dq[i] = dz[i];
        if (dA)
            for (int k = 0; k < p; ++k)
                for (int j = 0; j < n; ++j) dA[(size_t)k * n + j] = dn[k] * z[j] + nu[k] * dz[j];
        if (db) for (int k = 0; k < p; ++k) db[k] = -dn[k];
        if (dG)
            for (int k = 0; k < m; ++k)
                for (int j = 0; j < n; ++j)
                    dG[(size_t)k * n + j] = lam[k] * dl[k] * z[j] + lam[k] * dz[j];
        if (dh) for (int k = 0; k < m; ++k) dh[k] = -lam[k] * dl[k];
        if (d_out) memcpy(d_out, d, sizeof(double) * N);
    }
out:
    free(M); free(d); free(piv);
    return rc;
}
