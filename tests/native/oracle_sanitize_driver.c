/* Test driver (no method arithmetic): runs the oracle's two entry points on a
 * few seeded problems and its edge cases, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py.  Exits 0 when
 * every call returns the expected status; the sanitizers abort on any error. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_qp_solve(int n, int m, int p, const double *Q, const double *q, const double *A,
                    const double *b, const double *G, const double *h, int max_iter, double tol,
                    int replay, double *z, double *s, double *lam, double *nu, int *iters);
int oracle_qp_backward(int n, int m, int p, const double *Q, const double *A, const double *G,
                       const double *h, const double *z, const double *lam, const double *nu,
                       const double *g, double *dQ, double *dq, double *dA, double *db,
                       double *dG, double *dh, double *d_out);

static unsigned long long st = 88172645463325252ull;
static double urand(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return (double)(st >> 11) / 9007199254740992.0; }
static double nrand(void) { double u = urand() + 1e-300, v = urand(); return sqrt(-2.0 * log(u)) * cos(6.283185307179586 * v); }

static int one(int n, int m, int p, int replay, int poison) {
    double *Q = malloc(sizeof(double) * n * n), *L = malloc(sizeof(double) * n * n);
    double *q = malloc(sizeof(double) * n), *z0 = malloc(sizeof(double) * n), *g = malloc(sizeof(double) * n);
    double *A = p ? malloc(sizeof(double) * p * n) : NULL, *b = p ? malloc(sizeof(double) * p) : NULL;
    double *G = m ? malloc(sizeof(double) * m * n) : NULL, *h = m ? malloc(sizeof(double) * m) : NULL;
    double *z = malloc(sizeof(double) * n), *s = m ? malloc(sizeof(double) * m) : NULL;
    double *lam = m ? malloc(sizeof(double) * m) : NULL, *nu = p ? malloc(sizeof(double) * p) : NULL;
    for (int i = 0; i < n * n; ++i) L[i] = nrand();
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double a = 0;
            for (int k = 0; k < n; ++k) a += L[i * n + k] * L[j * n + k];
            Q[i * n + j] = a / n + (i == j ? 1e-3 : 0.0);
        }
    for (int i = 0; i < n; ++i) { q[i] = nrand(); z0[i] = nrand(); g[i] = nrand(); }
    for (int k = 0; k < p; ++k) {
        double a = 0;
        for (int j = 0; j < n; ++j) { A[k * n + j] = nrand(); a += A[k * n + j] * z0[j]; }
        b[k] = a;
    }
    for (int k = 0; k < m; ++k) {
        double a = 0;
        for (int j = 0; j < n; ++j) { G[k * n + j] = nrand(); a += G[k * n + j] * z0[j]; }
        h[k] = a + urand();
    }
    if (poison) q[0] = NAN;
    int it = 0;
    int rc = oracle_qp_solve(n, m, p, Q, q, A, b, G, h, 30, 1e-8, replay, z, s, lam, nu, &it);
    int ok = poison ? rc == 3 : (rc == 0 || rc == 1);
    if (!poison) {
        double *dQ = malloc(sizeof(double) * n * n), *dq = malloc(sizeof(double) * n);
        double *dA = p ? malloc(sizeof(double) * p * n) : NULL, *db = p ? malloc(sizeof(double) * p) : NULL;
        double *dG = m ? malloc(sizeof(double) * m * n) : NULL, *dh = m ? malloc(sizeof(double) * m) : NULL;
        double *d = malloc(sizeof(double) * (n + m + p));
        int rb = oracle_qp_backward(n, m, p, Q, A, G, h, z, lam, nu, g, dQ, dq, dA, db, dG, dh, d);
        ok = ok && rb == 0;
        for (int i = 0; i < n; ++i) ok = ok && isfinite(dq[i]);
        free(dQ); free(dq); free(dA); free(db); free(dG); free(dh); free(d);
    }
    printf("n=%d m=%d p=%d replay=%d poison=%d: status %d iters %d %s\n", n, m, p, replay, poison, rc, it,
           ok ? "ok" : "FAILED");
    free(Q); free(L); free(q); free(z0); free(g); free(A); free(b); free(G); free(h);
    free(z); free(s); free(lam); free(nu);
    return ok;
}

int main(void) {
    int ok = 1;
    ok &= one(10, 20, 5, -1, 0);
    ok &= one(1, 2, 0, -1, 0);
    ok &= one(6, 0, 0, -1, 0);
    ok &= one(5, 0, 2, -1, 0);
    ok &= one(17, 33, 3, 3, 0);
    ok &= one(30, 45, 0, -1, 0);
    ok &= one(8, 12, 2, -1, 1);
    return ok ? 0 : 1;
}
