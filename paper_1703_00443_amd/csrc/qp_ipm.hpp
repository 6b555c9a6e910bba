// The primal-dual interior point method of Section 3.1, written once over a
// factorization policy F that owns the reduced KKT factor (and where G lives).
//
// Per iterate (order chosen so that the factor kept for the backward pass is
// the one of the returned iterate):
//   residuals r_x, r_s, r_y and mu = s^T lambda / nineq        (KKT conditions)
//   D = lambda / s, factor [Qs + G^T D G, A^T; A, 0]           (symmetrised K)
//   stop test
//   affine direction (eq. cvxgen:affine), step to the boundary, mu_aff,
//   sigma = (mu_aff / mu)^3, centering-plus-corrector direction
//   (eq. cvxgen:cc) with the same factor, combined step with 0.99 of the
//   step to the boundary (capped at 1), update of (z, s, lambda, nu).
//
// Policy interface (all calls made by every thread of the workgroup; each
// call ends with a barrier when its outputs are read by other threads):
//   bool factor(const T *D)                    form and factor at scaling D
//   void solve(f, r4, dz, dnu)                 [H A^T; A 0][dz; dnu] = [f; r4]
//   void gt_mv(v, out)   out = G^T v           void g_mv(x, out)   out = G x
//   void qs_mv(z, out)   out = Qs z
//   static constexpr bool kRefineAlways        refine every combined direction
//   static constexpr bool kSolveGz             solve_g(f, r4, dz, dnu, gz) also
//                                              returns G dz (see solve_gz)
//   static constexpr bool kFormResidual        factor_res(D, z, lam, s, h, gz,
//                                              gtl, gtw, wsc) factors as factor(D)
//                                              and returns G z, G^T lam and the
//                                              affine step's G^T (lam + D r_s)
//                                              from the rows of G the formation
//                                              of H reads (wsc: m entries of
//                                              scratch)
//   bool finish(D)                             write the factor of [H A^T; A 0]
//                                              at D to the state (false: none)
#pragma once
#include "qp_core.hpp"

namespace qpmi {

template <typename T>
struct Prob {
    int n, m, p;
    const T *Q, *q, *A, *b, *G, *h;
    T *z, *lam, *nu, *s;
    char *state;
    int out;        // index into status / iters
    int variant;    // requested variant (QP_VARIANT_*)
    int lds_limit;  // device LDS per workgroup (the streamed policy sizes its chunks by it)
    unsigned flags; // QP_FLAG_* of the call
};

template <typename T>
__device__ __forceinline__ Prob<T> fwd_problem(const FwdLaunch &L, int idx) {
    Prob<T> P;
    P.lds_limit = L.lds_limit;
    P.flags = L.flags;
    if (L.desc == nullptr) {
        const int j = idx;
        P.n = L.nz; P.m = L.nineq; P.p = L.neq;
        P.Q = (const T *)L.Q + (size_t)j * L.sQ;
        P.q = (const T *)L.q + (size_t)j * L.sq;
        P.A = (const T *)L.A + (size_t)j * L.sA;
        P.b = (const T *)L.b + (size_t)j * L.sb;
        P.G = (const T *)L.G + (size_t)j * L.sG;
        P.h = (const T *)L.h + (size_t)j * L.sh;
        P.z = (T *)L.z + (size_t)j * P.n;
        P.lam = (T *)L.lam + (size_t)j * P.m;
        P.s = (T *)L.s + (size_t)j * P.m;
        P.nu = (T *)L.nu + (size_t)j * P.p;
        P.state = L.state + (size_t)j * L.state_stride;
        P.out = j;
        P.variant = L.variant;
    } else {
        const int j = L.order ? L.order[idx] : idx;
        const qp_problem_desc d = L.desc[j];
        const T *base = (const T *)L.base_in;
        P.n = d.nz; P.m = d.nineq; P.p = d.neq;
        P.Q = base + d.Q; P.q = base + d.q; P.A = base + d.A;
        P.b = base + d.b; P.G = base + d.G; P.h = base + d.h;
        P.z = (T *)L.z + d.z; P.lam = (T *)L.lam + d.lam; P.s = (T *)L.s + d.lam;
        P.nu = (T *)L.nu + d.nu;
        P.state = L.state + d.state;
        P.out = j;
        P.variant = d.variant ? d.variant : L.variant;
    }
    return P;
}

// LDS vector layout of the interior point driver, in elements of T.  The
// policy's own LDS region starts at `end`.
// The iteration's vectors in LDS.  The combined step of the slacks and duals
// reuses w and tm (each entry is read there just before it is overwritten), and
// the last iterate with a good factor is kept in the problem's own output
// buffers, idle until the end; both keep LDS for the factorization policies.
struct IpmLayout {
    int z, rx, f, y, dza, dzc, tn, tn2;  // n-vectors
    int s, lam, rz, D, dsa, dla, w, tm;  // m-vectors
    int nu, ry, dna, dnc, tp, tp2;       // p-vectors
    int red;                             // 64 reduction slots
    int end;
    __host__ __device__ IpmLayout(int n, int m, int p) {
        const int N = pad4(n), M = pad4(m), Pp = pad4(p);
        int o = 0;
        z = o; o += N; rx = o; o += N; f = o; o += N; y = o; o += N; dza = o; o += N;
        dzc = o; o += N; tn = o; o += N; tn2 = o; o += N;
        s = o; o += M; lam = o; o += M; rz = o; o += M; D = o; o += M; dsa = o; o += M;
        dla = o; o += M; w = o; o += M; tm = o; o += M;
        nu = o; o += Pp; ry = o; o += Pp; dna = o; o += Pp; dnc = o; o += Pp; tp = o; o += Pp;
        tp2 = o; o += Pp;
        red = o; o += 64;
        end = (o + 15) & ~15;
    }
};

// dz (and dnu) of the reduced system, and in gz the product G dz that
// recovers ds = r_s - G dz and dlam = c + D G dz.  A policy whose solve yields
// w = D G dz itself (F::kSolveGz) returns gz = D^{-1} w: dlam then carries w's
// own rounding instead of dz's multiplied by D.
template <typename T, class F>
__device__ __forceinline__ void solve_gz(F &fac, const T *f, const T *r4, T *dz, T *dnu, T *gz) {
    if constexpr (F::kSolveGz) {
        fac.solve_g(f, r4, dz, dnu, gz);
    } else {
        fac.solve(f, r4, dz, dnu);
        fac.g_mv(dz, gz);
    }
}

template <typename T, int NT, class F>
__device__ __forceinline__ void ipm_solve(const Prob<T> &P, T *sm, const IpmLayout &Lo, F &fac, int max_iter, T tol,
                          int32_t *status, int32_t *iters) {
    const int n = P.n, m = P.m, p = P.p;
    const int tid = threadIdx.x;
    T *z = sm + Lo.z, *rx = sm + Lo.rx, *f = sm + Lo.f, *y = sm + Lo.y, *dza = sm + Lo.dza,
      *dzc = sm + Lo.dzc, *tn = sm + Lo.tn, *tn2 = sm + Lo.tn2;
    T *s = sm + Lo.s, *lam = sm + Lo.lam, *rz = sm + Lo.rz, *D = sm + Lo.D, *dsa = sm + Lo.dsa,
      *dla = sm + Lo.dla, *w = sm + Lo.w, *tm = sm + Lo.tm;
    T *dsc = tm, *dlc = w;  // combined step, written over the entries just read
    T *nu = sm + Lo.nu, *ry = sm + Lo.ry, *dna = sm + Lo.dna, *dnc = sm + Lo.dnc,
      *tp = sm + Lo.tp, *tp2 = sm + Lo.tp2;
    T *red = sm + Lo.red;
    const T *__restrict__ A = P.A;
    // the problem's pointers as plain locals (keeps the descriptor out of
    // scratch memory in the larger policy instantiations)
    const T *__restrict__ Pq = P.q, *__restrict__ Ph = P.h, *__restrict__ Pb = P.b;
    const T *__restrict__ PQ = P.Q, *__restrict__ PG = P.G;
    T *Pz = P.z, *Ps = P.s, *Plam = P.lam, *Pnu = P.nu;
    const int Pout = P.out;
    // last iterate with a good factor: the output buffers, each entry written
    // and read back by the same thread
    T *zp = Pz, *sp = Ps, *lp = Plam, *nup = Pnu;

    // Input finiteness (one pass over every input).
    bool fin = true;
    for (int e = tid; e < n * n; e += NT) fin &= isfinite(PQ[e]);
    for (int e = tid; e < m * n; e += NT) fin &= isfinite(PG[e]);
    for (int e = tid; e < p * n; e += NT) fin &= isfinite(A[e]);
    for (int e = tid; e < n; e += NT) fin &= isfinite(Pq[e]);
    for (int e = tid; e < m; e += NT) fin &= isfinite(Ph[e]);
    for (int e = tid; e < p; e += NT) fin &= isfinite(Pb[e]);
    {
        T bad = fin ? T(0) : T(1), d0 = 0, d1 = 0;
        block_reduce3<T, NT>(bad, d0, d1, red);
        fin = bad == T(0);
    }
    int st = QP_STATUS_MAX_ITER, it = 0;
    bool stalled = false;  // re-running the previous iterate after a breakdown
    constexpr T kEps = sizeof(T) == 8 ? T(2.220446049250313e-16) : T(1.1920929e-7);
    T gnorm = 0;
    if (!fin) {
        st = QP_STATUS_NONFINITE;
        for (int e = tid; e < n; e += NT) z[e] = 0;
        for (int e = tid; e < m; e += NT) { s[e] = 0; lam[e] = 0; D[e] = 0; }
        for (int e = tid; e < p; e += NT) nu[e] = 0;
        __syncthreads();
        goto finish;
    }
    fac.prepare();

    // Row 1-norms of G (state scratch) and the largest column 1-norm: they bound
    // how much the rounding of G dz, multiplied by D = lambda / s when the
    // multiplier step is recovered, can leave in the first Newton row (below).
    // The product of the largest row and column 1-norms of G: with eps |dz|
    // max D it bounds what the rounding of G dz, multiplied by D = lambda / s
    // when the multiplier step is recovered, can leave in the first Newton row.
    // (The iteration's vectors are idle until the initial point: their space
    // holds the partial column sums.)
    gnorm = max_row_abs_sum<T, NT>(PG, n, m, n, red) * max_col_abs_sum<T, NT>(PG, n, m, n, sm, Lo.red, red);
    // ---- initial point: K with the (D(lambda), D(s)) pair replaced by (I, I)
    for (int e = tid; e < m; e += NT) D[e] = T(1);
    __syncthreads();
    {
        const bool ok = fac.factor(D);
        if (!ok) {
            st = QP_STATUS_BREAKDOWN;
            for (int e = tid; e < n; e += NT) z[e] = 0;
            for (int e = tid; e < m; e += NT) { s[e] = 0; lam[e] = 0; }
            for (int e = tid; e < p; e += NT) nu[e] = 0;
            __syncthreads();
            goto finish;
        }
        // f = -q + G^T h  (r1 = -q, r2 = 0, r3 = h, r4 = b)
        fac.gt_mv(Ph, f);
        for (int i = tid; i < n; i += NT) f[i] -= Pq[i];
        for (int k = tid; k < p; k += NT) tp2[k] = Pb[k];
        __syncthreads();
        if (m > 0) {
            solve_gz<T>(fac, f, tp2, z, nu, tm);
            T mns = pinf<T>(), mnl = pinf<T>(), dummy = 0;
            for (int k = tid; k < m; k += NT) {
                const T sk = Ph[k] - tm[k];
                s[k] = sk;
                lam[k] = -sk;
                mns = fmin(mns, sk);
                mnl = fmin(mnl, -sk);
            }
            T mx = -pinf<T>();
            block_reduce3<T, NT>(dummy, mx, mns, red);
            dummy = 0; mx = -pinf<T>();
            block_reduce3<T, NT>(dummy, mx, mnl, red);
            for (int k = tid; k < m; k += NT) {
                if (mns <= T(0)) s[k] += T(1) - mns;
                if (mnl <= T(0)) lam[k] += T(1) - mnl;
            }
            __syncthreads();
        } else {
            fac.solve(f, tp2, z, nu);
            st = QP_STATUS_OPTIMAL;
            goto store_factor;
        }
    }

    // ---- Newton loop
    for (it = 0;; ++it) {
        // residuals: rx = -(Qs z + q + G^T lam + A^T nu), rz = -(G z + s - h), ry = -(A z - b).
        // Where G is streamed (F::kFormResidual), H is formed and factored
        // first, at D = lam / s, and G z, G^T lam and the affine right-hand
        // side's G^T (lam + D rz) (into f; rz serves as scratch until it is
        // set below) come from the same reads of G; the stop test and the
        // status logic below are unchanged.
        bool ok_res = true;
        if constexpr (F::kFormResidual) {
            for (int k = tid; k < m; k += NT) D[k] = lam[k] / s[k];
            __syncthreads();
            ok_res = fac.factor_res(D, z, lam, s, Ph, tm, rx, f, rz);
        } else {
            fac.g_mv(z, tm);
            fac.gt_mv(lam, rx);
        }
        fac.qs_mv(z, tn);
        if (p > 0) {
            mv_rows<T, NT>(A, n, p, n, z, ry);  // A z
            mv_cols<T, NT>(A, n, p, n, nu, tn2);  // A^T nu
            __syncthreads();
        }
        T vsum = 0, vmax = 0, vmin = pinf<T>(), emax = 0;
        for (int i = tid; i < n; i += NT) {
            T acc = tn[i] + Pq[i] + rx[i];
            if (p > 0) acc += tn2[i];
            rx[i] = -acc;
            vmax = fmax(vmax, fabs(acc));
            vmin = fmin(vmin, isfinite(acc) ? T(1) : T(0));
        }
        for (int k = tid; k < m; k += NT) {
            const T r = -(tm[k] + s[k] - Ph[k]);
            rz[k] = r;
            vmax = fmax(vmax, fabs(r));
            vmin = fmin(vmin, isfinite(r) ? T(1) : T(0));
            vsum += s[k] * lam[k];
            const T dk = lam[k] / s[k];
            D[k] = dk;
            emax = fmax(emax, dk);
        }
        for (int k = tid; k < p; k += NT) {
            const T r = -(ry[k] - Pb[k]);
            ry[k] = r;
            vmax = fmax(vmax, fabs(r));
            vmin = fmin(vmin, isfinite(r) ? T(1) : T(0));
        }
        block_reduce4<T, NT>(vsum, vmax, emax, vmin, red);
        const T mu = vsum / T(m);
        const T err = fmax(mu, vmax);
        const bool finite_now = vmin > T(0) && isfinite(mu);

        // factor at this iterate
        bool ok;
        if constexpr (F::kFormResidual) ok = finite_now && ok_res;
        else ok = finite_now && fac.factor(D);

        if (!finite_now) { st = QP_STATUS_NONFINITE; break; }
        if (stalled) { st = ok ? QP_STATUS_STALLED : QP_STATUS_BREAKDOWN; break; }
        if (!ok) {
            if (it == 0) { st = QP_STATUS_BREAKDOWN; break; }
            // working precision exhausted: go back to the previous iterate,
            // whose factorization succeeded, and return it with that factor
            // (recomputed by the same code, so identical); one factor call site
            for (int i = tid; i < n; i += NT) z[i] = zp[i];
            for (int k = tid; k < m; k += NT) { s[k] = sp[k]; lam[k] = lp[k]; }
            for (int k = tid; k < p; k += NT) nu[k] = nup[k];
            __syncthreads();
            stalled = true;
            it -= 2;
            continue;
        }
        if (err <= tol) { st = QP_STATUS_OPTIMAL; break; }
        if (it >= max_iter) { st = QP_STATUS_MAX_ITER; break; }
        for (int i = tid; i < n; i += NT) zp[i] = z[i];
        for (int k = tid; k < m; k += NT) { sp[k] = s[k]; lp[k] = lam[k]; }
        for (int k = tid; k < p; k += NT) nup[k] = nu[k];

        // ---- affine direction: f = rx + G^T (lam + D rz), r4 = ry
        if constexpr (!F::kFormResidual) {
            for (int k = tid; k < m; k += NT) tm[k] = lam[k] + D[k] * rz[k];
            __syncthreads();
            fac.gt_mv(tm, f);
        }
        for (int i = tid; i < n; i += NT) f[i] += rx[i];
        __syncthreads();
        solve_gz<T>(fac, f, ry, dza, dna, tm);
        T amin = pinf<T>(), d0 = 0, d1 = 0;
        for (int k = tid; k < m; k += NT) {
            const T ds = rz[k] - tm[k];
            const T dl = -lam[k] - D[k] * ds;
            dsa[k] = ds;
            dla[k] = dl;
            if (ds < T(0)) amin = fmin(amin, -s[k] / ds);
            if (dl < T(0)) amin = fmin(amin, -lam[k] / dl);
        }
        block_reduce3<T, NT>(d0, d1, amin, red);
        const T a_aff = fmin(T(1), amin);
        T msum = 0;
        for (int k = tid; k < m; k += NT) msum += (s[k] + a_aff * dsa[k]) * (lam[k] + a_aff * dla[k]);
        msum = block_sum<T, NT>(msum, red);
        const T mu_aff = msum / T(m);
        const T ratio = mu_aff / mu;
        const T sigma = ratio * ratio * ratio;

        // ---- centering-plus-corrector: w = (sigma mu - dsa dla) / s, f = -G^T w, r4 = 0
        for (int k = tid; k < m; k += NT) w[k] = (sigma * mu - dsa[k] * dla[k]) / s[k];
        for (int k = tid; k < p; k += NT) tp[k] = T(0);
        __syncthreads();
        fac.gt_mv(w, f);
        for (int i = tid; i < n; i += NT) f[i] = -f[i];
        __syncthreads();
        solve_gz<T>(fac, f, tp, dzc, dnc, tm);
        // combined direction (dz in dza, dnu in dna, ds in tm, dlam in w)
        amin = pinf<T>(); d0 = 0;
        T dzmax = 0;
        for (int k = tid; k < m; k += NT) {
            const T dsc_k = -tm[k];
            const T dlc_k = w[k] - D[k] * dsc_k;
            const T ds = dsa[k] + dsc_k;
            const T dl = dla[k] + dlc_k;
            dsc[k] = ds;
            dlc[k] = dl;
            if (ds < T(0)) amin = fmin(amin, -s[k] / ds);
            if (dl < T(0)) amin = fmin(amin, -lam[k] / dl);
        }
        for (int i = tid; i < n; i += NT) {
            const T dz = dza[i] + dzc[i];
            dza[i] = dz;
            dzmax = fmax(dzmax, fabs(dz));
        }
        for (int k = tid; k < p; k += NT) dna[k] += dnc[k];
        block_reduce3<T, NT>(d0, dzmax, amin, red);

        // One step of iterative refinement of the combined direction on the
        // residual of the unreduced Newton system, with the same factor, when
        // the error that recovering dlam = c + D G dz can leave in the first row
        // may reach a quarter of the tolerance (large D near the end of the
        // solve).  The bound eps |dz| max_k D_k max_k |G_k|_1 max_j |G^T e_j|_1
        // overestimated the error seen in the dual residual by about 10x, hence
        // the test against 2.5 tol.  Without it the dual residual can grow from
        // one iterate to the next there instead of shrinking with the step.
        // Early steps, whose residuals are far above that error, skip it: it
        // runs only when the bound is also at least a tenth of the current
        // error max(mu, residuals) (the error itself then at least about 1% of
        // it), which is where the next residual can be made of it.
        // Policies whose solve leaves an error that does not scale with |dz|
        // (F::kRefineAlways) refine every step.
        const T rbound = kEps * dzmax * emax * gnorm;
        if (F::kRefineAlways || (rbound >= T(2.5) * tol && rbound >= T(0.1) * err)) {
            // e2 = (sigma mu - s lam - dsa dla) - (lam ds + s dl)        -> dla
            for (int k = tid; k < m; k += NT)
                dla[k] = (sigma * mu - s[k] * lam[k] - dsa[k] * dla[k]) - (lam[k] * dsc[k] + s[k] * dlc[k]);
            __syncthreads();
            fac.g_mv(dza, dsa);    // G dz
            fac.qs_mv(dza, tn);    // Qs dz
            fac.gt_mv(dlc, tn2);   // G^T dlam
            if (p > 0) {
                mv_cols<T, NT>(A, n, p, n, dna, y);  // A^T dnu
                mv_rows<T, NT>(A, n, p, n, dza, tp);  // A dz
                __syncthreads();
            }
            // e3 = rz - (G dz + ds) -> dsa;  c = (e2 - lam e3) / s -> dla
            for (int k = tid; k < m; k += NT) {
                const T e3 = rz[k] - (dsa[k] + dsc[k]);
                dsa[k] = e3;
                dla[k] = (dla[k] - lam[k] * e3) / s[k];
            }
            // e1 = rx - (Qs dz + G^T dlam + A^T dnu) -> f;  e4 = ry - A dz -> tp2
            for (int i = tid; i < n; i += NT) {
                T acc = tn[i] + tn2[i];
                if (p > 0) acc += y[i];
                f[i] = rx[i] - acc;
            }
            for (int k = tid; k < p; k += NT) tp2[k] = ry[k] - tp[k];
            __syncthreads();
            fac.gt_mv(dla, tn);    // G^T c
            for (int i = tid; i < n; i += NT) f[i] -= tn[i];
            __syncthreads();
            solve_gz<T>(fac, f, tp2, dzc, dnc, rz);  // G ddz (r_s is not read again in this step)
            amin = pinf<T>(); d0 = 0; d1 = 0;
            for (int k = tid; k < m; k += NT) {
                const T ds = dsc[k] + (dsa[k] - rz[k]);          // + e3 - G ddz
                const T dl = dlc[k] + (dla[k] + D[k] * rz[k]);   // + c + D G ddz
                dsc[k] = ds;
                dlc[k] = dl;
                if (ds < T(0)) amin = fmin(amin, -s[k] / ds);
                if (dl < T(0)) amin = fmin(amin, -lam[k] / dl);
            }
            for (int i = tid; i < n; i += NT) dza[i] += dzc[i];
            for (int k = tid; k < p; k += NT) dna[k] += dnc[k];
            block_reduce3<T, NT>(d0, d1, amin, red);
        }
        const T alpha = fmin(T(1), T(0.99) * amin);
        for (int i = tid; i < n; i += NT) z[i] += alpha * dza[i];
        for (int k = tid; k < m; k += NT) { s[k] += alpha * dsc[k]; lam[k] += alpha * dlc[k]; }
        for (int k = tid; k < p; k += NT) nu[k] += alpha * dna[k];
        __syncthreads();
    }

store_factor:
    if (!fac.finish(D)) {
        // Only a policy whose Newton steps factor another matrix than H (the
        // elimination order) can get here: H itself lost positive
        // definiteness at the returned iterate.  As when the next iterate's
        // factorization fails inside the loop, the previous iterate (kept in
        // the output buffers since its step) is returned with its factor.
        if (it >= 1 && (st == QP_STATUS_OPTIMAL || st == QP_STATUS_MAX_ITER)) {
            for (int i = tid; i < n; i += NT) z[i] = zp[i];
            for (int k = tid; k < m; k += NT) {
                s[k] = sp[k];
                lam[k] = lp[k];
                D[k] = lp[k] / sp[k];
            }
            for (int k = tid; k < p; k += NT) nu[k] = nup[k];
            __syncthreads();
            st = QP_STATUS_STALLED;
            it -= 1;
            if (!fac.finish(D)) st = QP_STATUS_BREAKDOWN;
        } else {
            st = QP_STATUS_BREAKDOWN;
        }
    }

finish:
    for (int i = tid; i < n; i += NT) Pz[i] = z[i];
    for (int k = tid; k < m; k += NT) { Ps[k] = s[k]; Plam[k] = lam[k]; }
    for (int k = tid; k < p; k += NT) Pnu[k] = nu[k];
    if (tid == 0) {
        status[Pout] = st;
        iters[Pout] = it;
        // the factor of the returned iterate is in the state unless the solve
        // broke down or met a non-finite value (the backward then writes zeros)
        *reinterpret_cast<int32_t *>(P.state + state_layout(sizeof(T), n, m, p).off_valid) =
            (st == QP_STATUS_BREAKDOWN || st == QP_STATUS_NONFINITE) ? 0 : 1;
    }
    __syncthreads();
}

}  // namespace qpmi
