// Backward kernels (Section 3.1.1, eq. grads-system and eq. grads).
//
// Kernel 1 (one workgroup per problem): solve the symmetrised KKT system at
// the solution with the factor stored by the forward,
//     K_sym [d_z; d_s; d~_lam; d_nu] = [-dl/dz; 0; 0; 0],
// where d~_lam = D(lambda) d_lam is the scaled multiplier adjoint, plus
// refine_steps steps of iterative refinement on the residual of the unreduced
// K_sym (matrix-vector products with Qs, G, A, D only; no new factorization).
// The adjoint vectors go to a workspace.
//
// Kernel 2 (many workgroups per problem, write-bound): the gradients
//     dQ = 1/2 (d_z z^T + z d_z^T),  dq = d_z,  dA = d_nu z^T + nu d_z^T,
//     db = -d_nu,  dG = d~_lam z^T + lambda d_z^T,  dh = -d~_lam.
#include "qp_core.hpp"

namespace qpmi {

template <typename T>
struct BProb {
    int n, m, p;
    const T *Q, *A, *G;
    const T *z, *lam, *nu, *s;
    const char *state;
    const T *g;
    T *adj;
    bool need;
    bool valid;  // the forward stored a factor (else the gradients are zero)
    // gradient outputs (nullable)
    T *dQ, *dq, *dA, *db, *dG, *dh;
};

template <typename T>
__device__ __forceinline__ BProb<T> bwd_problem(const BwdLaunch &L, int j) {
    BProb<T> P;
    if (L.desc == nullptr) {
        P.adj = (T *)L.adj + (size_t)j * L.adj_stride;
        P.n = L.nz; P.m = L.nineq; P.p = L.neq;
        P.Q = (const T *)L.Q + (size_t)j * L.sQ;
        P.A = (const T *)L.A + (size_t)j * L.sA;
        P.G = (const T *)L.G + (size_t)j * L.sG;
        P.z = (const T *)L.z + (size_t)j * P.n;
        P.lam = (const T *)L.lam + (size_t)j * P.m;
        P.s = (const T *)L.s + (size_t)j * P.m;
        P.nu = (const T *)L.nu + (size_t)j * P.p;
        P.g = (const T *)L.dl_dz + (size_t)j * P.n;
        P.state = L.state + (size_t)j * L.state_stride;
        P.need = true;
        const size_t n = P.n, m = P.m, p = P.p;
        P.dQ = L.dQ ? (T *)L.dQ + j * n * n : nullptr;
        P.dq = L.dq ? (T *)L.dq + j * n : nullptr;
        P.dA = L.dA ? (T *)L.dA + j * p * n : nullptr;
        P.db = L.db ? (T *)L.db + j * p : nullptr;
        P.dG = L.dG ? (T *)L.dG + j * m * n : nullptr;
        P.dh = L.dh ? (T *)L.dh + j * m : nullptr;
    } else {
        const qp_problem_desc d = L.desc[j];
        const T *base = (const T *)L.base_in;
        P.adj = (T *)L.adj + d.z + d.lam + d.nu;  // packed: prefix sum of nz + nineq + neq
        P.n = d.nz; P.m = d.nineq; P.p = d.neq;
        P.Q = base + d.Q; P.A = base + d.A; P.G = base + d.G;
        P.z = (const T *)L.z + d.z; P.lam = (const T *)L.lam + d.lam;
        P.s = (const T *)L.s + d.lam; P.nu = (const T *)L.nu + d.nu;
        P.g = (const T *)L.dl_dz + d.z;
        P.state = L.state + d.state;
        P.need = L.need ? (L.need[j] != 0) : true;
        T *gb = (T *)L.grad_base;
        P.dQ = gb + d.Q; P.dq = gb + d.q; P.dA = gb + d.A;
        P.db = gb + d.b; P.dG = gb + d.G; P.dh = gb + d.h;
    }
    P.valid = *reinterpret_cast<const int32_t *>(P.state + state_layout(sizeof(T), P.n, P.m, P.p).off_valid) != 0;
    return P;
}

struct BwdLayout {
    int z, g, dz, f, y, tn, tn2, r1, ez;              // n
    int lam, s, D, dl, ds, r2, r3, tm, el, es, tm2;   // m
    int nu, dn, r4, tp, tp2, en;                      // p
    int scr;                                          // partial sums of the split products
    int red, end;
    __host__ __device__ BwdLayout(int n, int m, int p) {
        const int N = pad4(n), M = pad4(m), Pp = pad4(p);
        int o = 0;
        z = o; o += N; g = o; o += N; dz = o; o += N; f = o; o += N; y = o; o += N;
        tn = o; o += N; tn2 = o; o += N; r1 = o; o += N; ez = o; o += N;
        lam = o; o += M; s = o; o += M; D = o; o += M; dl = o; o += M; ds = o; o += M;
        r2 = o; o += M; r3 = o; o += M; tm = o; o += M; el = o; o += M; es = o; o += M;
        tm2 = o; o += M;
        nu = o; o += Pp; dn = o; o += Pp; r4 = o; o += Pp; tp = o; o += Pp; tp2 = o; o += Pp;
        en = o; o += Pp;
        scr = o; o += 512;
        red = o; o += 64;
        end = o;
    }
};

// FP32 problems: the reduced adjoint system
//     [H A^T; A 0] [d_z; d_nu] = [-dl/dz; 0],   H = Qs + G^T D G,  D = lambda / s,
// (K_sym with d_s = -G d_z and d~_lam = D G d_z eliminated) is solved by
// projected preconditioned conjugate gradients (Gould, Hribar and Nocedal,
// 2001) with FP64 vectors, residuals and products (the FP32 inputs are exact
// in FP64).  Preconditioner and projection: the constraint system
// [M A^T; A 0] with the FP32 factor stored by the forward (M = its H),
// applied to the residual scaled to unit max norm.  After every projection
// the residual loses its A^T v part and v is accumulated into the multiplier
// (their residual update): the residual of projected CG tends to A^T nu, not
// to zero, and projecting that large vector in FP32 would leave an error that
// never shrinks.  Stationary refinement in
// FP32 stalls once cond(H) eps32 approaches 1; the Krylov iteration only
// needs the FP32 factor as a preconditioner.  At most 10 * refine_steps
// iterations; it stops when a correction of d_z, or the next one predicted
// from the rate of the last two, is below 1e-7 relative (about the resolution
// of the FP32 result).
// stage >= 1: Q, G and A are copied to LDS once (the iteration reads them
// four times per step); stage 2 also copies the stored factor (U, Wt, US),
// which every projection reads twice.  The choice depends on the problem's
// dims and the device LDS size only, and the same code runs on either copy.
struct BwdMixedLayout {
    int f, y, gz, r4, tp, tp2, gn, scr, qs, gs, as, us, wts, uss; // FP32, offsets in floats
    int x, r, gv, d, t1, t2, t3, tm, v, va, scr64, red;           // FP64, offsets in doubles from dbase
    int dbase, end;                                               // bytes
    __host__ __device__ BwdMixedLayout(int n, int m, int p, int stage) {
        const int N = pad4(n), M = pad4(m), Pp = pad4(p);
        int o = 0;
        f = o; o += N; y = o; o += N; gz = o; o += N;
        r4 = o; o += Pp; tp = o; o += Pp; tp2 = o; o += Pp; gn = o; o += Pp;
        scr = o; o += 512;
        qs = gs = as = us = wts = uss = 0;
        if (stage >= 1) { qs = o; o += n * n; gs = o; o += m * n; as = o; o += p * n; }
        if (stage >= 2) { us = o; o += u_ld(n) * u_ld(n); wts = o; o += p * n; uss = o; o += p * p; }
        dbase = (o * 4 + 15) & ~15;
        int q = 0;
        x = q; q += N; r = q; q += N; gv = q; q += N; d = q; q += N;
        t1 = q; q += N; t2 = q; q += N; t3 = q; q += N;
        tm = q; q += M; v = q; q += Pp; va = q; q += Pp; scr64 = q; q += 512; red = q; q += 64;
        end = dbase + q * 8;
    }
};

__host__ __device__ inline int bwd_mixed_stage(int n, int m, int p, int lds_limit) {
    if (BwdMixedLayout(n, m, p, 2).end <= lds_limit) return 2;
    return BwdMixedLayout(n, m, p, 1).end <= lds_limit ? 1 : 0;
}

// Refinement in the working precision (FP64, or FP32 with QP_FLAG_BWD_FP32):
// G (read six times per refinement step) is copied to LDS after the vectors
// when it fits; the choice depends on dims, element size and the device LDS only.
__host__ __device__ inline bool bwd_stage_g(int esz, int n, int m, int p, int lds_limit) {
    return ((size_t)BwdLayout(n, m, p).end + (size_t)m * n) * esz <= (size_t)lds_limit;
}

size_t bwd_vec_lds_bytes(int esz, int n, int m, int p, int lds_limit, unsigned flags) {
    if (esz == 4 && !(flags & QP_FLAG_BWD_FP32))
        return (size_t)BwdMixedLayout(n, m, p, bwd_mixed_stage(n, m, p, lds_limit)).end;
    return ((size_t)BwdLayout(n, m, p).end + (bwd_stage_g(esz, n, m, p, lds_limit) ? (size_t)m * n : 0)) * esz;
}

template <int NT, int STAGE>
__device__ void bwd_solve_mixed(const BProb<float> &P, unsigned char *smem, int refine_steps) {
    const int n = P.n, m = P.m, p = P.p;
    const int tid = threadIdx.x;
    const BwdMixedLayout Lo(n, m, p, STAGE);
    const StateLayout SL = state_layout(4, n, m, p);
    const float *U = (const float *)(P.state + SL.off_U);
    const float *Wt = (const float *)(P.state + SL.off_Wt);
    const float *US = (const float *)(P.state + SL.off_US);
    const float *__restrict__ lam = P.lam;
    const float *__restrict__ sl = P.s;
    float *fs = reinterpret_cast<float *>(smem);
    const float *Q = P.Q, *G = P.G, *A = P.A;
    if constexpr (STAGE >= 1) {
        float *qs = fs + Lo.qs, *gs = fs + Lo.gs, *as = fs + Lo.as;
        for (int e = tid; e < n * n; e += NT) qs[e] = P.Q[e];
        for (int e = tid; e < m * n; e += NT) gs[e] = P.G[e];
        for (int e = tid; e < p * n; e += NT) as[e] = P.A[e];
        Q = qs; G = gs; A = as;
    }
    if constexpr (STAGE >= 2) {
        float *us = fs + Lo.us, *wts = fs + Lo.wts, *uss = fs + Lo.uss;
        const int lu = u_ld(n);
        for (int e = tid; e < lu * lu; e += NT) us[e] = U[e];
        for (int e = tid; e < p * n; e += NT) wts[e] = Wt[e];
        for (int e = tid; e < p * p; e += NT) uss[e] = US[e];
        U = us; Wt = wts; US = uss;
    }
    if constexpr (STAGE >= 1) __syncthreads();
    double *ds = reinterpret_cast<double *>(smem + Lo.dbase);
    float *f = fs + Lo.f, *y = fs + Lo.y, *gz = fs + Lo.gz, *r4 = fs + Lo.r4, *tp = fs + Lo.tp,
          *tp2 = fs + Lo.tp2, *gn = fs + Lo.gn, *scr = fs + Lo.scr;
    double *x = ds + Lo.x, *r = ds + Lo.r, *gv = ds + Lo.gv, *d = ds + Lo.d, *t1 = ds + Lo.t1,
           *t2 = ds + Lo.t2, *t3 = ds + Lo.t3, *tm = ds + Lo.tm, *v = ds + Lo.v, *va = ds + Lo.va,
           *scr64 = ds + Lo.scr64, *red = ds + Lo.red;

    // t1 = H w  (FP64); returns w^T H w
    auto h_mv = [&](const double *w) {
        mv_rows<float, NT, double>(Q, n, n, n, w, t1);
        mv_rows<float, NT, double>(G, n, m, n, w, tm);
        colsum_split<float, NT, double>(Q, n, n, n, w, t2, scr64);  // ends with a barrier
        for (int k = tid; k < m; k += NT) tm[k] *= (double)lam[k] / (double)sl[k];
        __syncthreads();
        colsum_split<float, NT, double>(G, n, m, n, tm, t3, scr64);
        double acc = 0;
        for (int i = tid; i < n; i += NT) {
            const double h = 0.5 * (t1[i] + t2[i]) + t3[i];
            t1[i] = h;
            acc += w[i] * h;
        }
        return block_sum<double, NT>(acc, red);  // its barriers also publish t1
    };
    // (gv, v): the solution of [M A^T; A 0] [gv; v] = [w; 0] in FP32 on w scaled to unit max norm
    auto project = [&](double *w) {
        double *w_upd = w;
        double mx = 0, d0 = 0, d1 = 0;
        for (int i = tid; i < n; i += NT) mx = fmax(mx, fabs(w[i]));
        block_reduce3<double, NT>(d0, mx, d1, red);
        const double sc = (mx > 0 && isfinite(mx)) ? mx : 0.0;
        const double inv = sc > 0 ? 1.0 / sc : 0.0;
        for (int i = tid; i < n; i += NT) f[i] = (float)(w[i] * inv);
        for (int k = tid; k < p; k += NT) r4[k] = 0.f;
        __syncthreads();
        kkt_solve<float, NT>(U, u_ld(n), Wt, US, n, p, f, r4, y, tp, tp2, gz, gn, scr);
        for (int i = tid; i < n; i += NT) gv[i] = sc * (double)gz[i];
        for (int k = tid; k < p; k += NT) v[k] = sc * (double)gn[k];
        __syncthreads();
        if (p > 0) {  // residual update: r -= A^T v, multiplier += v
            colsum_split<float, NT, double>(A, n, p, n, v, t2, scr64);  // ends with a barrier
            for (int i = tid; i < n; i += NT) w_upd[i] -= t2[i];
            for (int k = tid; k < p; k += NT) va[k] += v[k];
            __syncthreads();
        }
    };
    auto dot = [&](const double *a, const double *b) {
        double acc = 0;
        for (int i = tid; i < n; i += NT) acc += a[i] * b[i];
        return block_sum<double, NT>(acc, red);
    };

    // x = 0, r = H x - (-g) = g, accumulated multiplier va = 0
    for (int i = tid; i < n; i += NT) { x[i] = 0.0; r[i] = (double)P.g[i]; }
    for (int k = tid; k < p; k += NT) va[k] = 0.0;
    __syncthreads();
    project(r);
    for (int i = tid; i < n; i += NT) d[i] = -gv[i];
    __syncthreads();
    double rg = dot(r, gv);
    const int max_it = 10 * (refine_steps > 0 ? refine_steps : 1);
    double prev_upd = 0;
    for (int it = 0; it < max_it && rg > 0 && isfinite(rg); ++it) {
        const double dhd = h_mv(d);
        if (!(dhd > 0) || !isfinite(dhd)) break;
        const double alpha = rg / dhd;
        double upd = 0, nxm = 0, d0 = 0;  // nxm: -max|x| through the min slot
        for (int i = tid; i < n; i += NT) {
            const double dx = alpha * d[i];
            x[i] += dx;
            r[i] += alpha * t1[i];
            upd = fmax(upd, fabs(dx));
            nxm = fmin(nxm, -fabs(x[i]));
        }
        block_reduce3<double, NT>(d0, upd, nxm, red);
        // converged: this correction, or the next one predicted from the rate of
        // the last two, below 1e-7 of d_z
        const double tolx = 1e-7 * -nxm;
        if (upd <= tolx || (prev_upd > 0 && upd * (upd / prev_upd) <= tolx)) break;
        prev_upd = upd;
        project(r);
        const double rg2 = dot(r, gv);
        const double beta = rg2 / rg;
        for (int i = tid; i < n; i += NT) d[i] = -gv[i] + beta * d[i];
        __syncthreads();
        rg = rg2;
    }
    // r = H x + g - A^T va  ->  0:  H x + A^T (-va) = -g,  so nu = -va
    // d_s = -G d_z (not stored), d~_lam = D G d_z
    mv_rows<float, NT, double>(G, n, m, n, x, tm);
    __syncthreads();
    for (int i = tid; i < n; i += NT) P.adj[i] = (float)x[i];
    for (int k = tid; k < m; k += NT) P.adj[n + k] = (float)((double)lam[k] / (double)sl[k] * tm[k]);
    for (int k = tid; k < p; k += NT) P.adj[n + m + k] = (float)(-va[k]);
    __syncthreads();
}

// WP: refinement in the working precision (FP64; FP32 with QP_FLAG_BWD_FP32).
// The two FP32 schemes are separate instantiations: carrying both in one
// kernel raised the default one from 154 registers to 256 with spills.
template <typename T, int NT, bool WP>
__global__ __launch_bounds__(NT) void qp_backward_solve_kernel(BwdLaunch L) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);
    const int tid = threadIdx.x;
    for (int j = blockIdx.x; j < L.count; j += gridDim.x) {
        const BProb<T> P = bwd_problem<T>(L, j);
        if (!P.need) continue;
        if (!P.valid) {  // no factor was stored: zero adjoint (the gradients are written as zeros)
            for (int e = tid; e < P.n + P.m + P.p; e += NT) P.adj[e] = T(0);
            continue;
        }
        if constexpr (!WP && sizeof(T) == 4) {
            const int stage = bwd_mixed_stage(P.n, P.m, P.p, L.lds_limit);
            if (stage == 2)
                bwd_solve_mixed<NT, 2>(P, smem_raw, L.refine_steps);
            else if (stage == 1)
                bwd_solve_mixed<NT, 1>(P, smem_raw, L.refine_steps);
            else
                bwd_solve_mixed<NT, 0>(P, smem_raw, L.refine_steps);
        } else {
        const int n = P.n, m = P.m, p = P.p;
        const BwdLayout Lo(n, m, p);
        const StateLayout SL = state_layout(sizeof(T), n, m, p);
        const T *U = (const T *)(P.state + SL.off_U);
        const T *Dst = (const T *)(P.state + SL.off_D);
        const T *Wt = (const T *)(P.state + SL.off_Wt);
        const T *US = (const T *)(P.state + SL.off_US);
        const T *__restrict__ Q = P.Q;
        const bool sg = bwd_stage_g(sizeof(T), n, m, p, L.lds_limit);
        if (sg) {
            T *gs = sm + Lo.end;
            for (int e = tid; e < m * n; e += NT) gs[e] = P.G[e];
        }
        const T *__restrict__ G = sg ? sm + Lo.end : P.G;
        const T *__restrict__ A = P.A;
        T *z = sm + Lo.z, *g = sm + Lo.g, *dz = sm + Lo.dz, *f = sm + Lo.f, *y = sm + Lo.y,
          *tn = sm + Lo.tn, *tn2 = sm + Lo.tn2, *r1 = sm + Lo.r1, *ez = sm + Lo.ez;
        T *lam = sm + Lo.lam, *s = sm + Lo.s, *D = sm + Lo.D, *dl = sm + Lo.dl, *ds = sm + Lo.ds,
          *r2 = sm + Lo.r2, *r3 = sm + Lo.r3, *tm = sm + Lo.tm, *el = sm + Lo.el, *es = sm + Lo.es,
          *tm2 = sm + Lo.tm2;
        T *nu = sm + Lo.nu, *dn = sm + Lo.dn, *r4 = sm + Lo.r4, *tp = sm + Lo.tp,
          *tp2 = sm + Lo.tp2, *en = sm + Lo.en, *scr = sm + Lo.scr;

        for (int i = tid; i < n; i += NT) { z[i] = P.z[i]; g[i] = P.g[i]; f[i] = -P.g[i]; }
        for (int k = tid; k < m; k += NT) { lam[k] = P.lam[k]; s[k] = P.s[k]; D[k] = Dst[k]; }
        for (int k = tid; k < p; k += NT) { nu[k] = P.nu[k]; r4[k] = T(0); }
        __syncthreads();
        kkt_solve<T, NT>(U, u_ld(n), Wt, US, n, p, f, r4, y, tp, tp2, dz, dn, scr);
        mv_rows<T, NT>(G, n, m, n, dz, tm);
        __syncthreads();
        for (int k = tid; k < m; k += NT) { ds[k] = -tm[k]; dl[k] = D[k] * tm[k]; }
        __syncthreads();

        // Iterative refinement on the unreduced K_sym residual, at most
        // refine_steps steps.  Each step multiplies the error by a factor rho
        // that the corrections estimate: for the first one its own size
        // relative to the solution (the relative error of one reduced solve),
        // later the ratio of consecutive corrections.  It stops once the error
        // left, the correction times rho, is below 1e-8 of the solution; a
        // correction larger than half the previous one (no longer converging)
        // is not applied.  Near the end of a solve H can be ill-conditioned
        // enough that one step leaves an adjoint error of 1e-2 where several
        // steps reach 1e-6 or better.
        T *red = sm + Lo.red;
        T prev_applied = pinf<T>();
        for (int r = 0; r < L.refine_steps; ++r) {
            // residual of K_sym [dz; ds; dl; dn] = [-g; 0; 0; 0]
            mv_rows<T, NT>(Q, n, n, n, dz, tn);
            mv_rows<T, NT>(G, n, m, n, dz, tm);
            if (p > 0) mv_rows<T, NT>(A, n, p, n, dz, tp);
            colsum_split<T, NT>(Q, n, n, n, dz, tn2, scr);
            colsum_split<T, NT>(G, n, m, n, dl, r1, scr);
            if (p > 0) colsum_split<T, NT>(A, n, p, n, dn, y, scr);
            for (int i = tid; i < n; i += NT) {
                T acc = T(0.5) * (tn[i] + tn2[i]) + r1[i];
                if (p > 0) acc += y[i];
                r1[i] = -g[i] - acc;
            }
            for (int k = tid; k < m; k += NT) {
                const T a2 = -(D[k] * ds[k] + dl[k]);
                const T a3 = -(tm[k] + ds[k]);
                r2[k] = a2;
                r3[k] = a3;
                tm2[k] = a2 - D[k] * a3;
            }
            for (int k = tid; k < p; k += NT) r4[k] = -tp[k];
            __syncthreads();
            // correction: f = r1 - G^T (r2 - D r3)
            colsum_split<T, NT>(G, n, m, n, tm2, f, scr);
            for (int i = tid; i < n; i += NT) f[i] = r1[i] - f[i];
            __syncthreads();
            kkt_solve<T, NT>(U, u_ld(n), Wt, US, n, p, f, r4, y, tp, tp2, ez, en, scr);
            mv_rows<T, NT>(G, n, m, n, ez, tm);
            __syncthreads();
            T emax = 0, nx = 0, dmy = 0;  // nx: minus the largest entry of the solution
            for (int i = tid; i < n; i += NT) { emax = fmax(emax, fabs(ez[i])); nx = fmin(nx, -fabs(dz[i])); }
            for (int k = tid; k < m; k += NT) {
                const T e_s = r3[k] - tm[k];
                const T e_l = r2[k] - D[k] * e_s;
                emax = fmax(emax, fmax(fabs(e_s), fabs(e_l)));
                nx = fmin(nx, -fmax(fabs(ds[k]), fabs(dl[k])));
            }
            for (int k = tid; k < p; k += NT) { emax = fmax(emax, fabs(en[k])); nx = fmin(nx, -fabs(dn[k])); }
            block_reduce3<T, NT>(dmy, emax, nx, red);
            if (r > 0 && emax > T(0.5) * prev_applied) break;
            for (int k = tid; k < m; k += NT) {
                const T e_s = r3[k] - tm[k];
                const T e_l = r2[k] - D[k] * e_s;
                ds[k] += e_s;
                dl[k] += e_l;
            }
            for (int i = tid; i < n; i += NT) dz[i] += ez[i];
            for (int k = tid; k < p; k += NT) dn[k] += en[k];
            __syncthreads();
            {
                // the target: 1e-8 of the solution in FP64, 1e-4 in FP32
                const T xs = fmax(-nx, sizeof(T) == 8 ? T(1e-300) : T(1e-30));
                const T rho = r == 0 ? emax / xs : emax / prev_applied;
                if (emax * rho <= (sizeof(T) == 8 ? T(1e-8) : T(1e-4)) * xs) break;
            }
            prev_applied = emax;
        }
        for (int i = tid; i < n; i += NT) P.adj[i] = dz[i];
        for (int k = tid; k < m; k += NT) P.adj[n + k] = dl[k];
        for (int k = tid; k < p; k += NT) P.adj[n + m + k] = dn[k];
        __syncthreads();
        }
    }
}

// Gradient assembly: blockIdx.x = problem, blockIdx.y = group of kRowsPerBlock
// rows of the concatenation [dQ (n rows); dG (m rows); dA (p rows); vectors].
constexpr int kRowsPerBlock = 8;

template <typename T, int NT>
__global__ __launch_bounds__(NT) void qp_grad_assemble_kernel(BwdLaunch L) {
    constexpr int NW = NT / 64;
    const int j = blockIdx.x;
    const BProb<T> P = bwd_problem<T>(L, j);
    if (!P.need) return;
    const int n = P.n, m = P.m, p = P.p;
    const int R = n + m + p + 1;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const T *dz = P.adj, *dl = P.adj + n, *dn = P.adj + n + m;
    // without a stored factor (forward BREAKDOWN / NONFINITE) every gradient is
    // zero: the adjoint is zero and the iterate is not read (it may be non-finite)
    const T *z = P.valid ? P.z : P.adj;  // the adjoint's zeros stand in for z
    const T *lamv = P.valid ? P.lam : P.adj + n;
    const T *nuv = P.valid ? P.nu : P.adj + n + m;
    for (int rr = w; rr < kRowsPerBlock; rr += NW) {
        const int r = blockIdx.y * kRowsPerBlock + rr;
        if (r >= R) break;
        if (r < n) {
            if (!P.dQ) continue;
            const T dzi = dz[r], zi = z[r];
            T *row = P.dQ + (size_t)r * n;
            for (int c = lane; c < n; c += 64) row[c] = T(0.5) * (dzi * z[c] + zi * dz[c]);
        } else if (r < n + m) {
            if (!P.dG) continue;
            const int k = r - n;
            const T a = dl[k], lk = lamv[k];
            T *row = P.dG + (size_t)k * n;
            for (int c = lane; c < n; c += 64) row[c] = a * z[c] + lk * dz[c];
        } else if (r < n + m + p) {
            if (!P.dA) continue;
            const int k = r - n - m;
            const T a = dn[k], nk = nuv[k];
            T *row = P.dA + (size_t)k * n;
            for (int c = lane; c < n; c += 64) row[c] = a * z[c] + nk * dz[c];
        } else {
            if (P.dq) for (int c = lane; c < n; c += 64) P.dq[c] = dz[c];
            if (P.dh) for (int c = lane; c < m; c += 64) P.dh[c] = -dl[c];
            if (P.db) for (int c = lane; c < p; c += 64) P.db[c] = -dn[c];
        }
    }
}

constexpr int kBwdThreads = 512;

template <typename T>
static hipError_t launch_bwd_t(const BwdLaunch &L, hipStream_t st, int max_rows) {
    if (L.count <= 0) return hipSuccess;
    // FP64 always refines in its own precision; FP32 does with QP_FLAG_BWD_FP32
    const bool wp = sizeof(T) == 8 || (L.flags & QP_FLAG_BWD_FP32) != 0;
    auto k1 = qp_backward_solve_kernel<T, kBwdThreads, true>;
    if constexpr (sizeof(T) == 4)
        if (!wp) k1 = qp_backward_solve_kernel<T, kBwdThreads, false>;
    static bool attr_done[2] = {false, false};
    if (!attr_done[wp]) {
        (void)hipFuncSetAttribute((const void *)k1, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsLimit);
        attr_done[wp] = true;
    }
    hipLaunchKernelGGL(k1, dim3(L.count), dim3(kBwdThreads), L.lds_bytes, st, L);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int gx = (max_rows + kRowsPerBlock - 1) / kRowsPerBlock;
    hipLaunchKernelGGL((qp_grad_assemble_kernel<T, kBwdThreads>), dim3(L.count, gx), dim3(kBwdThreads),
                       0, st, L);
    return hipGetLastError();
}

hipError_t launch_backward(qp_dtype dt, const BwdLaunch &L, hipStream_t st) {
    return dt == QP_F64 ? launch_bwd_t<double>(L, st, L.max_rows) : launch_bwd_t<float>(L, st, L.max_rows);
}

}  // namespace qpmi
