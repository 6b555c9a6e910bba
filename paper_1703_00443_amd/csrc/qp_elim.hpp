// The paper's own elimination order for the Newton systems (Section 3.1.1,
// the footnote on the LU decomposition of K_sym): the nz x nz and neq x neq
// blocks, which do not involve D = D(lambda / s), are factored once per solve,
// and each iterate factors only an nineq x nineq matrix.
//
// With Qs = L_Q L_Q^T, U_Q = L_Q^{-T} (so Qs^{-1} = U_Q U_Q^T), the equality
// block in those coordinates At = A U_Q (the state's Wt region), its Schur
// complement S_A = At At^T = L_A L_A^T (inverse factor U_A, the state's US
// region) and the projector P_A = At^T S_A^{-1} At onto the row space of At:
//   V  = G U_Q                       nineq x nz
//   Vh = V (I - P_A)                 (= V when neq = 0)
//   Z  = V At^T S_A^{-1}             nineq x neq
//   C  = Vh Vh^T                     nineq x nineq, fixed for the solve
// C's strict lower triangle is kept in the strict lower triangle of the
// state's U region (U_Q uses the upper triangle only; nineq <= u_ld(nz)), its
// diagonal in LDS.
// The reduced system [H A^T; A 0][dz; dnu] = [f; r4] with H = Qs + G^T D G,
// written in xi = U_Q^{-1} dz and with w = D G dz eliminated last, becomes
//   u   = U_Q^T f
//   nu0 = S_A^{-1} (At u - r4),  xi0 = u - At^T nu0     (the solve with D = 0)
//   (C + D^{-1}) w = Vh xi0 + Z r4                       (the per-iterate factor)
//   xi  = xi0 - Vh^T w,  dnu = nu0 - Z^T w,  dz = U_Q xi
// which is the same solution as the policies that factor H, up to rounding.
// C + D^{-1} is factored with the register-tile Cholesky of the tiled policy.
//
// The caller factors Qs first (factor_qs); where that fails (Qs not positive
// definite in working precision) it solves the problem with the tiled policy
// instead.  The factor kept for the backward is the one the other policies
// keep (H at the returned iterate): it is formed and factored once more in
// finish(), so the backward is shared.
#pragma once
#include "qp_stream.hpp"

namespace qpmi {

// LDS regions of the elimination policy after the driver's vectors: the
// nineq x nineq register-tile factor's own region, then Vh (ld nz | 1), Z
// (ld pad4(neq)), the diagonal of C, the diagonal of C + D^{-1} and the
// solve's vectors.  The factorizations of Qs (prepare) and of H (finish) use
// the n x n tiled layout from the same base: both run while none of these
// regions is live.
// With `uq`, a copy of U_Q (upper triangle read, ld u_ld(nz)) follows, for the
// two triangular products of every solve.
struct ElimLayout {
    int vh, ldv, zz, ldz, cdg, dinv, u, xi, tn3, nu0, g1, wv, t1, t2, scr, uq, end;
    __host__ __device__ ElimLayout(int base, int n, int m, int p, bool with_uq) {
        // the nineq x nineq factor is seeded, never formed: its G staging
        // region (the end of its layout) is not used, and Vh starts there
        const TiledLayout<false> Ls(base, m, 0, 0);
        const int N = pad4(n), M = pad4(m), Pp = pad4(p);
        int o = Ls.G;
        ldv = n | 1; vh = o; o += m * ldv;
        ldz = Pp; zz = o; o += m * ldz;
        cdg = o; o += M;
        dinv = o; o += M;
        u = o; o += N; xi = o; o += N; tn3 = o; o += N;
        nu0 = o; o += Pp; g1 = o; o += M; wv = o; o += M; t1 = o; o += Pp; t2 = o; o += Pp;
        scr = o; o += 64 * kTiledWaves;
        uq = o; o += with_uq ? n * u_ld(n) : 0;
        end = o;
    }
};

// LDS elements of the policy: its own regions, and those of the nz x nz
// factorizations (the tiled layout, or BIG: the streamed one), whichever is larger;
// 0 when the streamed layout does not fit (BIG).
// Whether U_Q is copied to LDS: up to nz = 128, where the policy's regions
// with the copy still fit (a function of the dims and the LDS size only).
__host__ __device__ inline bool elim_uq_in_lds(int esz, int base, int n, int m, int p, int lds_limit) {
    if (n > kTiledMaxN) return false;
    const int a = ElimLayout(base, n, m, p, true).end, b = TiledLayout<false>(base, n, m, p).end;
    return (a > b ? a : b) * esz <= lds_limit;
}

__host__ __device__ inline int elim_lds_elems(int esz, int base, int n, int m, int p, bool big, int lds_limit) {
    const int a = ElimLayout(base, n, m, p, !big && elim_uq_in_lds(esz, base, n, m, p, lds_limit)).end;
    int b = TiledLayout<false>(base, n, m, p).end;
    if (big) {
        int kc = 4;
        bool s_lds = true;
        if (!stream_plan(esz, base, n, m, p, lds_limit, &kc, &s_lds)) return 0;
        b = StreamLayout(base, n, m, p, kc, s_lds).end;
    }
    return a > b ? a : b;
}

// out(i, j) = sum_{k < kdim} a(i, k) b(k, j) by 16x16 MFMA tiles, one
// wavefront per tile in turn (tiles above the diagonal skipped when `lower`);
// a and b return 0 outside their matrices; store(i, j, v) runs for i < rows,
// j < cols.  Ends with a workgroup barrier.
template <typename T, class FA, class FB, class FS>
__device__ __forceinline__ void tile_product(int rows, int cols, int kdim, bool lower, FA a, FB b, FS store) {
    using v4 = typename Mfma<T>::v4;
    const int t0 = opaque_tid();
    const int lane = t0 & 63, g = lane >> 4, c = lane & 15;
    const int w = __builtin_amdgcn_readfirstlane(t0 >> 6);
    const int rt = (rows + 15) / 16, ct = (cols + 15) / 16;
    for (int t = w; t < rt * ct; t += kTiledWaves) {
        const int I = t / ct, J = t - I * ct;
        if (lower && J > I) continue;
        v4 d = {0, 0, 0, 0};
        for (int kb = 0; kb < kdim; kb += 4) {
            const int k = kb + g;
            d = Mfma<T>::mma(a(16 * I + c, k), b(k, 16 * J + c), d);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * I + Mfma<T>::row(g, r), col = 16 * J + c;
            if (row < rows && col < cols) store(row, col, d[r]);
        }
    }
    __syncthreads();
}

// One register-tile factor object serves all three factorizations (Qs once,
// C + D^{-1} every Newton step, H at the end), re-aimed between the nz x nz
// and the nineq x nineq sizes: separate objects for them kept three sets of
// register tiles alive and spilled to scratch memory.  BIG (nz above the
// register tiles' 128): Qs and H are factored by the streamed-tile policy in
// the state buffer instead (objects local to factor_qs() and finish(), which
// hold no registers between its calls), and the register-tile object is only
// the nineq x nineq factor.
template <typename T, bool EQ, bool BIG = false>
struct ElimFactor {
    static constexpr int NT = 64 * kTiledWaves;
    // dz = U_Q (xi0 - Vh^T w) carries a rounding error of the size of
    // eps |U_Q| |U_Q^T f|, which does not shrink with the step.  It stays out
    // of the multiplier step, which is recovered from w (kSolveGz), not from
    // D G dz.  In FP64 that is enough (measured: the Newton step counts of the
    // tiled policy on every test problem); in FP32 it still slowed some
    // problems down to the step limit, and one refinement on the unreduced
    // residual every Newton step removes that.
    static constexpr bool kRefineAlways = sizeof(T) == 4;
    // the solve yields w = D G dz directly (the paper's unknown in the
    // nineq x nineq system); solve_g returns D^{-1} w for G dz
    static constexpr bool kSolveGz = true;
    static constexpr bool kFormResidual = false;
    using TF = TiledFactor<T, false, 8, EQ, false>;
    using SF = StreamFactor<T, EQ, false>;
    Prob<T> Pr;  // BIG: the streamed factor objects are built from it
    T *sm;
    int base;
    int n, m, p, ldu, ldv, ldz;
    const T *Q, *G;
    T *Ust, *Wt, *US;
    T *vh, *zz, *cdg, *dinv, *u, *xi, *tn3, *nu0, *g1, *wv, *t1, *t2, *scr;
    T *Uq;          // U_Q for the solves: the LDS copy where it fits, else the state's U region
    bool uq_lds;
    const T *Dcur;  // the scaling of the last factor() call
    TF tf;  // nz x nz in factor_qs(), prepare() and finish(), nineq x nineq in between

    __device__ __forceinline__ ElimFactor(const Prob<T> &P, T *sm_, int base_)
        : Pr(P), sm(sm_), base(base_), tf(P, sm_, base_) {
        n = P.n; m = P.m; p = P.p;
        Q = P.Q; G = P.G;
        const StateLayout SL = state_layout(sizeof(T), n, m, p);
        Ust = (T *)(P.state + SL.off_U);
        Wt = (T *)(P.state + SL.off_Wt);
        US = (T *)(P.state + SL.off_US);
        ldu = u_ld(n);
        uq_lds = !BIG && elim_uq_in_lds(sizeof(T), base, n, m, p, P.lds_limit);
        const ElimLayout L(base, n, m, p, uq_lds);
        Uq = uq_lds ? sm + L.uq : Ust;
        ldv = L.ldv; ldz = L.ldz;
        vh = sm + L.vh; zz = sm + L.zz; cdg = sm + L.cdg; dinv = sm + L.dinv;
        u = sm + L.u; xi = sm + L.xi; tn3 = sm + L.tn3; nu0 = sm + L.nu0; g1 = sm + L.g1;
        wv = sm + L.wv; t1 = sm + L.t1; t2 = sm + L.t2; scr = sm + L.scr;
    }

    // Once per solve, before the driver starts: U_Q, At and U_A into the
    // state.  False (uniformly) when Qs or A's Schur complement does not factor.
    __device__ __forceinline__ bool factor_qs() {
        if constexpr (BIG) {
            // the streamed policy factors in place in the state's U region
            // (upper triangle: U_Q), with equality rows At and S_A too
            SF qf(Pr, sm, base);
            qf.m = 0;  // H = Qs: no rows of G
            const bool ok = qf.factor(nullptr);
            if constexpr (EQ)
                if (ok && qf.s_lds)
                    for (int e = threadIdx.x; e < p * p; e += NT) {
                        const int i = e / p, j = e - i * p;
                        US[e] = qf.S[i * qf.lds + j];
                    }
            __syncthreads();
            return ok;
        }
        tf.retarget(n, 0, p, sm, base);  // H = Qs: no rows of G
        tf.prepare();                     // no equality rows: Qs staged in the state's U region
        const bool ok = tf.factor(nullptr);  // with equality rows: U_Q, At and S_A too
        if constexpr (!EQ) {
            if (ok) tf.store_u();
        } else {
            if (ok)
                for (int e = threadIdx.x; e < p * p; e += NT) {
                    const int i = e / p, j = e - i * p;
                    US[e] = tf.S[i * tf.lds + j];
                }
        }
        __syncthreads();
        return ok;
    }

    // The driver's once-per-solve step: Vh and Z into LDS; C below U_Q in the
    // state and its diagonal in LDS.
    __device__ __forceinline__ void prepare() {
        if (uq_lds) {
            // the upper triangle only: C is about to go below it in the state
            for (int e = threadIdx.x; e < n * ldu; e += NT) {
                const int i = e / ldu, j = e - i * ldu;
                if (j >= i && j < n) Uq[e] = Ust[e];
            }
            __syncthreads();
        }
        if (m == 0) return;
        const T *Gp = G, *Up = Ust;
        T *vp = vh;
        const int nn = n, mm = m, lu = ldu, lv = ldv;
        // V = G U_Q  (U_Q upper triangular)
        tile_product<T>(
            m, n, n, false,
            [=](int i, int k) {
                const bool in = i < mm && k < nn;
                const T v = Gp[in ? (size_t)i * nn + k : 0];
                return in ? v : T(0);
            },
            [=](int k, int j) {
                const bool in = k < nn && j < nn && k <= j;
                const T v = Up[in ? (size_t)k * lu + j : 0];
                return in ? v : T(0);
            },
            [=](int i, int j, T v) { vp[(size_t)i * lv + j] = v; });
        if constexpr (EQ) {
            const T *Wp = Wt;
            T *zp = zz;
            const int pp = p, lz = ldz;
            // Y = V At^T into Z's region
            tile_product<T>(
                m, p, n, false,
                [=](int i, int k) {
                    const bool in = i < mm && k < nn;
                    const T v = vp[in ? (size_t)i * lv + k : 0];
                    return in ? v : T(0);
                },
                [=](int k, int j) {
                    const bool in = k < nn && j < pp;
                    const T v = Wp[in ? (size_t)j * nn + k : 0];
                    return in ? v : T(0);
                },
                [=](int i, int j, T v) { zp[(size_t)i * lz + j] = v; });
            // Z = Y S_A^{-1} = (Y U_A) U_A^T, one row per thread, in place:
            // Y U_A from the last column down, then times U_A^T from the first
            for (int i = threadIdx.x; i < m; i += NT) {
                T *row = zz + (size_t)i * ldz;
                for (int j = p - 1; j >= 0; --j) {
                    T acc = 0;
                    for (int l = 0; l <= j; ++l) acc += row[l] * US[(size_t)l * p + j];
                    row[j] = acc;
                }
                for (int j = 0; j < p; ++j) {
                    T acc = 0;
                    for (int l = j; l < p; ++l) acc += row[l] * US[(size_t)j * p + l];
                    row[j] = acc;
                }
            }
            __syncthreads();
            // Vh = V - Z At
            tile_product<T>(
                m, n, p, false,
                [=](int i, int k) {
                    const bool in = i < mm && k < pp;
                    const T v = zp[in ? (size_t)i * lz + k : 0];
                    return in ? v : T(0);
                },
                [=](int k, int j) {
                    const bool in = k < pp && j < nn;
                    const T v = Wp[in ? (size_t)k * nn + j : 0];
                    return in ? v : T(0);
                },
                [=](int i, int j, T v) { vp[(size_t)i * lv + j] -= v; });
        }
        // C = Vh Vh^T (lower tiles): strict lower triangle under U_Q, diagonal to LDS
        T *cp = Ust, *dp = cdg;
        tile_product<T>(
            m, m, n, true,
            [=](int i, int k) {
                const bool in = i < mm && k < nn;
                const T v = vp[in ? (size_t)i * lv + k : 0];
                return in ? v : T(0);
            },
            [=](int k, int j) {
                const bool in = j < mm && k < nn;
                const T v = vp[in ? (size_t)j * lv + k : 0];
                return in ? v : T(0);
            },
            [=](int i, int j, T v) {
                if (i > j) cp[(size_t)i * lu + j] = v;
                else if (i == j) dp[i] = v;
            });
        tf.retarget(m, 0, 0, sm, base);  // the nineq x nineq factor from here on
    }

    // Per iterate: C + D^{-1} into the register tiles, Cholesky and inverse.
    __device__ __forceinline__ bool factor(const T *D) {
        Dcur = D;
        if (m == 0) return true;
        for (int k = threadIdx.x; k < m; k += NT) dinv[k] = cdg[k] + T(1) / D[k];
        __syncthreads();
        tf.seed(Ust, ldu, dinv);
        return tf.chol_inv();
    }

    __device__ __forceinline__ void solve(const T *f, const T *r4, T *dz, T *dnu) {
        ut_mv_split<T, NT>(Uq, ldu, n, f, u, scr);  // u = U_Q^T f
        const T *x0 = u;
        if constexpr (EQ) {
            mv_rows<T, NT>(Wt, n, p, n, u, t1);
            __syncthreads();
            for (int k = threadIdx.x; k < p; k += NT) t1[k] -= r4[k];
            __syncthreads();
            ut_mv<T, NT>(US, p, p, t1, t2);
            __syncthreads();
            u_mv<T, NT>(US, p, p, t2, nu0);
            __syncthreads();
            for (int i = threadIdx.x; i < n; i += NT) {
                T acc = u[i];
                for (int k = 0; k < p; ++k) acc -= Wt[(size_t)k * n + i] * nu0[k];
                xi[i] = acc;
            }
            __syncthreads();
            x0 = xi;
        }
        if (m > 0) {
            rowdot_split<T, NT>(vh, ldv, m, n, x0, g1, scr);  // Vh xi0
            if constexpr (EQ) {
                for (int k = threadIdx.x; k < m; k += NT) {
                    T acc = g1[k];
                    for (int j = 0; j < p; ++j) acc += zz[(size_t)k * ldz + j] * r4[j];
                    g1[k] = acc;
                }
                __syncthreads();
            }
            tf.solve(g1, nullptr, wv, nullptr);               // w = (C + D^{-1})^{-1} g1 (p = 0 here)
            colsum_split<T, NT>(vh, ldv, m, n, wv, tn3, scr);  // Vh^T w
            for (int i = threadIdx.x; i < n; i += NT) tn3[i] = x0[i] - tn3[i];
            if constexpr (EQ)
                for (int j = threadIdx.x; j < p; j += NT) {
                    T acc = nu0[j];
                    for (int k = 0; k < m; ++k) acc -= zz[(size_t)k * ldz + j] * wv[k];
                    dnu[j] = acc;
                }
            __syncthreads();
            x0 = tn3;
        } else if constexpr (EQ) {
            for (int j = threadIdx.x; j < p; j += NT) dnu[j] = nu0[j];
            __syncthreads();
        }
        u_mv<T, NT>(Uq, ldu, n, x0, dz);  // dz = U_Q xi
        __syncthreads();
    }

    // solve() and G dz as D^{-1} w from the same solve
    __device__ __forceinline__ void solve_g(const T *f, const T *r4, T *dz, T *dnu, T *gz) {
        solve(f, r4, dz, dnu);
        for (int k = threadIdx.x; k < m; k += NT) gz[k] = wv[k] / Dcur[k];
        __syncthreads();
    }

    __device__ __forceinline__ void gt_mv(const T *v, T *out) { colsum_split<T, NT>(G, n, m, n, v, out, scr); }
    __device__ __forceinline__ void g_mv(const T *x, T *out) {
        mv_rows<T, NT>(G, n, m, n, x, out);
        __syncthreads();
    }
    // Qs z = (Q z + Q^T z) / 2 over coalesced rows of Q (the state's U region
    // holds U_Q, not Qs)
    __device__ __forceinline__ void qs_mv(const T *z, T *out) {
        colsum_split<T, NT>(Q, n, n, n, z, out, scr);
        mv_rows<T, NT>(Q, n, n, n, z, tn3);
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += NT) out[i] = T(0.5) * (out[i] + tn3[i]);
        __syncthreads();
    }

    // The factor of H = Qs + G^T D G at the returned iterate, as the tiled
    // policy stores it (G staged in chunks through LDS).  The nineq x nineq
    // factor can stay positive definite at iterates where H no longer is in
    // working precision; false then (the driver returns the previous iterate).
    __device__ __forceinline__ bool finish(const T *D) {
        if constexpr (BIG) {
            SF hf(Pr, sm, base);
            return hf.factor(D) && hf.finish(D);
        }
        tf.retarget(n, m, p, sm, base);
        tf.prepare();
        return tf.factor(D) && tf.finish(D);
    }
};

}  // namespace qpmi
