// Streamed-tile factorization policy for problems whose factor does not fit
// in registers or LDS: the padded square of 16x16 tiles is factored in place
// in the U region of the state buffer (ld u_ld(nz)), and the tiles stream
// through the registers of the eight wavefronts for each MFMA update.
//
//   form:  H = Qs + G^T D G, lower tiles, GT output tiles per wavefront and
//          pass held in MFMA accumulators; G streamed through LDS in chunks
//          of kc rows (each pass reads G once); upper tiles zeroed.
//   chol:  the fused Cholesky + inverse of the tiled policy, by 16-column
//          panels: column P of the square to LDS, the diagonal tile's 16
//          steps in one wavefront, panel tiles times X_PP^T, then the
//          rank-16 update of every tile right of the panel (loaded from the
//          state, four MFMAs, stored back), four tiles in flight per wavefront.
//   solve: triangular matrix-vector products over the stored U.
//   Schur complement on A (equality rows): as in the tiled policy.
//   UNIT (QP_FLAG_G_UNIT_ROWS, a separate instantiation): G^T D G is the
//          diagonal of per-column sums of D (no G streaming), and products with
//          G are gathers; the row lists sit in the staging region after the
//          Schur block, which neither the factorization nor the solves use.
#pragma once
#include "qp_policies.hpp"

namespace qpmi {

// s_lds: the Schur block S sits in LDS (sharing the staging buffer); otherwise
// it is factored in place in the US region of the state.
struct StreamLayout {
    int yv, xv, panel, scratch, flag, xdp, pv1, pv2, buf, end;
    __host__ __device__ StreamLayout(int base, int n, int m, int p, int kc, bool s_lds) {
        (void)m;
        const int nt = (n + 15) / 16, np = 16 * nt;
        int o = base;
        yv = o; o += np; xv = o; o += np;
        panel = o; o += np * 17;
        scratch = o; o += 64 * kTiledWaves;
        flag = o; o += 4;
        xdp = o; o += pad4(p); pv1 = o; o += pad4(p); pv2 = o; o += pad4(p);
        o = (o + 15) & ~15;
        buf = o;  // G staging chunk, then the Schur block S (ld p | 1)
        const int gsz = kc * (np + 1), ssz = (p > 0 && s_lds) ? p * h_ld(p) : 0;
        end = o + (gsz > ssz ? gsz : ssz);
    }
};

// Plan of the policy: rows of G per staging chunk (the largest of 64, 32, ...,
// 4 that fits), with S in LDS if any chunk size fits that way, else with S in
// the state.  Returns false when nothing fits.
__host__ __device__ inline bool stream_plan(int esz, int base, int n, int m, int p, int lds_limit, int *kc,
                                            bool *s_lds) {
    for (int pass = 0; pass < 2; ++pass) {
        const bool sl = pass == 0;
        if (!sl && p == 0) break;
        for (int k = 64; k >= 4; k >>= 1)
            if (StreamLayout(base, n, m, p, k, sl).end * esz <= lds_limit) {
                *kc = k;
                *s_lds = sl;
                return true;
            }
    }
    return false;
}

template <typename T, bool EQ, bool UNIT = false>
struct StreamFactor {
    static constexpr bool kRefineAlways = false;
    static constexpr bool kSolveGz = false;
    // the residual's G z and G^T lam from the rows of G the formation stages
    // (not in the unit-row instantiation, whose products are gathers)
    static constexpr bool kFormResidual = !UNIT;
    static constexpr int NT = 64 * kTiledWaves;
    static constexpr int GT = 8;   // form(): tiles per wavefront and pass
    static constexpr int SE = sizeof(T) == 4 ? 32 : 16;  // form(): G elements staged per thread and chunk
    using v4 = typename Mfma<T>::v4;
    int n, m, p, nt, np, pt, ldg, lds, ldu, kc;
    bool s_lds;
    const T *Q, *Gsrc, *A;
    T *U, *Dst, *Wt, *US;
    T *yv, *xv, *panel, *scratch, *xdp, *pv1, *pv2, *gbuf, *S;
    int fcap;  // form(): elements from the panel to the end of the layout (idle during the formation)
    int *flag;
    bool unit;
    UnitRows<T, NT> ur;
    int w, lane, g, c;

    __device__ __forceinline__ void lane_ids() {
        const int t = opaque_tid();
        lane = t & 63; g = lane >> 4; c = lane & 15;
        w = __builtin_amdgcn_readfirstlane(t >> 6);
    }

    __device__ __forceinline__ StreamFactor(const Prob<T> &P, T *sm, int base) {
        n = P.n; m = P.m; p = P.p;
        nt = (n + 15) / 16; np = 16 * nt; pt = (p + 15) / 16;
        Q = P.Q; Gsrc = P.G; A = P.A;
        const StateLayout SL = state_layout(sizeof(T), n, m, p);
        U = (T *)(P.state + SL.off_U);
        Dst = (T *)(P.state + SL.off_D);
        Wt = (T *)(P.state + SL.off_Wt);
        US = (T *)(P.state + SL.off_US);
        kc = 4; s_lds = true;
        (void)stream_plan(sizeof(T), base, n, m, p, P.lds_limit, &kc, &s_lds);
        const StreamLayout L(base, n, m, p, kc, s_lds);
        yv = sm + L.yv; xv = sm + L.xv; panel = sm + L.panel; scratch = sm + L.scratch;
        flag = reinterpret_cast<int *>(sm + L.flag);
        xdp = sm + L.xdp; pv1 = sm + L.pv1; pv2 = sm + L.pv2;
        gbuf = sm + L.panel;
        fcap = L.end - L.panel;
        ldg = np + 1; ldu = u_ld(n);
        if (s_lds) { S = sm + L.buf; lds = h_ld(p); } else { S = US; lds = p; }
        lane = threadIdx.x & 63; w = threadIdx.x >> 6; g = lane >> 4; c = lane & 15;
        const int uo = L.buf + ((EQ && s_lds) ? p * h_ld(p) : 0);
        unit = UNIT && (P.flags & QP_FLAG_G_UNIT_ROWS) != 0 && m > 0 &&
               uo + UnitRows<T, NT>::elems(n, m) <= L.end;
        ur.place(sm + uo, n, m);
    }

    __device__ __forceinline__ void prepare() {
        if (UNIT && unit) unit = ur.detect(Gsrc, n, m, scratch);
    }

    // Lower tile t (row-major order over the lower triangle of the tile grid).
    __device__ __forceinline__ static void lower_tile(int t, int &I, int &J) {
        int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
        while ((i + 1) * (i + 2) / 2 <= t) ++i;
        while (i * (i + 1) / 2 > t) --i;
        I = i;
        J = t - i * (i + 1) / 2;
    }

    // RES: the first pass over the tiles also takes gz = G zr (16 lanes per
    // row, as mv_rows), the row weights wsc = lr + D rz with
    // rz = -(gz + sv - hv), gtl = G^T lr and gtw = G^T wsc (accumulated by the
    // thread that owns the column) from each staged chunk, so that neither the
    // residual of the iterate nor the affine right-hand side needs a pass of
    // its own over G.
    template <bool RES = false>
    __device__ __forceinline__ void form(const T *D, const T *zr = nullptr, const T *lr = nullptr,
                                         const T *sv = nullptr, const T *hv = nullptr,
                                         T *gz = nullptr, T *gtl = nullptr, T *gtw = nullptr,
                                         T *wsc = nullptr) {
        if (UNIT && unit) ur.diag(D, xv, n);  // G^T D G is diagonal
        if constexpr (RES)
            for (int i = threadIdx.x; i < n; i += NT) { gtl[i] = T(0); gtw[i] = T(0); }
        lane_ids();
        // upper tiles start at zero (they become X^T = L^{-T} strictly above the diagonal)
        for (int t = w; t < nt * nt; t += kTiledWaves) {
            const int I = t / nt, J = t - I * nt;
            if (I >= J) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) U[(size_t)(16 * I + Mfma<T>::row(g, r)) * ldu + 16 * J + c] = T(0);
        }
        const int NL = nt * (nt + 1) / 2;
        // chunk rows: what fits in the region from the panel to the end of the
        // layout (the panel, the solve vectors and the Schur block are idle
        // during the formation), at most 64 and at most SE elements per
        // thread; staged element i of this thread sits at row-major position
        // threadIdx.x + i NT of the chunk, walked without divisions
        const int kcf = min(64, (fcap / ldg) & ~3);
        const int kcr = min(kcf, max(4, ((SE * NT) / np) & ~3));
        const int q_np = NT / np, r_np = NT - q_np * np;
        const int k_base = threadIdx.x / np, c_base = threadIdx.x - k_base * np;
        for (int t0 = 0; t0 < NL; t0 += kTiledWaves * GT) {
            int ti[GT], tj[GT];
            v4 acc[GT];
#pragma unroll
            for (int j = 0; j < GT; ++j) {
                const int t = t0 + w * GT + j;
                int I = -1, J = 0;
                if (t < NL) lower_tile(t, I, J);
                // wave-uniform: keep the tile coordinates in scalar registers
                I = __builtin_amdgcn_readfirstlane(I);
                J = __builtin_amdgcn_readfirstlane(J);
                ti[j] = I; tj[j] = J;
                v4 a = {0, 0, 0, 0};
                if (I >= 0) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = 16 * I + Mfma<T>::row(g, r), col = 16 * J + c;
                        const bool in = row < n && col < n;
                        const T qa = Q[in ? (size_t)row * n + col : 0];
                        const T qb = Q[in ? (size_t)col * n + row : 0];
                        T qs = T(0.5) * (qa + qb);
                        if (UNIT && unit && in && row == col) qs += xv[row];
                        a[r] = in ? qs : (row == col ? T(1) : T(0));
                    }
                }
                acc[j] = a;
            }
            for (int k0 = 0; k0 < ((UNIT && unit) ? 0 : m); k0 += kcr) {
                const int rows = min(kcr, m - k0), rp = (rows + 3) & ~3;
                // all SE loads of this thread are issued before any store
                T stg[SE];
                {
                    int k = k_base, col = c_base;
#pragma unroll
                    for (int i = 0; i < SE; ++i) {
                        const bool v = k < rows && col < n;
                        const T x = Gsrc[v ? (size_t)(k0 + k) * n + col : 0];
                        stg[i] = v ? x : T(0);
                        k += q_np; col += r_np;
                        if (col >= np) { col -= np; ++k; }
                    }
                }
                __syncthreads();  // previous chunk consumed
                {
                    int k = k_base, col = c_base;
#pragma unroll
                    for (int i = 0; i < SE; ++i) {
                        if (k < rp) gbuf[k * ldg + col] = stg[i];
                        k += q_np; col += r_np;
                        if (col >= np) { col -= np; ++k; }
                    }
                }
                __syncthreads();
                lane_ids();
                if constexpr (RES)
                    if (t0 == 0) chunk_rows_res<T, NT>(gbuf, ldg, k0, rows, n, zr, lr, D, sv, hv, gz, wsc);
                for (int kb = 0; kb < rows; kb += 4) {
                    const int k = kb + g;
                    const T *Gk = gbuf + k * ldg;
                    const int kg = k0 + k;
                    const T dk = D[kg < m ? kg : m - 1] * T(kg < m ? 1 : 0);
                    // all operand loads first (unused tiles read row 0), then the MFMAs
                    T av[GT], bv[GT];
#pragma unroll
                    for (int j = 0; j < GT; ++j) {
                        const int I = ti[j] < 0 ? 0 : ti[j];
                        av[j] = Gk[16 * I + c];
                        bv[j] = dk * Gk[16 * tj[j] + c];
                    }
#pragma unroll
                    for (int j = 0; j < GT; ++j) {
                        if (ti[j] < 0) continue;
                        acc[j] = Mfma<T>::mma(av[j], bv[j], acc[j]);
                    }
                }
                if constexpr (RES) {
                    if (t0 == 0) {
                        __syncthreads();  // the chunk's row weights
                        for (int i = threadIdx.x; i < n; i += NT) {
                            T a0 = 0, a1 = 0, a2 = 0, a3 = 0, b0 = 0, b1 = 0, b2 = 0, b3 = 0;
                            int k = 0;
                            for (; k + 3 < rows; k += 4) {
                                const T g0 = gbuf[k * ldg + i], g1 = gbuf[(k + 1) * ldg + i];
                                const T g2 = gbuf[(k + 2) * ldg + i], g3 = gbuf[(k + 3) * ldg + i];
                                a0 += g0 * lr[k0 + k];
                                a1 += g1 * lr[k0 + k + 1];
                                a2 += g2 * lr[k0 + k + 2];
                                a3 += g3 * lr[k0 + k + 3];
                                b0 += g0 * wsc[k0 + k];
                                b1 += g1 * wsc[k0 + k + 1];
                                b2 += g2 * wsc[k0 + k + 2];
                                b3 += g3 * wsc[k0 + k + 3];
                            }
                            for (; k < rows; ++k) {
                                const T g0 = gbuf[k * ldg + i];
                                a0 += g0 * lr[k0 + k];
                                b0 += g0 * wsc[k0 + k];
                            }
                            gtl[i] += (a0 + a1) + (a2 + a3);
                            gtw[i] += (b0 + b1) + (b2 + b3);
                        }
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < GT; ++j) {
                if (ti[j] < 0) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * ti[j] + Mfma<T>::row(g, r), col = 16 * tj[j] + c;
                    U[(size_t)row * ldu + col] = (ti[j] == tj[j] && row < col) ? T(0) : acc[j][r];
                }
            }
        }
        __syncthreads();
    }

    // Trailing tile u of panel P: columns C > P, rows R <= P or R >= C, in
    // column-major order of that set.
    __device__ __forceinline__ void trail_tile(int P, int u, int &R, int &C) const {
        int cc = P + 1, cnt = P + 1 + nt - cc;
        while (u >= cnt) { u -= cnt; ++cc; cnt = P + 1 + nt - cc; }
        C = cc;
        R = (u <= P) ? u : cc + (u - (P + 1));
    }

    __device__ __forceinline__ bool chol_inv() {
        if (threadIdx.x == 0) *flag = 0;
        for (int P = 0; P < nt; ++P) {
            // ---- (1a) column P of the square to the LDS panel, ld 17
            for (int e = threadIdx.x; e < np * 16; e += NT) {
                const int row = e >> 4, col = e & 15;
                panel[row * 17 + col] = U[(size_t)row * ldu + 16 * P + col];
            }
            __syncthreads();
            lane_ids();
            // ---- (1b) the diagonal tile: factor and inverse in one wavefront
            if (w == (P & 7)) {
                T xr[4];
                const bool ok = diag_chol_inv16<T>(panel + 16 * P * 17, lane, xr);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = g + 4 * r;
                    if (row <= c) U[(size_t)(16 * P + row) * ldu + 16 * P + c] = xr[r];
                }
                if (!ok && lane == 0) *flag = 1;
            }
            __syncthreads();
            if (*flag) return false;
            // ---- (2) panel tiles R != P:  tile <- tile * X_PP^T
            lane_ids();
            for (int R = w; R < nt; R += kTiledWaves) {
                if (R == P) continue;
                v4 d = {0, 0, 0, 0};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int kq = 4 * q + g;
                    const T a = panel[(16 * R + c) * 17 + kq];
                    const T bx = panel[(16 * P + kq) * 17 + c];
                    d = Mfma<T>::mma(a, (kq <= c) ? bx : T(0), d);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * R + Mfma<T>::row(g, r);
                    panel[row * 17 + c] = d[r];
                    U[(size_t)row * ldu + 16 * P + c] = d[r];
                }
            }
            __syncthreads();
            if (P + 1 == nt) break;
            // ---- (3) rank-16 update of the tiles right of the panel
            const int cols = nt - P - 1;
            const int total = cols * (P + 1) + cols * (cols + 1) / 2;
            lane_ids();
            for (int u0 = w; u0 < total; u0 += 4 * kTiledWaves) {
                int R[4], C[4];
                v4 tl[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int u = u0 + b * kTiledWaves;
                    R[b] = -1; C[b] = 0;
                    if (u < total) trail_tile(P, u, R[b], C[b]);
                    v4 x = {0, 0, 0, 0};
                    if (R[b] >= 0) {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            x[r] = U[(size_t)(16 * R[b] + Mfma<T>::row(g, r)) * ldu + 16 * C[b] + c];
                    }
                    tl[b] = x;
                }
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    if (R[b] < 0) continue;
                    v4 d = {0, 0, 0, 0};
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int kq = 4 * q + g;
                        T a = panel[(16 * R[b] + c) * 17 + kq];
                        if (R[b] == P) a = (kq >= c) ? a : T(0);  // X rows of the panel: steps k >= r only
                        const T bb = panel[(16 * C[b] + c) * 17 + kq];
                        d = Mfma<T>::mma(a, bb, d);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = 16 * R[b] + Mfma<T>::row(g, r), col = 16 * C[b] + c;
                        const bool keep = !(R[b] == C[b] && row < col);  // X part of a diagonal tile
                        U[(size_t)row * ldu + col] = tl[b][r] - (keep ? d[r] : T(0));
                    }
                }
            }
            __syncthreads();
        }
        return true;
    }

    __device__ __forceinline__ bool schur() {
        lane_ids();
        for (int t = w; t < pt * nt; t += kTiledWaves) {
            const int K = t / nt, J = t - K * nt;
            const int arow = 16 * K + c, col = 16 * J + c;
            const int kend = min(n, 16 * J + 16);
            v4 d = {0, 0, 0, 0};
            for (int kb = 0; kb < kend; kb += 4) {
                const int k = kb + g;
                const bool ka = arow < p && k < n, kbv = k < n && col < n && k <= col;
                const T av = A[ka ? (size_t)arow * n + k : 0];
                const T bv = U[kbv ? (size_t)k * ldu + col : 0];
                d = Mfma<T>::mma(ka ? av : T(0), kbv ? bv : T(0), d);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * K + Mfma<T>::row(g, r);
                if (row < p && col < n) Wt[(size_t)row * n + col] = d[r];
            }
        }
        __syncthreads();
        lane_ids();
        for (int t = w; t < pt * pt; t += kTiledWaves) {
            const int K = t / pt, Lb = t - K * pt;
            const int ra = 16 * K + c, rb = 16 * Lb + c;
            v4 d = {0, 0, 0, 0};
            if (Lb <= K) {
                for (int kb = 0; kb < n; kb += 4) {
                    const int k = kb + g;
                    const bool va = ra < p && k < n, vb = rb < p && k < n;
                    const T av = Wt[va ? (size_t)ra * n + k : 0];
                    const T bv = Wt[vb ? (size_t)rb * n + k : 0];
                    d = Mfma<T>::mma(va ? av : T(0), vb ? bv : T(0), d);
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * K + Mfma<T>::row(g, r), col = 16 * Lb + c;
                if (row < p && col < p) S[row * lds + col] = (col <= row) ? d[r] : T(0);
            }
        }
        __syncthreads();
        return ::qpmi::chol_inv<T, NT>(S, lds, p, xdp);
    }

    __device__ __forceinline__ bool factor(const T *D) {
        form(D);
        if (!chol_inv()) return false;
        if constexpr (EQ) return schur();
        return true;
    }

    // factor(D), plus gz = G zr, gtl = G^T lr and gtw = G^T (lr + D rz),
    // rz = -(gz + sv - hv), from the chunks of G that the formation stages
    // (form() ends with a barrier)
    __device__ __forceinline__ bool factor_res(const T *D, const T *zr, const T *lr, const T *sv,
                                               const T *hv, T *gz, T *gtl, T *gtw, T *wsc) {
        static_assert(kFormResidual, "dense-G instantiations only");
        form<true>(D, zr, lr, sv, hv, gz, gtl, gtw, wsc);
        if (!chol_inv()) return false;
        if constexpr (EQ) return schur();
        return true;
    }

    // y = U^T f;  (equality rows) dnu = US US^T (Wt y - r4), y -= Wt^T dnu;  dz = U y
    __device__ __forceinline__ void solve(const T *f, const T *r4, T *dz, T *dnu) {
        ut_mv<T, NT>(U, ldu, n, f, yv);
        __syncthreads();
        if constexpr (EQ) {
            mv_rows<T, NT>(Wt, n, p, n, yv, pv1);
            __syncthreads();
            for (int k = threadIdx.x; k < p; k += NT) pv1[k] -= r4[k];
            __syncthreads();
            ut_mv<T, NT>(S, lds, p, pv1, pv2);
            __syncthreads();
            u_mv<T, NT>(S, lds, p, pv2, dnu);
            __syncthreads();
            for (int i = threadIdx.x; i < n; i += NT) {
                T acc = yv[i];
                for (int k = 0; k < p; ++k) acc -= Wt[(size_t)k * n + i] * dnu[k];
                yv[i] = acc;
            }
            __syncthreads();
        }
        u_mv<T, NT>(U, ldu, n, yv, dz);
        __syncthreads();
    }

    __device__ __forceinline__ void gt_mv(const T *v, T *out) {
        if (UNIT && unit) {
            ur.gt(v, out, n);
            return;
        }
        colsum_split<T, NT>(Gsrc, n, m, n, v, out, scratch);
    }
    __device__ __forceinline__ void g_mv(const T *x, T *out) {
        if (UNIT && unit) {
            ur.g(x, out, m);
            return;
        }
        mv_rows<T, NT>(Gsrc, n, m, n, x, out);
        __syncthreads();
    }
    __device__ __forceinline__ void qs_mv(const T *z, T *out) {
        colsum_split<T, NT>(Q, n, n, n, z, out, scratch);
        mv_rows<T, NT>(Q, n, n, n, z, xv);
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += NT) out[i] = T(0.5) * (out[i] + xv[i]);
        __syncthreads();
    }
    __device__ __forceinline__ bool finish(const T *D) {
        for (int k = threadIdx.x; k < m; k += NT) Dst[k] = D[k];
        if constexpr (EQ)
            if (s_lds)
                for (int e = threadIdx.x; e < p * p; e += NT) {
                    const int i = e / p, j = e - i * p;
                    US[e] = S[i * lds + j];
                }
        __syncthreads();
        return true;
    }
};

}  // namespace qpmi
