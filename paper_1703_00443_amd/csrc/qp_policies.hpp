// Factorization policies of the interior point driver (qp_ipm.hpp).
//
// GenericFactor: the factor lives in LDS (HL) or in the global state buffer;
//   plain per-element loops; any size; any number of equality rows.
// TiledFactor: the padded square of 16x16 tiles lives in the registers of
//   eight wavefronts in the MFMA accumulator layout; H = Qs + G^T D G is
//   formed with v_mfma_*_16x16x4 from G in LDS (resident, or staged in
//   chunks); the Cholesky factorisation and the triangular inverse are one
//   blocked sequence (diagonal tile chain, MFMA panel and trailing updates);
//   the Schur complement on A is two MFMA products and a small LDS
//   factorisation; the triangular solves are register matrix-vector products.
//   nz <= 128 (NTL = 8), or nz <= 256 in FP32 (NTL = 16).
#pragma once
#include "qp_ipm.hpp"

namespace qpmi {

__host__ __device__ inline int h_ld(int n) { return n | 1; }

// The padded square is an NTL x NTL grid of 16x16 tiles (nz <= 16 NTL, NTL =
// 8 or 16) spread over eight wavefronts: tile (I, J) lives in wavefront
// (I + J) mod 8, so every wavefront holds NTL / 8 tiles of each tile row and
// the lower triangle is shared evenly.  Register slot s of wavefront w holds
// tile (s / H, ((w - s / H) mod 8) + 8 (s mod H)), H = NTL / 8.
constexpr int kTiledWaves = 8;

// The lane id through an opaque move: index arithmetic derived from it is
// recomputed where it is used instead of being hoisted out of the Newton loop
// (hoisting it made the tiled kernel spill).
__device__ __forceinline__ int opaque_tid() {
    int t;
    asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
    return t;
}
constexpr int kTiledMaxN = 128;      // NTL = 8 (FP32 and FP64)
constexpr int kTiledBigMaxN = 256;   // NTL = 16 (FP32 only: 32 register tiles per wavefront)
constexpr int kGChunk = 32;          // rows of G staged per LDS chunk when G is not LDS-resident

// LDS regions of the policies (elements of T, after the driver's vectors).
template <bool HL>
struct GenericLayout {
    int xd, xdp, y, t1, t2, tq, scr, H, end;
    __host__ __device__ GenericLayout(int base, int n, int m, int p) {
        (void)m;
        int o = base;
        const int N = pad4(n), Pp = pad4(p);
        xd = o; o += N; xdp = o; o += Pp; y = o; o += N; t1 = o; o += Pp; t2 = o; o += Pp;
        tq = o; o += N; scr = o; o += 64 * kTiledWaves;
        o = (o + 15) & ~15;
        H = o;
        end = HL ? o + n * h_ld(n) : o;
    }
};

// GL: all of G resident in LDS (rows padded to a multiple of 4, ld 16 nt + 1);
// otherwise a staging buffer of kGChunk rows.  S: the Schur complement block
// (ld p | 1) with its pivot scratch and two p-vectors.
template <bool GL>
struct TiledLayout {
    int part, yv, xv, panel, scratch, flag, S, xdp, pv1, pv2, G, end;
    __host__ __device__ TiledLayout(int base, int n, int m, int p) {
        const int nt = (n + 15) / 16, np = 16 * nt;
        int o = base;
        part = o; o += nt * np; yv = o; o += np; xv = o; o += np;
        panel = o; o += np * 17;
        scratch = o; o += 64 * kTiledWaves;
        flag = o; o += 4;
        S = o; o += p > 0 ? p * h_ld(p) : 0;
        xdp = o; o += pad4(p); pv1 = o; o += pad4(p); pv2 = o; o += pad4(p);
        o = (o + 15) & ~15;
        G = o;
        end = o + (GL ? ((m + 3) & ~3) : kGChunk) * (np + 1);
    }
};

// ---------------------------------------------------------------------------
template <typename T, int NT, bool HL>
struct GenericFactor {
    static constexpr bool kRefineAlways = false;
    static constexpr bool kSolveGz = false;
    static constexpr bool kFormResidual = false;
    int n, m, p;
    const T *Q, *G, *A;
    T *H;
    int ldh;
    T *U_state, *Dst, *Wt, *US;
    T *xd, *xdp, *y, *t1, *t2, *tq, *scr;

    __device__ __forceinline__ GenericFactor(const Prob<T> &P, T *sm, int base) {
        n = P.n; m = P.m; p = P.p;
        Q = P.Q; G = P.G; A = P.A;
        const StateLayout SL = state_layout(sizeof(T), n, m, p);
        U_state = (T *)(P.state + SL.off_U);
        Dst = (T *)(P.state + SL.off_D);
        Wt = (T *)(P.state + SL.off_Wt);
        US = (T *)(P.state + SL.off_US);
        const GenericLayout<HL> L(base, n, m, p);
        xd = sm + L.xd; xdp = sm + L.xdp; y = sm + L.y; t1 = sm + L.t1; t2 = sm + L.t2;
        tq = sm + L.tq; scr = sm + L.scr;
        if (HL) { H = sm + L.H; ldh = h_ld(n); } else { H = U_state; ldh = u_ld(n); }
    }
    __device__ __forceinline__ void prepare() {}
    __device__ __forceinline__ bool factor(const T *D) {
        form_h<T, NT>(Q, G, D, n, m, H, ldh);
        bool ok = chol_inv<T, NT>(H, ldh, n, xd);
        if (ok && p > 0) ok = schur<T, NT>(H, ldh, A, n, p, Wt, US, xdp);
        return ok;
    }
    __device__ __forceinline__ void solve(const T *f, const T *r4, T *dz, T *dnu) {
        kkt_solve<T, NT>(H, ldh, Wt, US, n, p, f, r4, y, t1, t2, dz, dnu, scr);
    }
    __device__ __forceinline__ void gt_mv(const T *v, T *out) {
        mv_cols<T, NT>(G, n, m, n, v, out);
        __syncthreads();
    }
    __device__ __forceinline__ void g_mv(const T *x, T *out) {
        mv_rows<T, NT>(G, n, m, n, x, out);
        __syncthreads();
    }
    __device__ __forceinline__ void qs_mv(const T *z, T *out) {
        mv_rows<T, NT>(Q, n, n, n, z, tq);
        mv_cols<T, NT>(Q, n, n, n, z, out);
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += NT) out[i] = T(0.5) * (out[i] + tq[i]);
        __syncthreads();
    }
    __device__ __forceinline__ bool finish(const T *D) {
        if (HL)
            for (int e = threadIdx.x; e < n * n; e += NT) {
                const int i = e / n, j = e - i * n;
                U_state[(size_t)i * u_ld(n) + j] = H[(size_t)i * ldh + j];
            }
        for (int k = threadIdx.x; k < m; k += NT) Dst[k] = D[k];
        __syncthreads();
        return true;
    }
};

// ---------------------------------------------------------------------------
template <typename T>
struct Mfma;
// Operand layouts of v_mfma_*_16x16x4 (lane l = 16 g + c, g = l >> 4, c = l & 15):
// A[i][k] from lane (k, i), B[k][j] from lane (k, j); the four accumulator
// values of lane l hold column c and rows row(g, r), r = 0..3.  The row map
// differs between the f64 (g + 4 r) and the f32 (4 g + r) instructions.
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __host__ __device__ static constexpr int row(int g, int r) { return g + 4 * r; }
    __device__ static __forceinline__ v4 mma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __host__ __device__ static constexpr int row(int g, int r) { return 4 * g + r; }
    __device__ static __forceinline__ v4 mma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};



// ---------------------------------------------------------------------------
// Cholesky of a 16x16 SPD block fused with the inverse of its factor, in one
// wavefront.  Register exchange only: DPP row_newbcast (lane k of every row of
// 16 lanes) and the gfx950 permlane16/32 swaps (one row of 16 lanes to all four).
//
// Chain layout (both element types): lane 16 g + c holds column c, rows
// g + 4 r (r = 0..3) of
//   a: the symmetric trailing block, A[row][c] (entries with row or column
//      below the current step may hold anything: they are never read again),
//   x: X^T, X = L^{-1}, seeded with the unit diagonal and exact zeros below it.
// Step k (A^(k) the trailing block, v = A^(k)[k][c], p = A^(k)[k][k]):
//   a[r] -= A^(k)[row][k] v / p                     (Cholesky trailing update)
//   x[r]  = c == k ? x[r] / sqrt(p)                 (column k of X^T final)
//         : c >  k ? x[r] - X^T[row][k] v / p       (forward substitution)
//         :          x[r]                           (finished columns)
// Only registers that can hold a row > k (a) or a row <= k (x) are touched.
template <typename T>
__device__ __forceinline__ T chain_rsqrt(T x) {
    if constexpr (sizeof(T) == 8) {
        const double y = __builtin_amdgcn_rsq(x);  // hardware estimate + one Newton step
        return y * (1.5 - 0.5 * x * y * y);
    } else {
        const float y = __builtin_amdgcn_rsqf(x);
        return y * (1.5f - 0.5f * x * y * y);
    }
}
template <int SRC>
__device__ __forceinline__ unsigned row_bcast16(unsigned v) {  // lane SRC of each row of 16
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x150 + SRC, 0xf, 0xf, false);
}
template <int SG>
__device__ __forceinline__ unsigned group_bcast(unsigned v) {  // row SG of 16 lanes to all rows
    const auto a = __builtin_amdgcn_permlane16_swap(v, v, false, false);  // rows {0,0,2,2} / {1,1,3,3}
    const unsigned y = (SG & 1) ? a[1] : a[0];
    const auto b = __builtin_amdgcn_permlane32_swap(y, y, false, false);  // rows {0,1,0,1} / {2,3,2,3}
    return (SG & 2) ? b[1] : b[0];
}
template <int SRC, typename T>
__device__ __forceinline__ T row_bcast16(T v) {
    if constexpr (sizeof(T) == 8) {
        // one 64-bit DPP move (row_newbcast is a DPP64 control on gfx950)
        return __builtin_amdgcn_update_dpp(T(0), v, 0x150 + SRC, 0xf, 0xf, false);
    } else {
        return __builtin_bit_cast(T, row_bcast16<SRC>(__builtin_bit_cast(unsigned, v)));
    }
}
template <int SG, typename T>
__device__ __forceinline__ T group_bcast(T v) {
    if constexpr (sizeof(T) == 8) {
        const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
        const unsigned lo = group_bcast<SG>((unsigned)u), hi = group_bcast<SG>((unsigned)(u >> 32));
        return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
    } else {
        return __builtin_bit_cast(T, group_bcast<SG>(__builtin_bit_cast(unsigned, v)));
    }
}
template <typename T, int K>
__device__ __forceinline__ void chain_steps(T *a, T *x, int c, bool &bad) {
    if constexpr (K < 16) {
        const T v = group_bcast<(K & 3)>(a[K >> 2]);  // A[K][c]
        const T p = row_bcast16<K>(v);                 // A[K][K]
        bad |= !(p > T(0)) || !isfinite(p);
        const T inv = chain_rsqrt(p);
        const T wc = v * (inv * inv);
        const T wcm = (c > K) ? wc : T(0);
        const T sc = (c == K) ? inv : T(1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (4 * r + 3 > K) a[r] = a[r] - row_bcast16<K>(a[r]) * wc;
            if (4 * r <= K) x[r] = x[r] * sc - row_bcast16<K>(x[r]) * wcm;
        }
        chain_steps<T, K + 1>(a, x, c, bad);
    }
}
// `pan`: the block inside an LDS panel (ld 17) whose lower triangle (incl.
// diagonal) holds the SPD block.  On return x[r] holds X^T[g + 4 r][c] (valid
// for g + 4 r <= c) and the upper triangle (incl. diagonal) of `pan` holds X^T
// once the caller has waited for the stores.  Returns false (uniformly) on a
// non-positive or non-finite pivot.
template <typename T>
__device__ __forceinline__ bool diag_chol_inv16(T *pan, int lane, T *x) {
    const int g = lane >> 4, c = lane & 15;
    T a[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = g + 4 * r;
        a[r] = pan[(row > c ? row : c) * 17 + (row > c ? c : row)];
        x[r] = (row == c) ? T(1) : T(0);
    }
    // the loads complete before any lane's later stores to the panel
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    bool bad = false;
    chain_steps<T, 0>(a, x, c, bad);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = g + 4 * r;
        if (row <= c) pan[row * 17 + c] = x[r];
    }
    return !bad;
}

// Rows of G that are signed unit vectors (QP_FLAG_G_UNIT_ROWS): row k has its
// one entry sign[k] in column col[k]; the rows of column j, in order, are
// row[off[j] .. off[j+1]).  The arrays take 3 nineq + nz + 1 elements of T
// from the region given to place().
template <typename T, int NT>
struct UnitRows {
    T *sign;
    int *col, *off, *row;

    __host__ __device__ static constexpr int elems(int n, int m) { return 3 * m + n + 1; }
    __device__ __forceinline__ void place(T *region, int n, int m) {
        sign = region;
        col = reinterpret_cast<int *>(region + m);
        off = col + m;
        row = off + n + 1;
    }
    // Finds each row's one entry; false (uniformly) if some row is not a signed
    // unit vector, true once the per-column row lists are built.
    __device__ __forceinline__ bool detect(const T *G, int n, int m, T *red) {
        T bad = 0, d0 = 0, d1 = 0;
        for (int k = threadIdx.x; k < m; k += NT) {
            int cj = 0, cnt = 0;
            T val = 0;
            for (int j = 0; j < n; ++j) {
                const T v = G[(size_t)k * n + j];
                if (v != T(0)) { ++cnt; cj = j; val = v; }
            }
            if (cnt != 1 || !(val == T(1) || val == T(-1))) bad = 1;
            col[k] = cj;
            sign[k] = val;
        }
        block_reduce3<T, NT>(bad, d0, d1, red);
        if (bad != T(0)) return false;
        // rows per column, offsets (one thread), rows in order
        for (int j = threadIdx.x; j < n; j += NT) {
            int cnt = 0;
            for (int k = 0; k < m; ++k) cnt += col[k] == j;
            off[j + 1] = cnt;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            off[0] = 0;
            for (int j = 0; j < n; ++j) off[j + 1] += off[j];
        }
        __syncthreads();
        for (int j = threadIdx.x; j < n; j += NT) {
            int o = off[j];
            for (int k = 0; k < m; ++k)
                if (col[k] == j) row[o++] = k;
        }
        __syncthreads();
        return true;
    }
    // out[j] = sum of D over the rows of column j (the diagonal G^T D G), in row order
    __device__ __forceinline__ void diag(const T *D, T *out, int n) const {
        for (int j = threadIdx.x; j < n; j += NT) {
            T a = 0;
            for (int t = off[j]; t < off[j + 1]; ++t) a += D[row[t]];
            out[j] = a;
        }
        __syncthreads();
    }
    // out = G^T v
    __device__ __forceinline__ void gt(const T *v, T *out, int n) const {
        for (int j = threadIdx.x; j < n; j += NT) {
            T a = 0;
            for (int t = off[j]; t < off[j + 1]; ++t) {
                const int k = row[t];
                a += sign[k] * v[k];
            }
            out[j] = a;
        }
        __syncthreads();
    }
    // out = G x
    __device__ __forceinline__ void g(const T *x, T *out, int m) const {
        for (int k = threadIdx.x; k < m; k += NT) out[k] = sign[k] * x[col[k]];
        __syncthreads();
    }
};

// Which tiles a wavefront holds (see the grid comment above).
template <int NTL>
struct TileMap {
    static constexpr int H = NTL / 8;    // tiles per tile row in one wavefront
    static constexpr int NS = NTL * H;   // register slots per wavefront
    __device__ static __forceinline__ int row(int s) { return s / H; }
    __device__ static __forceinline__ int col(int w, int s) { return ((w - s / H) & 7) + 8 * (s % H); }
    __device__ static __forceinline__ int diag_slot(int P) { return P * H + (P >> 3); }
};

// EQ: the problem has equality rows (Schur complement on A).  Instantiated
// separately so that the no-equality solve carries none of that code.
// UNIT: the call set QP_FLAG_G_UNIT_ROWS; a separate instantiation, so that the
// dense kernels carry none of the unit-row code.
template <typename T, bool GL, int NTL, bool EQ, bool UNIT = false>
struct TiledFactor {
    static constexpr int NT = 64 * kTiledWaves;
    static constexpr bool kRefineAlways = false;
    static constexpr bool kSolveGz = false;
    // G streamed in chunks: the residual's G z and G^T lam from the staged rows
    // (not in the unit-row instantiations, whose products are gathers)
    static constexpr bool kFormResidual = !GL && !UNIT;
    static constexpr int NS = TileMap<NTL>::NS;
    using v4 = typename Mfma<T>::v4;
    int n, m, p, nt, np, pt, ldg, lds, ldu;
    const T *Q, *Gsrc, *A;
    const T *G;  // LDS copy (GL) or the staging chunk
    T *Ust, *Dst, *Wt, *US;  // state: U (row-major, ld n), D, Wt (p x n), US (p x p)
    T *part, *yv, *xv, *panel, *scratch, *S, *xdp, *pv1, *pv2;
    int *flag;
    int w, lane, g, c;
    // rows of G that are signed unit vectors (QP_FLAG_G_UNIT_ROWS), in the G region
    bool unit;
    UnitRows<T, NT> ur;
    v4 sq[NS];

    __device__ __forceinline__ int trow(int s) const { return TileMap<NTL>::row(s); }
    __device__ __forceinline__ int tcol(int s) const { return TileMap<NTL>::col(w, s); }
    __device__ __forceinline__ void lane_ids() {
        const int t = opaque_tid();
        lane = t & 63; g = lane >> 4; c = lane & 15;
        w = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform: tile skips are scalar branches
    }

    __device__ __forceinline__ TiledFactor(const Prob<T> &P, T *sm, int base) {
        n = P.n; m = P.m; p = P.p;
        nt = (n + 15) / 16; np = 16 * nt; pt = (p + 15) / 16;
        Q = P.Q; Gsrc = P.G; A = P.A;
        const StateLayout SL = state_layout(sizeof(T), n, m, p);
        Ust = (T *)(P.state + SL.off_U);
        Dst = (T *)(P.state + SL.off_D);
        Wt = (T *)(P.state + SL.off_Wt);
        US = (T *)(P.state + SL.off_US);
        const TiledLayout<GL> L(base, n, m, p);
        part = sm + L.part; yv = sm + L.yv; xv = sm + L.xv;
        panel = sm + L.panel; scratch = sm + L.scratch;
        S = sm + L.S; xdp = sm + L.xdp; pv1 = sm + L.pv1; pv2 = sm + L.pv2;
        flag = reinterpret_cast<int *>(sm + L.flag);
        G = sm + L.G; ldg = np + 1; lds = h_ld(p); ldu = u_ld(n);
        lane = threadIdx.x & 63; w = threadIdx.x >> 6; g = lane >> 4; c = lane & 15;
        const int gcap = (GL ? ((m + 3) & ~3) : kGChunk) * (np + 1);
        unit = UNIT && (P.flags & QP_FLAG_G_UNIT_ROWS) != 0 && m > 0 &&
               UnitRows<T, NT>::elems(n, m) <= gcap;
        ur.place(sm + L.G, n, m);
    }

    // Re-aims the object at an n_ x n_ factor with m_ rows of G and p_ equality
    // rows whose LDS regions start at `base` (the problem's inputs and state
    // pointers, and ldu, stay as constructed).  One object can then factor
    // matrices of two sizes in turn with the same register tiles.
    __device__ __forceinline__ void retarget(int n_, int m_, int p_, T *sm, int base) {
        n = n_; m = m_; p = p_;
        nt = (n + 15) / 16; np = 16 * nt; pt = (p + 15) / 16;
        const TiledLayout<GL> L(base, n, m, p);
        part = sm + L.part; yv = sm + L.yv; xv = sm + L.xv;
        panel = sm + L.panel; scratch = sm + L.scratch;
        S = sm + L.S; xdp = sm + L.xdp; pv1 = sm + L.pv1; pv2 = sm + L.pv2;
        flag = reinterpret_cast<int *>(sm + L.flag);
        G = sm + L.G; ldg = np + 1; lds = h_ld(p);
    }

    // Rows [k0, k0 + rows) of G into the LDS buffer, zero-padded to whole MFMA
    // steps (rows to a multiple of 4, columns to 16 nt).
    __device__ __forceinline__ void stage_g(int k0, int rows) {
        const int rp = (rows + 3) & ~3;
        T *dst = const_cast<T *>(G);
        for (int e = threadIdx.x; e < rp * np; e += NT) {
            const int k = e / np, i = e - k * np;
            dst[k * ldg + i] = (k < rows && i < n) ? Gsrc[(size_t)(k0 + k) * n + i] : T(0);
        }
    }

    // Without equality rows the U region of the state is free until finish():
    // it holds Qs = (Q + Q^T) / 2 (row-major, ld nz) for coalesced single
    // loads in form() and qs_mv().  With equality rows the Schur step stores U there every
    // factorization, and Qs is taken from Q itself.
    __device__ __forceinline__ void prepare() {
        // any row that is not a signed unit vector sends the problem down the dense path
        if (UNIT && unit) unit = ur.detect(Gsrc, n, m, scratch);
        if (!EQ)
            for (int e = threadIdx.x; e < n * n; e += NT) {
                const int i = e / n, j = e - i * n;
                Ust[e] = T(0.5) * (Q[(size_t)i * n + j] + Q[(size_t)j * n + i]);
            }
        if (GL && !(UNIT && unit)) stage_g(0, m);
        __syncthreads();
    }

    // H = Qs + G^T D G into the register tiles (lower tiles), X region zero.
    // Accumulators start from Qs = (Q + Q^T) / 2 (identity on the padding); the
    // k loop runs outside the tile loop so that the MFMAs of the tiles of a
    // wavefront are independent and overlap their operand loads.
    // RES (G streamed in chunks): each staged chunk of rows also gives its
    // entries of gz = G zr (16 lanes per row, as mv_rows), the row weights
    // wsc = lr + D rz with rz = -(gz + sv - hv), and its terms of gtl = G^T lr
    // and gtw = G^T wsc (one thread per column, n <= NT), so that neither the
    // residual of the iterate nor the affine right-hand side needs a pass of
    // its own over G.
    template <bool RES = false>
    __device__ __forceinline__ void form(const T *D, const T *zr = nullptr, const T *lr = nullptr,
                                         const T *sv = nullptr, const T *hv = nullptr,
                                         T *gz = nullptr, T *gtl = nullptr, T *gtw = nullptr,
                                         T *wsc = nullptr) {
        static_assert(!RES || (!GL && 16 * NTL <= NT), "column sums take one thread per column");
        T cs0 = 0, cs1 = 0, cs2 = 0, cs3 = 0;  // column threadIdx.x of G^T lr, rows k mod 4
        T cw0 = 0, cw1 = 0, cw2 = 0, cw3 = 0;  // column threadIdx.x of G^T wsc
        if (UNIT && unit) ur.diag(D, xv, n);  // G^T D G is diagonal
        lane_ids();
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int I = trow(s), J = tcol(s);
            v4 acc = {0, 0, 0, 0};
            if (I < nt && J < nt && I >= J) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * I + Mfma<T>::row(g, r), col = 16 * J + c;
                    const bool in = row < n && col < n;
                    T qs;
                    if (!EQ) {
                        qs = Ust[in ? (size_t)row * n + col : 0];
                    } else {
                        const T qa = Q[in ? (size_t)row * n + col : 0];
                        const T qb = Q[in ? (size_t)col * n + row : 0];
                        qs = T(0.5) * (qa + qb);
                    }
                    if (UNIT && unit && in && row == col) qs += xv[row];
                    acc[r] = in ? qs : (row == col ? T(1) : T(0));
                }
            }
            sq[s] = acc;
        }
        for (int k0 = 0; k0 < ((UNIT && unit) ? 0 : m); k0 += (GL ? m : kGChunk)) {
            const int rows = GL ? m : min(kGChunk, m - k0);
            if (!GL) {
                __syncthreads();  // previous chunk consumed
                stage_g(k0, rows);
                __syncthreads();
                lane_ids();
            }
            if constexpr (RES) chunk_rows_res<T, NT>(G, ldg, k0, rows, n, zr, lr, D, sv, hv, gz, wsc);
            for (int kb = 0; kb < rows; kb += 4) {
                const int k = kb + g;
                const T *Gk = G + (size_t)k * ldg;
                const int kg = k0 + k;
                const T dk = D[kg < m ? kg : m - 1] * T(kg < m ? 1 : 0);
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const int I = trow(s), J = tcol(s);
                    if (I >= nt || J >= nt || I < J) continue;
                    sq[s] = Mfma<T>::mma(Gk[16 * I + c], dk * Gk[16 * J + c], sq[s]);
                }
            }
            if constexpr (RES) {
                __syncthreads();  // the chunk's row weights
                const int i = threadIdx.x;
                if (i < n) {
                    int k = 0;
                    for (; k + 3 < rows; k += 4) {
                        const T g0 = G[(size_t)k * ldg + i], g1 = G[(size_t)(k + 1) * ldg + i];
                        const T g2 = G[(size_t)(k + 2) * ldg + i], g3 = G[(size_t)(k + 3) * ldg + i];
                        cs0 += g0 * lr[k0 + k];
                        cs1 += g1 * lr[k0 + k + 1];
                        cs2 += g2 * lr[k0 + k + 2];
                        cs3 += g3 * lr[k0 + k + 3];
                        cw0 += g0 * wsc[k0 + k];
                        cw1 += g1 * wsc[k0 + k + 1];
                        cw2 += g2 * wsc[k0 + k + 2];
                        cw3 += g3 * wsc[k0 + k + 3];
                    }
                    for (; k < rows; ++k) {
                        const T g0 = G[(size_t)k * ldg + i];
                        cs0 += g0 * lr[k0 + k];
                        cw0 += g0 * wsc[k0 + k];
                    }
                }
            }
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (trow(s) >= nt || tcol(s) != trow(s)) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (Mfma<T>::row(g, r) < c) sq[s][r] = T(0);  // X part of the diagonal tile
        }
        if constexpr (RES)
            if ((int)threadIdx.x < n) {
                gtl[threadIdx.x] = (cs0 + cs1) + (cs2 + cs3);
                gtw[threadIdx.x] = (cw0 + cw1) + (cw2 + cw3);
            }
    }

    // The register tiles from a symmetric n x n matrix whose strict lower
    // triangle is that of C (row-major, ld ldc) and whose diagonal is diag: the
    // same tiles form() leaves, with no contraction (identity on the padding,
    // the X part of the diagonal tiles zero).
    __device__ __forceinline__ void seed(const T *C, int ldc, const T *diag) {
        lane_ids();
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int I = trow(s), J = tcol(s);
            v4 acc = {0, 0, 0, 0};
            if (I < nt && J < nt && I >= J) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * I + Mfma<T>::row(g, r), col = 16 * J + c;
                    const bool in = row < n && col < n, lo = in && col < row;
                    const T v = C[lo ? (size_t)row * ldc + col : 0];
                    const T d = diag[in && row == col ? row : 0];
                    acc[r] = lo ? v : (in && row == col ? d : (!in && row == col ? T(1) : T(0)));
                }
            }
            sq[s] = acc;
        }
    }

    // Fused Cholesky + inverse.  Step k is the rank-1 update
    //     S[r][c] -= s_r s_c   where r >= c > k (trailing block of L)
    //                          or    r <= k < c (rows of X = L^{-1})
    // with s = column k of S scaled by 1/sqrt(S[k][k]) and s_k = 1/sqrt(S[k][k]);
    // column k is then replaced by s.  After all steps the strict lower triangle
    // holds L, the diagonal 1/L[k][k] and the strict upper triangle X^T, so the
    // upper triangle (incl. diagonal) is U = L^{-T}.
    //
    // Blocked by 16-column panels P:
    //  (1) the diagonal tile (P,P) runs the 16 steps alone, inside the one
    //      wavefront that holds it (wave-local LDS exchange, no workgroup
    //      barrier): lower part -> L_PP, upper part -> X_PP^T;
    //  (2) every other tile of the panel column becomes  tile * X_PP^T
    //      (for rows below the diagonal block this is L_RP = H_RP L_PP^{-T},
    //      for rows above it the block forward substitution X_PR = X_PP A_PR);
    //  (3) the columns right of the panel get the rank-16 update of the 16
    //      steps as one MFMA product per tile, masked where a step's condition
    //      excludes it.
    __device__ __forceinline__ bool chol_inv() {
        if (threadIdx.x == 0) *flag = 0;
        __syncthreads();
        for (int P = 0; P < nt; ++P) {
            lane_ids();
            const int wd = (2 * P) & 7;  // owner of the diagonal tile (P,P)
            const int sd = TileMap<NTL>::diag_slot(P);
            // ---- (1a) old panel tiles (R != P) to LDS, ld 17
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int R = trow(s);
                if (R >= nt || R == P || tcol(s) != P) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) panel[(16 * R + Mfma<T>::row(g, r)) * 17 + c] = sq[s][r];
            }
            // ---- (1b) the diagonal tile: factor and inverse in the one wavefront that holds it
            if (w == wd) {
                v4 t = {0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < NS; ++s)
                    if (s == sd) t = sq[s];
                T *pan = panel + 16 * P * 17;
#pragma unroll
                for (int r = 0; r < 4; ++r) pan[Mfma<T>::row(g, r) * 17 + c] = t[r];
                // wave-local LDS exchange: the stores must land before other lanes load
                __builtin_amdgcn_s_waitcnt(0);
                __builtin_amdgcn_wave_barrier();
                T xr[4];
                const bool ok = diag_chol_inv16<T>(pan, lane, xr);
                if constexpr (sizeof(T) == 8) {
                    // the f64 accumulator layout is the chain layout (row g + 4 r)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (Mfma<T>::row(g, r) <= c) t[r] = xr[r];
                } else {
                    __builtin_amdgcn_s_waitcnt(0);
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = Mfma<T>::row(g, r);
                        if (row <= c) t[r] = pan[row * 17 + c];  // X_PP^T (upper incl. diagonal)
                    }
                }
#pragma unroll
                for (int s = 0; s < NS; ++s)
                    if (s == sd) sq[s] = t;
                if (!ok && lane == 0) *flag = 1;
            }
            __syncthreads();
            if (*flag) return false;
            // ---- (2) panel tiles R != P:  tile <- tile * X_PP^T
            lane_ids();
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int R = trow(s);
                if (R >= nt || R == P || tcol(s) != P) continue;
                v4 d = {0, 0, 0, 0};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int kq = 4 * q + g;
                    const T a = panel[(16 * R + c) * 17 + kq];
                    // X_PP^T[kq][c] sits in the upper triangle (incl. diagonal) of tile (P,P)
                    const T bx = panel[(16 * P + kq) * 17 + c];
                    const T b = (kq <= c) ? bx : T(0);
                    d = Mfma<T>::mma(a, b, d);
                }
                sq[s] = d;
#pragma unroll
                for (int r = 0; r < 4; ++r) panel[(16 * R + Mfma<T>::row(g, r)) * 17 + c] = d[r];
            }
            __syncthreads();
            if (P + 1 == nt) break;
            // ---- (3) rank-16 update of the tiles right of the panel
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int R = trow(s), C = tcol(s);
                if (R >= nt || C >= nt || C <= P) continue;
                if (R > P && R < C) continue;  // rows of X below the panel: no step applies
                v4 d = {0, 0, 0, 0};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int kq = 4 * q + g;
                    T a = panel[(16 * R + c) * 17 + kq];
                    if (R == P) a = (kq >= c) ? a : T(0);  // X rows of the panel: steps k >= r only
                    const T b = panel[(16 * C + c) * 17 + kq];
                    d = Mfma<T>::mma(a, b, d);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * R + Mfma<T>::row(g, r), col = 16 * C + c;
                    const bool keep = !(R == C && row < col);  // X part of a diagonal tile: untouched
                    sq[s][r] -= keep ? d[r] : T(0);
                }
            }
            __syncthreads();
        }
        return true;
    }

    // U (upper register tiles, incl. diagonal) to the state, row-major ld n.
    __device__ __forceinline__ void store_u() {
        lane_ids();
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int I = trow(s), J = tcol(s);
            if (I >= nt || J >= nt || I > J) continue;
            const int col = 16 * J + c;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * I + Mfma<T>::row(g, r);
                if (row <= col && row < n && col < n) Ust[(size_t)row * ldu + col] = sq[s][r];
            }
        }
    }

    // Schur complement on A (neq > 0): Wt = A U (MFMA tiles over the stored
    // U, a p x n product), S = Wt Wt^T (lower triangle, LDS), S = LS LS^T with
    // its inverse factor in place.
    __device__ __forceinline__ bool schur() {
        store_u();
        __syncthreads();
        lane_ids();
        for (int t = w; t < pt * nt; t += kTiledWaves) {
            const int K = t / nt, J = t - K * nt;
            const int arow = 16 * K + c, col = 16 * J + c;
            const int kend = min(n, 16 * J + 16);  // U[k][col] = 0 for k > col
            v4 d = {0, 0, 0, 0};
            for (int kb = 0; kb < kend; kb += 4) {
                const int k = kb + g;
                const bool ka = arow < p && k < n, kbv = k < n && col < n && k <= col;
                const T av = A[ka ? (size_t)arow * n + k : 0];
                const T bv = Ust[kbv ? (size_t)k * ldu + col : 0];
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
    // (visible to every thread when it returns: chol_inv starts with a barrier)
    __device__ __forceinline__ bool factor_res(const T *D, const T *zr, const T *lr, const T *sv,
                                               const T *hv, T *gz, T *gtl, T *gtw, T *wsc) {
        static_assert(kFormResidual, "dense-G instantiations only");
        form<true>(D, zr, lr, sv, hv, gz, gtl, gtw, wsc);
        if (!chol_inv()) return false;
        if constexpr (EQ) return schur();
        return true;
    }

    // [H A^T; A 0][dz; dnu] = [f; r4] with U = L^{-T} in the upper register
    // tiles:  y = U^T f;  (p > 0) dnu = US US^T (Wt y - r4), y -= Wt^T dnu;
    // dz = U y.
    __device__ __forceinline__ void solve(const T *f, const T *r4, T *dz, T *dnu) {
        lane_ids();
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int I = trow(s), J = tcol(s);
            if (I >= nt || J >= nt) continue;
            if (I > J) continue;
            const int col = 16 * J + c;
            T acc = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * I + Mfma<T>::row(g, r);
                const T fr = f[row < n ? row : 0];
                acc += (row <= col && row < n) ? sq[s][r] * fr : T(0);
            }
            {
                T a, b;
                row_swap<false>(acc, a, b);  // rows 0+1, 2+3
                row_swap<true>(a + b, a, b); // + the other half
                acc = a + b;
            }
            if (g == 0) part[I * np + col] = acc;
        }
        __syncthreads();
        for (int col = threadIdx.x; col < np; col += NT) {
            T acc = 0;
            for (int I = 0; I <= (col >> 4); ++I) acc += part[I * np + col];
            yv[col] = acc;
        }
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
        lane_ids();
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int I = trow(s), J = tcol(s);
            if (I >= nt || J >= nt) continue;
            if (I > J) continue;
            const int col = 16 * J + c;
            const T yc = yv[col];
            T v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * I + Mfma<T>::row(g, r);
                v[r] = (col >= row) ? sq[s][r] * yc : T(0);
            }
            // reduce-scatter over the 16 lanes of the row group: partners
            // c <-> 15 - c (row_mirror) and c <-> 7 - c within each 8
            // (row_half_mirror) flip bits 3 and 2 of c, then the quad sum
            const bool hi = (c & 8) != 0;
            T k0 = hi ? v[2] : v[0], k1 = hi ? v[3] : v[1];
            k0 += dpp_move<0x140>(hi ? v[0] : v[2]);
            k1 += dpp_move<0x140>(hi ? v[1] : v[3]);
            const bool h2 = (c & 4) != 0;
            T keep = h2 ? k1 : k0;
            keep += dpp_move<0x141>(h2 ? k0 : k1);
            keep += dpp_move<0x4E>(keep);
            keep += dpp_move<0xB1>(keep);
            if ((c & 3) == 0) part[J * np + 16 * I + Mfma<T>::row(g, (hi ? 2 : 0) + (h2 ? 1 : 0))] = keep;
        }
        __syncthreads();
        for (int row = threadIdx.x; row < n; row += NT) {
            T acc = 0;
            for (int J = row >> 4; J < nt; ++J) acc += part[J * np + row];
            dz[row] = acc;
        }
        __syncthreads();
    }
    __device__ __forceinline__ void colsum(const T *M, int ld, int rows, int cols, const T *v, T *out) {
        colsum_split<T, NT>(M, ld, rows, cols, v, out, scratch);
    }
    __device__ __forceinline__ void rowdot(const T *M, int ld, int rows, int cols, const T *x, T *out) {
        rowdot_split<T, NT>(M, ld, rows, cols, x, out, scratch);
    }
    __device__ __forceinline__ void gt_mv(const T *v, T *out) {
        if (UNIT && unit) {
            ur.gt(v, out, n);
            return;
        }
        if (GL) colsum(G, ldg, m, n, v, out);
        else colsum(Gsrc, n, m, n, v, out);
    }
    __device__ __forceinline__ void g_mv(const T *x, T *out) {
        if (UNIT && unit) {
            ur.g(x, out, m);
            return;
        }
        if (GL) {
            rowdot(G, ldg, m, n, x, out);
        } else {
            mv_rows<T, NT>(Gsrc, n, m, n, x, out);
            __syncthreads();
        }
    }
    // Qs z: column sums over the staged Qs (no equality rows), else
    // (Q z + Q^T z) / 2 from column sums and row dots over coalesced rows of Q
    __device__ __forceinline__ void qs_mv(const T *z, T *out) {
        if constexpr (!EQ) {
            colsum(Ust, n, n, n, z, out);
            return;
        }
        colsum(Q, n, n, n, z, out);
        mv_rows<T, NT>(Q, n, n, n, z, xv);
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += NT) out[i] = T(0.5) * (out[i] + xv[i]);
        __syncthreads();
    }
    __device__ __forceinline__ bool finish(const T *D) {
        store_u();
        for (int k = threadIdx.x; k < m; k += NT) Dst[k] = D[k];
        if constexpr (EQ)
            for (int e = threadIdx.x; e < p * p; e += NT) {
                const int i = e / p, j = e - i * p;
                US[e] = S[i * lds + j];
            }
        __syncthreads();
        return true;
    }
};

}  // namespace qpmi
