// Device building blocks shared by the forward and backward kernels.
//
// Execution model: one workgroup of NT threads (NT/64 wavefronts of 64 lanes)
// owns one QP at a time.  Every routine below is called by all threads of the
// workgroup in uniform control flow and ends with a workgroup barrier when its
// results are read by other threads.
//
// The reduced KKT system.  The symmetrised Newton system of Section 3.1
// (second block row of K scaled by D(1/s)) has unknowns (dz, ds, dlam, dnu)
// and the matrix
//     [ Qs  0  G^T  A^T ]
//     [ 0   D  I    0   ]      D = D(lambda / s)
//     [ G   I  0    0   ]
//     [ A   0  0    0   ]
// Eliminating ds and dlam leaves [H A^T; A 0] with H = Qs + G^T D G, which
// is factored as H = L L^T; the Schur complement S = A H^{-1} A^T = Wt Wt^T,
// Wt = (L^{-1} A^T)^T, is factored as LS LS^T.  The kernels keep the inverse
// factors U = L^{-T} and US = LS^{-T} (upper triangular), so that every
// solve is a pair of triangular matrix-vector products.
#pragma once
#include <hip/hip_runtime.h>

#include "qp_internal.h"

namespace qpmi {

__host__ __device__ constexpr int pad4(int x) { return (x + 3) & ~3; }

// Wavefront reductions by register exchange only (no LDS): DPP quad_perm
// (lane ^ 1, lane ^ 2), DPP row_half_mirror and row_mirror (within rows of 16),
// then the gfx950 permlane16/32 swaps across the four rows.  Every step
// combines a value with a partner whose own step combines the same two values,
// so all 64 lanes end with bit-identical results; the order is fixed.
template <int CTRL>
__device__ __forceinline__ unsigned dpp_u32(unsigned v) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, true);
}
template <int CTRL, typename T>
__device__ __forceinline__ T dpp_move(T v) {
    if constexpr (sizeof(T) == 8) {
        const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
        const unsigned lo = dpp_u32<CTRL>((unsigned)u), hi = dpp_u32<CTRL>((unsigned)(u >> 32));
        return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
    } else {
        return __builtin_bit_cast(T, dpp_u32<CTRL>(__builtin_bit_cast(unsigned, v)));
    }
}
// partner values across rows: {own row pair's even row, odd row} (permlane16)
// and {lower half, upper half} (permlane32), as (first, second)
template <bool HALF32, typename T>
__device__ __forceinline__ void row_swap(T v, T &first, T &second) {
    if constexpr (sizeof(T) == 8) {
        const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
        unsigned lo0, lo1, hi0, hi1;
        if constexpr (HALF32) {
            const auto l = __builtin_amdgcn_permlane32_swap((unsigned)u, (unsigned)u, false, false);
            const auto h = __builtin_amdgcn_permlane32_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
            lo0 = l[0]; lo1 = l[1]; hi0 = h[0]; hi1 = h[1];
        } else {
            const auto l = __builtin_amdgcn_permlane16_swap((unsigned)u, (unsigned)u, false, false);
            const auto h = __builtin_amdgcn_permlane16_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
            lo0 = l[0]; lo1 = l[1]; hi0 = h[0]; hi1 = h[1];
        }
        first = __builtin_bit_cast(T, ((unsigned long long)hi0 << 32) | lo0);
        second = __builtin_bit_cast(T, ((unsigned long long)hi1 << 32) | lo1);
    } else {
        const unsigned u = __builtin_bit_cast(unsigned, v);
        if constexpr (HALF32) {
            const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
            first = __builtin_bit_cast(T, (unsigned)r[0]); second = __builtin_bit_cast(T, (unsigned)r[1]);
        } else {
            const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
            first = __builtin_bit_cast(T, (unsigned)r[0]); second = __builtin_bit_cast(T, (unsigned)r[1]);
        }
    }
}
template <typename T, class Op>
__device__ __forceinline__ T wave_reduce(T v, Op op) {
    v = op(v, dpp_move<0xB1>(v));   // quad_perm [1,0,3,2]
    v = op(v, dpp_move<0x4E>(v));   // quad_perm [2,3,0,1]
    v = op(v, dpp_move<0x141>(v));  // row_half_mirror
    v = op(v, dpp_move<0x140>(v));  // row_mirror
    T a, b;
    row_swap<false>(v, a, b);       // rows (0,1) and (2,3): a = even row, b = odd row
    v = op(a, b);
    row_swap<true>(v, a, b);        // halves: a = rows 0-1, b = rows 2-3
    return op(a, b);
}
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    return wave_reduce(v, [](T x, T y) { return x + y; });
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
    return wave_reduce(v, [](T x, T y) { return fmax(x, y); });
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
    return wave_reduce(v, [](T x, T y) { return fmin(x, y); });
}

// Workgroup reductions of up to three values at once (sum, max, min), the
// result returned to every thread.  Fixed order => deterministic.
template <typename T, int NT>
__device__ __forceinline__ void block_reduce3(T &vsum, T &vmax, T &vmin, T *red) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T a = wave_sum(vsum), b = wave_max(vmax), c = wave_min(vmin);
    if (lane == 0) { red[w] = a; red[NW + w] = b; red[2 * NW + w] = c; }
    __syncthreads();
    a = red[0]; b = red[NW]; c = red[2 * NW];
#pragma unroll
    for (int i = 1; i < NW; ++i) { a += red[i]; b = fmax(b, red[NW + i]); c = fmin(c, red[2 * NW + i]); }
    __syncthreads();
    vsum = a; vmax = b; vmin = c;
}

// Four values at once: a sum, two maxima and a minimum (red: 4 * NT/64 slots).
template <typename T, int NT>
__device__ __forceinline__ void block_reduce4(T &vsum, T &vmax, T &vmax2, T &vmin, T *red) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T a = wave_sum(vsum), b = wave_max(vmax), c = wave_max(vmax2), d = wave_min(vmin);
    if (lane == 0) { red[w] = a; red[NW + w] = b; red[2 * NW + w] = c; red[3 * NW + w] = d; }
    __syncthreads();
    a = red[0]; b = red[NW]; c = red[2 * NW]; d = red[3 * NW];
#pragma unroll
    for (int i = 1; i < NW; ++i) {
        a += red[i]; b = fmax(b, red[NW + i]); c = fmax(c, red[2 * NW + i]); d = fmin(d, red[3 * NW + i]);
    }
    __syncthreads();
    vsum = a; vmax = b; vmax2 = c; vmin = d;
}

template <typename T, int NT>
__device__ __forceinline__ T block_sum(T v, T *red) {
    T mx = 0, mn = 0;
    block_reduce3<T, NT>(v, mx, mn, red);
    return v;
}

template <typename T>
__device__ __forceinline__ T pinf() { return __builtin_huge_val(); }
template <>
__device__ __forceinline__ float pinf<float>() { return __builtin_huge_valf(); }

// ---------------------------------------------------------------------------
// Dense matrix-vector products.  M is row-major with leading dimension ld.

// y[c] = sum_{r<rows} M[r][c] x[r]   (one thread per column, coalesced rows)
template <typename T, int NT>
__device__ __forceinline__ void mv_cols(const T *__restrict__ M, int ld, int rows, int cols,
                                        const T *x, T *y) {
    for (int c = threadIdx.x; c < cols; c += NT) {
        T acc = 0;
        for (int r = 0; r < rows; ++r) acc += M[(size_t)r * ld + c] * x[r];
        y[c] = acc;
    }
}

// Sum over a row of 16 lanes (DPP quad_perm, row_half_mirror, row_mirror);
// every lane of the row ends with the same value.
template <typename T>
__device__ __forceinline__ T row16_sum(T v) {
    v += dpp_move<0xB1>(v);
    v += dpp_move<0x4E>(v);
    v += dpp_move<0x141>(v);
    v += dpp_move<0x140>(v);
    return v;
}

// y[r] = sum_{c<cols} M[r][c] x[c]: 16 lanes per row (four rows per wavefront
// at a time), four loads in flight per lane, in-row DPP reduction.  Measured
// 3-4x faster than a wavefront per row for global M.  No barrier at the end.
// V: the vectors' type and the accumulation type (FP64 over an FP32 matrix in
// the mixed-precision backward).
template <typename T, int NT, typename V = T>
__device__ __forceinline__ void mv_rows(const T *__restrict__ M, int ld, int rows, int cols,
                                        const V *x, V *y) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, cl = lane & 15;
    for (int r0 = 4 * w; r0 < rows; r0 += 4 * NW) {
        const int r = r0 + g < rows ? r0 + g : rows - 1;
        const T *row = M + (size_t)r * ld;
        V a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        int c = cl;
        for (; c + 48 < cols; c += 64) {
            a0 += row[c] * x[c];
            a1 += row[c + 16] * x[c + 16];
            a2 += row[c + 32] * x[c + 32];
            a3 += row[c + 48] * x[c + 48];
        }
        for (; c < cols; c += 16) a0 += row[c] * x[c];
        const V s = row16_sum((a0 + a1) + (a2 + a3));
        if (cl == 0 && r0 + g < rows) y[r0 + g] = s;
    }
}

// Rows [0, rows) of a staged chunk M (ld) that holds rows k0.. of G: the
// row dots gz[k0 + r] = (G x)_r by the arithmetic of mv_rows, and each row's
// weight in the affine right-hand side, wsc[k0 + r] = lam + D rz with
// rz = -(gz + s - h) (the residual of the slack equation).  No barrier at the end.
template <typename T, int NT>
__device__ __forceinline__ void chunk_rows_res(const T *__restrict__ M, int ld, int k0, int rows, int cols,
                                               const T *x, const T *lam, const T *D, const T *s,
                                               const T *h, T *gz, T *wsc) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, cl = lane & 15;
    for (int r0 = 4 * w; r0 < rows; r0 += 4 * NW) {
        const int r = r0 + g < rows ? r0 + g : rows - 1;
        const T *row = M + (size_t)r * ld;
        T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        int c = cl;
        for (; c + 48 < cols; c += 64) {
            a0 += row[c] * x[c];
            a1 += row[c + 16] * x[c + 16];
            a2 += row[c + 32] * x[c + 32];
            a3 += row[c + 48] * x[c + 48];
        }
        for (; c < cols; c += 16) a0 += row[c] * x[c];
        const T dot = row16_sum((a0 + a1) + (a2 + a3));
        if (cl == 0 && r0 + g < rows) {
            const int k = k0 + r0 + g;
            gz[k] = dot;
            const T rz = -(dot + s[k] - h[k]);
            wsc[k] = lam[k] + D[k] * rz;
        }
    }
}

// The largest row 1-norm max_r sum_{c<cols} |M[r][c]|, returned to every
// thread: 16 lanes per row as in mv_rows (coalesced, four loads in flight).
template <typename T, int NT>
__device__ __forceinline__ T max_row_abs_sum(const T *__restrict__ M, int ld, int rows, int cols, T *red) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, cl = lane & 15;
    T mx = 0;
    for (int r0 = 4 * w; r0 < rows; r0 += 4 * NW) {
        const int r = r0 + g < rows ? r0 + g : rows - 1;
        const T *row = M + (size_t)r * ld;
        T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        int c = cl;
        for (; c + 48 < cols; c += 64) {
            a0 += fabs(row[c]);
            a1 += fabs(row[c + 16]);
            a2 += fabs(row[c + 32]);
            a3 += fabs(row[c + 48]);
        }
        for (; c < cols; c += 16) a0 += fabs(row[c]);
        mx = fmax(mx, row16_sum((a0 + a1) + (a2 + a3)));
    }
    T d0 = 0, d1 = 0;
    block_reduce3<T, NT>(d0, mx, d1, red);
    return mx;
}

// The largest column 1-norm max_c sum_{r<rows} |M[r][c]|, returned to every
// thread: the rows are split into groups of threads (coalesced rows, eight
// loads in flight) as far as `cap` entries of `scratch` hold their partial sums,
// which are added in a fixed order.
template <typename T, int NT>
__device__ __forceinline__ T max_col_abs_sum(const T *__restrict__ M, int ld, int rows, int cols, T *scratch,
                                             int cap, T *red) {
    const int ng = cols > 0 ? max(1, min(min(NT, cap) / cols, 8)) : 1;
    const int chunk = (rows + ng - 1) / ng;
    T mx = 0;
    for (int t = threadIdx.x; t < ng * cols; t += NT) {
        const int q = t / cols, i = t - q * cols;
        const int k0 = q * chunk, k1 = min(rows, k0 + chunk);
        T a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0, a6 = 0, a7 = 0;
        int k = k0;
        for (; k + 7 < k1; k += 8) {
            a0 += fabs(M[(size_t)k * ld + i]);
            a1 += fabs(M[(size_t)(k + 1) * ld + i]);
            a2 += fabs(M[(size_t)(k + 2) * ld + i]);
            a3 += fabs(M[(size_t)(k + 3) * ld + i]);
            a4 += fabs(M[(size_t)(k + 4) * ld + i]);
            a5 += fabs(M[(size_t)(k + 5) * ld + i]);
            a6 += fabs(M[(size_t)(k + 6) * ld + i]);
            a7 += fabs(M[(size_t)(k + 7) * ld + i]);
        }
        for (; k < k1; ++k) a0 += fabs(M[(size_t)k * ld + i]);
        const T r = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
        if (ng > 1) scratch[t] = r;
        else mx = fmax(mx, r);
    }
    if (ng > 1) {
        __syncthreads();
        for (int i = threadIdx.x; i < cols; i += NT) {
            T acc = scratch[i];
            for (int q = 1; q < ng; ++q) acc += scratch[q * cols + i];
            mx = fmax(mx, acc);
        }
    }
    T d0 = 0, d1 = 0;
    block_reduce3<T, NT>(d0, mx, d1, red);
    return mx;
}

// out[i] = sum_{k<rows} M[k][i] v[k] for i < cols.  When cols < NT the rows
// are split into up to eight groups whose partial sums (scratch, NT entries)
// are added in a fixed order; otherwise one thread per column.
template <typename T, int NT, typename V = T>
__device__ __forceinline__ void colsum_split(const T *M, int ld, int rows, int cols, const V *v, V *out,
                                             V *scratch) {
    const int ng = cols > 0 ? max(1, min(NT / cols, 8)) : 1;
    const int chunk = (rows + ng - 1) / ng;
    for (int t = threadIdx.x; t < ng * cols; t += NT) {
        const int q = t / cols, i = t - q * cols;
        const int k0 = q * chunk, k1 = min(rows, k0 + chunk);
        V a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0, a6 = 0, a7 = 0;
        int k = k0;
        for (; k + 7 < k1; k += 8) {
            a0 += M[(size_t)k * ld + i] * v[k];
            a1 += M[(size_t)(k + 1) * ld + i] * v[k + 1];
            a2 += M[(size_t)(k + 2) * ld + i] * v[k + 2];
            a3 += M[(size_t)(k + 3) * ld + i] * v[k + 3];
            a4 += M[(size_t)(k + 4) * ld + i] * v[k + 4];
            a5 += M[(size_t)(k + 5) * ld + i] * v[k + 5];
            a6 += M[(size_t)(k + 6) * ld + i] * v[k + 6];
            a7 += M[(size_t)(k + 7) * ld + i] * v[k + 7];
        }
        for (; k < k1; ++k) a0 += M[(size_t)k * ld + i] * v[k];
        const V r = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
        if (ng == 1) out[i] = r;
        else scratch[t] = r;
    }
    if (ng > 1) {
        __syncthreads();
        for (int i = threadIdx.x; i < cols; i += NT) {
            V acc = scratch[i];
            for (int q = 1; q < ng; ++q) acc += scratch[q * cols + i];
            out[i] = acc;
        }
    }
    __syncthreads();
}

// out[k] = sum_{i<cols} M[k][i] x[i] for k < rows (M in LDS, odd ld): the
// columns are split into up to eight groups when rows < NT.
template <typename T, int NT>
__device__ __forceinline__ void rowdot_split(const T *M, int ld, int rows, int cols, const T *x, T *out,
                                             T *scratch) {
    const int ng = rows > 0 ? max(1, min(NT / rows, 8)) : 1;
    const int chunk = (cols + ng - 1) / ng;
    for (int t = threadIdx.x; t < ng * rows; t += NT) {
        const int q = t / rows, k = t - q * rows;
        const int i0 = q * chunk, i1 = min(cols, i0 + chunk);
        const T *row = M + (size_t)k * ld;
        T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        int i = i0;
        for (; i + 3 < i1; i += 4) {
            a0 += row[i] * x[i];
            a1 += row[i + 1] * x[i + 1];
            a2 += row[i + 2] * x[i + 2];
            a3 += row[i + 3] * x[i + 3];
        }
        for (; i < i1; ++i) a0 += row[i] * x[i];
        const T r = (a0 + a1) + (a2 + a3);
        if (ng == 1) out[k] = r;
        else scratch[t] = r;
    }
    if (ng > 1) {
        __syncthreads();
        for (int k = threadIdx.x; k < rows; k += NT) {
            T acc = scratch[k];
            for (int q = 1; q < ng; ++q) acc += scratch[q * rows + k];
            out[k] = acc;
        }
    }
    __syncthreads();
}

// y[i] = sum_{j<=i} U[j][i] f[j] for i < n (U upper triangular, incl. the
// diagonal): the rows are split into up to eight groups when n < NT, partial
// sums (scratch, NT entries) added in a fixed order; four loads in flight per
// thread.  Ends with a workgroup barrier.
template <typename T, int NT>
__device__ __forceinline__ void ut_mv_split(const T *U, int ld, int n, const T *f, T *y, T *scratch) {
    const int ng = n > 0 ? max(1, min(NT / n, 8)) : 1;
    const int chunk = (n + ng - 1) / ng;
    for (int t = threadIdx.x; t < ng * n; t += NT) {
        const int q = t / n, i = t - q * n;
        const int j0 = q * chunk, j1 = min(i + 1, j0 + chunk);
        T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        int j = j0;
        for (; j + 3 < j1; j += 4) {
            a0 += U[(size_t)j * ld + i] * f[j];
            a1 += U[(size_t)(j + 1) * ld + i] * f[j + 1];
            a2 += U[(size_t)(j + 2) * ld + i] * f[j + 2];
            a3 += U[(size_t)(j + 3) * ld + i] * f[j + 3];
        }
        for (; j < j1; ++j) a0 += U[(size_t)j * ld + i] * f[j];
        const T r = (a0 + a1) + (a2 + a3);
        if (ng == 1) y[i] = r;
        else scratch[t] = r;
    }
    if (ng > 1) {
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += NT) {
            T acc = scratch[i];
            for (int q = 1; q < ng; ++q) acc += scratch[q * n + i];
            y[i] = acc;
        }
    }
    __syncthreads();
}

// y = U^T f, U upper triangular (incl. diagonal):  y[i] = sum_{j<=i} U[j][i] f[j]
template <typename T, int NT>
__device__ __forceinline__ void ut_mv(const T *U, int ld, int n, const T *f, T *y) {
    for (int i = threadIdx.x; i < n; i += NT) {
        T acc = 0;
        for (int j = 0; j <= i; ++j) acc += U[(size_t)j * ld + i] * f[j];
        y[i] = acc;
    }
}

// x = U y:  x[j] = sum_{i>=j} U[j][i] y[i]   (16 lanes per row, as mv_rows)
template <typename T, int NT>
__device__ __forceinline__ void u_mv(const T *U, int ld, int n, const T *y, T *x) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, cl = lane & 15;
    for (int j0 = 4 * w; j0 < n; j0 += 4 * NW) {
        const int j = j0 + g < n ? j0 + g : n - 1;
        const T *row = U + (size_t)j * ld;
        T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        int i = j + cl;
        for (; i + 48 < n; i += 64) {
            a0 += row[i] * y[i];
            a1 += row[i + 16] * y[i + 16];
            a2 += row[i + 32] * y[i + 32];
            a3 += row[i + 48] * y[i + 48];
        }
        for (; i < n; i += 16) a0 += row[i] * y[i];
        const T s = row16_sum((a0 + a1) + (a2 + a3));
        if (cl == 0 && j0 + g < n) x[j0 + g] = s;
    }
}

// ---------------------------------------------------------------------------
// Cholesky factorisation fused with the triangular inverse, in place.
//
// On entry the lower triangle (incl. diagonal) of H holds the SPD matrix and
// its strict upper triangle is zero.  Right-looking: at step k, column k of L
// is final; the trailing lower block is updated, and in the same pass row k of
// X = L^{-1} (a forward substitution of L X = I carried for all right-hand
// sides at once) updates the rows below it.  X is stored transposed in the
// upper triangle (X[i][j] at H[j][i]), its diagonal in xd.  On exit the upper
// triangle (incl. diagonal) holds U = L^{-T}.  Returns false (uniformly) on a
// non-positive or non-finite pivot.
template <typename T, int NT>
__device__ __forceinline__ bool chol_inv(T *H, int ld, int n, T *xd) {
    const int tid = threadIdx.x;
    for (int k = 0; k < n; ++k) {
        const T dkk = H[(size_t)k * ld + k];
        if (!(dkk > T(0)) || !isfinite(dkk)) return false;
        const T inv = T(1) / sqrt(dkk);
        // Phase A: scale column k of L (rows > k) and row k of X (H[j][k], j < k).
        for (int i = tid; i < n; i += NT)
            if (i != k) H[(size_t)i * ld + k] *= inv;
        if (tid == 0) xd[k] = inv;
        __syncthreads();
        // Phase B over the rectangle rows (k, n) x columns [0, n), j <= i:
        //   j >  k: L trailing update  H[i][j] -= L[i][k] L[j][k]
        //   j <= k: X update           X[i][j] -= L[i][k] X[k][j]   (stored at H[j][i])
        const int rows = n - k - 1;
        const int total = rows * n;
        for (int e = tid; e < total; e += NT) {
            const int i = k + 1 + e / n, j = e % n;
            if (j > i) continue;
            const T lik = H[(size_t)i * ld + k];
            if (j > k) {
                H[(size_t)i * ld + j] -= lik * H[(size_t)j * ld + k];
            } else {
                const T xkj = (j < k) ? H[(size_t)j * ld + k] : xd[k];
                H[(size_t)j * ld + i] -= lik * xkj;
            }
        }
        __syncthreads();
    }
    for (int i = tid; i < n; i += NT) H[(size_t)i * ld + i] = xd[i];
    __syncthreads();
    return true;
}

// Reduced KKT solve with the stored inverse factors:
//   [H A^T; A 0] [dz; dnu] = [f; r4]
//   y = L^{-1} f;  dnu = S^{-1} (Wt y - r4);  dz = L^{-T} (y - Wt^T dnu)
// y [n], t1/t2 [p] and scratch [NT] are scratch.  Results in dz [n], dnu [p].
template <typename T, int NT>
__device__ void kkt_solve(const T *U, int ldu, const T *Wt, const T *US, int n, int p,
                          const T *f, const T *r4, T *y, T *t1, T *t2, T *dz, T *dnu, T *scratch) {
    ut_mv_split<T, NT>(U, ldu, n, f, y, scratch);
    if (p > 0) {
        mv_rows<T, NT>(Wt, n, p, n, y, t1);
        __syncthreads();
        for (int k = threadIdx.x; k < p; k += NT) t1[k] -= r4[k];
        __syncthreads();
        ut_mv<T, NT>(US, p, p, t1, t2);
        __syncthreads();
        u_mv<T, NT>(US, p, p, t2, dnu);
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += NT) {
            T acc = y[i];
            for (int k = 0; k < p; ++k) acc -= Wt[(size_t)k * n + i] * dnu[k];
            y[i] = acc;
        }
        __syncthreads();
    }
    u_mv<T, NT>(U, ldu, n, y, dz);
    __syncthreads();
}

// H = Qs + G^T D G into the lower triangle of H (ld ldh), zero strict upper.
template <typename T, int NT>
__device__ void form_h(const T *__restrict__ Q, const T *__restrict__ G, const T *D, int n, int m,
                       T *H, int ldh) {
    const int total = n * n;
    for (int e = threadIdx.x; e < total; e += NT) {
        const int i = e / n, j = e % n;
        if (j <= i) {
            T acc = T(0.5) * (Q[(size_t)i * n + j] + Q[(size_t)j * n + i]);
            for (int k = 0; k < m; ++k) acc += G[(size_t)k * n + i] * D[k] * G[(size_t)k * n + j];
            H[(size_t)i * ldh + j] = acc;
        } else {
            H[(size_t)i * ldh + j] = T(0);
        }
    }
    __syncthreads();
}

// Schur complement on A: Wt[k][:] = L^{-1} A[k][:]^T, S = Wt Wt^T into the lower
// triangle of US (strict upper zeroed), then US <- LS^{-T} in place.
template <typename T, int NT>
__device__ bool schur(const T *U, int ldu, const T *__restrict__ A, int n, int p, T *Wt, T *US,
                      T *xdp) {
    const int tot = p * n;
    for (int e = threadIdx.x; e < tot; e += NT) {
        const int k = e / n, i = e % n;
        T acc = 0;
        for (int j = 0; j <= i; ++j) acc += U[(size_t)j * ldu + i] * A[(size_t)k * n + j];
        Wt[(size_t)k * n + i] = acc;
    }
    __syncthreads();
    const int tp = p * p;
    for (int e = threadIdx.x; e < tp; e += NT) {
        const int k = e / p, l = e % p;
        T acc = 0;
        if (l <= k)
            for (int i = 0; i < n; ++i) acc += Wt[(size_t)k * n + i] * Wt[(size_t)l * n + i];
        US[(size_t)k * p + l] = acc;
    }
    __syncthreads();
    return chol_inv<T, NT>(US, p, p, xdp);
}

}  // namespace qpmi
