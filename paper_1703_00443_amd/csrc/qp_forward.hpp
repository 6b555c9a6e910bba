// Forward kernels: the interior point method of Section 3.1 for a batch of
// QPs, one workgroup (512 threads, eight wavefronts) per problem, the whole
// solve (initial point, Newton loop, stored factor) in one launch.
//
// * Uniform batch (every problem has the same dims, hence the same plan): one
//   kernel per factorization policy with the solve inlined.
// * Uneven batch: one persistent kernel over a work queue; each workgroup
//   picks the policy of the problem it takes from that problem's own dims.
//
// Included by one translation unit per element type.
#pragma once
#include "qp_elim.hpp"
#include "qp_stream.hpp"

namespace qpmi {

constexpr int kFwdThreads = 64 * kTiledWaves;

__host__ __device__ inline int plan_policy(int esz, int n, int m, int p, int variant, int lds_limit,
                                           int *lds_bytes) {
    const int base = IpmLayout(n, m, p).end;
    if (variant == QP_VARIANT_ELIM && m <= u_ld(n) && m <= kTiledMaxN) {
        // taken on request (or from an autotune table); where it does not
        // apply the automatic plan runs.  Above the register tiles' nz the
        // nz x nz factorizations run on the streamed policy (BIG).
        const bool big = n > kTiledMaxN;
        const int el = elim_lds_elems(esz, base, n, m, p, big, lds_limit) * esz;
        if (el > 0 && el <= lds_limit) { *lds_bytes = el; return big ? kPolicyElimBig : kPolicyElim; }
    }
    if (variant == QP_VARIANT_AUTO || variant == QP_VARIANT_TILED || variant == QP_VARIANT_ELIM) {
        if (n <= kTiledMaxN) {
            const int gl = TiledLayout<true>(base, n, m, p).end * esz;
            if (gl <= lds_limit) { *lds_bytes = gl; return kPolicyTiledGLds; }
            const int gg = TiledLayout<false>(base, n, m, p).end * esz;
            if (gg <= lds_limit) { *lds_bytes = gg; return kPolicyTiledGGlobal; }
        } else if (esz == 4 && n <= kTiledBigMaxN) {
            const int gg = TiledLayout<false>(base, n, m, p).end * esz;
            if (gg <= lds_limit) { *lds_bytes = gg; return kPolicyTiledBig; }
        }
    }
    if (variant == QP_VARIANT_AUTO || variant == QP_VARIANT_STREAM || variant == QP_VARIANT_ELIM) {
        int kc = 0;
        bool s_lds = true;
        if (stream_plan(esz, base, n, m, p, lds_limit, &kc, &s_lds)) {
            *lds_bytes = StreamLayout(base, n, m, p, kc, s_lds).end * esz;
            return kPolicyStream;
        }
    }
    if (variant != QP_VARIANT_GENERIC) {
        const int hl = GenericLayout<true>(base, n, m, p).end * esz;
        if (hl <= lds_limit) { *lds_bytes = hl; return kPolicyGenericLds; }
    }
    const int gg = GenericLayout<false>(base, n, m, p).end * esz;
    if (gg <= lds_limit) { *lds_bytes = gg; return kPolicyGenericGlobal; }
    *lds_bytes = gg;
    return kPolicyNone;
}

// One problem under one policy (uneven batches).  Inlined: measured 9% faster
// on the 4096-problem uneven batch than out-of-line calls, whose calling
// convention saved and spilled registers.
template <typename T, class F>
__device__ __forceinline__ void run_policy(const Prob<T> P, T *sm, const FwdLaunch &L) {
    const IpmLayout Lo(P.n, P.m, P.p);
    F f(P, sm, Lo.end);
    ipm_solve<T, kFwdThreads>(P, sm, Lo, f, L.max_iter, (T)L.tol, L.status, L.iters);
}

// The elimination order, or the tiled policy where Qs does not factor (the
// decision is made before the solve, so each Newton loop is its own code).
template <typename T, bool EQ, bool BIG>
__device__ __forceinline__ void run_elim(const Prob<T> &P, T *sm, const FwdLaunch &L) {
    const IpmLayout Lo(P.n, P.m, P.p);
    {
        ElimFactor<T, EQ, BIG> f(P, sm, Lo.end);
        if (f.factor_qs()) {
            ipm_solve<T, kFwdThreads>(P, sm, Lo, f, L.max_iter, (T)L.tol, L.status, L.iters);
            return;
        }
    }
    if constexpr (BIG) {
        StreamFactor<T, EQ> f(P, sm, Lo.end);
        ipm_solve<T, kFwdThreads>(P, sm, Lo, f, L.max_iter, (T)L.tol, L.status, L.iters);
    } else {
        TiledFactor<T, false, 8, EQ> f(P, sm, Lo.end);
        ipm_solve<T, kFwdThreads>(P, sm, Lo, f, L.max_iter, (T)L.tol, L.status, L.iters);
    }
}

template <typename T, bool EQ, bool UNIT>
__device__ __forceinline__ void run_tiled(int pol, const Prob<T> &P, T *sm, const FwdLaunch &L) {
    if (pol == kPolicyTiledGLds) {
        run_policy<T, TiledFactor<T, true, 8, EQ, UNIT>>(P, sm, L);
    } else if (pol == kPolicyTiledGGlobal) {
        run_policy<T, TiledFactor<T, false, 8, EQ, UNIT>>(P, sm, L);
    } else if constexpr (sizeof(T) == 4) {
        run_policy<T, TiledFactor<T, false, 16, EQ, UNIT>>(P, sm, L);
    }
}

// ELIM: the instantiation that also carries the elimination-order policy,
// launched only when some problem of the batch plans it (the policy's code in
// the kernel costs the others registers).  UNIT: the instantiation whose tiled
// and streamed policies take the unit-row path (QP_FLAG_G_UNIT_ROWS set on the
// call; each problem's G is still checked, and a dense G runs the dense path).
// A call with both gets the ELIM instantiation, where the flag is not used.
template <typename T, bool ELIM, bool UNIT>
__global__ __launch_bounds__(kFwdThreads) void qp_forward_varlen_kernel(FwdLaunch L) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int next_idx;
    T *sm = reinterpret_cast<T *>(smem_raw);
    int idx = blockIdx.x;
    for (;;) {
        if (L.queue) {
            // work queue: problems are taken in `order` (largest first) as
            // workgroups free up; every workgroup exits once the queue is empty
            if (threadIdx.x == 0) next_idx = atomicAdd(L.queue, 1);
            __syncthreads();
            idx = next_idx;
            __syncthreads();
        }
        if (idx >= L.count) break;
        const Prob<T> P = fwd_problem<T>(L, idx);
        int bytes = 0;
        const int pol = plan_policy(sizeof(T), P.n, P.m, P.p, P.variant, L.lds_limit, &bytes);
        if (pol == kPolicyTiledGLds || pol == kPolicyTiledGGlobal || pol == kPolicyTiledBig) {
            if (P.p > 0) run_tiled<T, true, UNIT>(pol, P, sm, L);
            else run_tiled<T, false, UNIT>(pol, P, sm, L);
        } else if (pol == kPolicyStream) {
            if (P.p > 0) run_policy<T, StreamFactor<T, true, UNIT>>(P, sm, L);
            else run_policy<T, StreamFactor<T, false, UNIT>>(P, sm, L);
        } else if (ELIM && (pol == kPolicyElim || pol == kPolicyElimBig)) {
            if constexpr (ELIM) {
                if (pol == kPolicyElimBig) {
                    if (P.p > 0) run_elim<T, true, true>(P, sm, L);
                    else run_elim<T, false, true>(P, sm, L);
                } else {
                    if (P.p > 0) run_elim<T, true, false>(P, sm, L);
                    else run_elim<T, false, false>(P, sm, L);
                }
            }
        } else if (pol == kPolicyGenericLds) {
            run_policy<T, GenericFactor<T, kFwdThreads, true>>(P, sm, L);
        } else {
            run_policy<T, GenericFactor<T, kFwdThreads, false>>(P, sm, L);
        }
        if (!L.queue) idx += gridDim.x;
    }
}

// Uniform batch: the plan is the same for every problem, so the launch runs
// one policy with the solve inlined.
template <typename T, class F>
__global__ __launch_bounds__(kFwdThreads) void qp_forward_uniform_kernel(FwdLaunch L) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);
    for (int idx = blockIdx.x; idx < L.count; idx += gridDim.x) {
        const Prob<T> P = fwd_problem<T>(L, idx);
        const IpmLayout Lo(P.n, P.m, P.p);
        F f(P, sm, Lo.end);
        ipm_solve<T, kFwdThreads>(P, sm, Lo, f, L.max_iter, (T)L.tol, L.status, L.iters);
    }
}

// Uniform batch on the elimination order (EQ: equality rows; BIG: streamed
// nz x nz factorizations).
template <typename T, bool EQ, bool BIG>
__global__ __launch_bounds__(kFwdThreads) void qp_forward_elim_kernel(FwdLaunch L) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);
    for (int idx = blockIdx.x; idx < L.count; idx += gridDim.x)
        run_elim<T, EQ, BIG>(fwd_problem<T>(L, idx), sm, L);
}

// Once per kernel (the flag is per instantiation, i.e. per kernel function).
template <auto Kern>
static void set_lds_limit_once(int lds_limit) {
    static bool done = false;
    if (!done) {
        (void)hipFuncSetAttribute((const void *)Kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds_limit);
        done = true;
    }
}

template <typename T, class F>
static hipError_t launch_uniform(const FwdLaunch &L, hipStream_t st) {
    auto kern = qp_forward_uniform_kernel<T, F>;
    set_lds_limit_once<qp_forward_uniform_kernel<T, F>>(L.lds_limit);
    hipLaunchKernelGGL(kern, dim3(L.count), dim3(kFwdThreads), L.lds_bytes, st, L);
    return hipGetLastError();
}

template <typename T, bool EQ, bool UNIT>
static hipError_t launch_uniform_tiled_u(int pol, const FwdLaunch &L, hipStream_t st) {
    if (pol == kPolicyTiledGLds) return launch_uniform<T, TiledFactor<T, true, 8, EQ, UNIT>>(L, st);
    if (pol == kPolicyTiledGGlobal) return launch_uniform<T, TiledFactor<T, false, 8, EQ, UNIT>>(L, st);
    if constexpr (sizeof(T) == 4) return launch_uniform<T, TiledFactor<T, false, 16, EQ, UNIT>>(L, st);
    return hipErrorInvalidValue;
}

// QP_FLAG_G_UNIT_ROWS selects the unit-row instantiations.
template <typename T, bool EQ>
static hipError_t launch_uniform_tiled(int pol, const FwdLaunch &L, hipStream_t st) {
    if ((L.flags & QP_FLAG_G_UNIT_ROWS) && L.nineq > 0) return launch_uniform_tiled_u<T, EQ, true>(pol, L, st);
    return launch_uniform_tiled_u<T, EQ, false>(pol, L, st);
}

template <typename T, bool EQ>
static hipError_t launch_uniform_stream(const FwdLaunch &L, hipStream_t st) {
    if ((L.flags & QP_FLAG_G_UNIT_ROWS) && L.nineq > 0) return launch_uniform<T, StreamFactor<T, EQ, true>>(L, st);
    return launch_uniform<T, StreamFactor<T, EQ, false>>(L, st);
}

__global__ void qp_zero_counter_kernel(int *c);

// Each launcher is instantiated in a translation unit of its own per element
// type (qp_forward_{f32,f64}.hip, qp_forward_elim_*.hip, qp_forward_varlen_*.hip)
// so that the kernels compile in parallel.
template <typename T, bool BIG>
static hipError_t launch_elim_k(const FwdLaunch &L, hipStream_t st) {
    auto kern = L.neq > 0 ? qp_forward_elim_kernel<T, true, BIG> : qp_forward_elim_kernel<T, false, BIG>;
    if (L.neq > 0) set_lds_limit_once<qp_forward_elim_kernel<T, true, BIG>>(L.lds_limit);
    else set_lds_limit_once<qp_forward_elim_kernel<T, false, BIG>>(L.lds_limit);
    hipLaunchKernelGGL(kern, dim3(L.count), dim3(kFwdThreads), L.lds_bytes, st, L);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_elim_t(const FwdLaunch &L, hipStream_t st, int big) {
    return big ? launch_elim_k<T, true>(L, st) : launch_elim_k<T, false>(L, st);
}

template <typename T>
hipError_t launch_uniform_t(const FwdLaunch &L, hipStream_t st);

template <typename T>
hipError_t launch_varlen_t(const FwdLaunch &L, hipStream_t st);

// Uniform batch: one kernel per policy (the elimination order's in its own unit).
template <typename T>
hipError_t launch_uniform_t(const FwdLaunch &L, hipStream_t st) {
    if (L.count <= 0) return hipSuccess;
    {
        int bytes = 0;
        const int pol = plan_policy(sizeof(T), L.nz, L.nineq, L.neq, L.variant, L.lds_limit, &bytes);
        if (pol == kPolicyTiledGLds || pol == kPolicyTiledGGlobal || pol == kPolicyTiledBig)
            return L.neq > 0 ? launch_uniform_tiled<T, true>(pol, L, st)
                             : launch_uniform_tiled<T, false>(pol, L, st);
        if (pol == kPolicyStream)
            return L.neq > 0 ? launch_uniform_stream<T, true>(L, st) : launch_uniform_stream<T, false>(L, st);
        if (pol == kPolicyElim || pol == kPolicyElimBig) return launch_elim_t<T>(L, st, pol == kPolicyElimBig);
        if (pol == kPolicyGenericLds) return launch_uniform<T, GenericFactor<T, kFwdThreads, true>>(L, st);
        return launch_uniform<T, GenericFactor<T, kFwdThreads, false>>(L, st);
    }
}

// Uneven batch: the persistent kernel (instantiation by the call's needs).
template <typename T>
hipError_t launch_varlen_t(const FwdLaunch &L, hipStream_t st) {
    if (L.count <= 0) return hipSuccess;
    const bool unit = !L.with_elim && (L.flags & QP_FLAG_G_UNIT_ROWS) != 0;
    auto kern = L.with_elim ? qp_forward_varlen_kernel<T, true, false>
                            : unit ? qp_forward_varlen_kernel<T, false, true> : qp_forward_varlen_kernel<T, false, false>;
    if (L.with_elim) set_lds_limit_once<qp_forward_varlen_kernel<T, true, false>>(L.lds_limit);
    else if (unit) set_lds_limit_once<qp_forward_varlen_kernel<T, false, true>>(L.lds_limit);
    else set_lds_limit_once<qp_forward_varlen_kernel<T, false, false>>(L.lds_limit);
    if (L.queue) {
        hipLaunchKernelGGL(qp_zero_counter_kernel, dim3(1), dim3(1), 0, st, L.queue);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int grid = L.grid > 0 ? L.grid : L.count;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kFwdThreads), L.lds_bytes, st, L);
    return hipGetLastError();
}

template <typename T>
int resident_t(int lds_bytes, bool with_elim) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 1;
    const hipError_t e =
        with_elim ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, qp_forward_varlen_kernel<T, true, false>,
                                                                 kFwdThreads, (size_t)lds_bytes)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, qp_forward_varlen_kernel<T, false, false>,
                                                                 kFwdThreads, (size_t)lds_bytes);
    if (e != hipSuccess || per < 1) per = 1;
    return cus * per;
}

}  // namespace qpmi
