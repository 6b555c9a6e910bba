// Forward kernel: the interior point method of Section 3.1 for a batch of
// QPs, one workgroup (256 threads) per problem, the whole solve (initial point,
// Newton loop, stored factor) in one launch.  Each workgroup picks the
// factorization policy of its problem from the problem's own dims.
#include "qp_policies.hpp"

namespace qpmi {

constexpr int kFwdThreads = 64 * kTiledWaves;

__host__ __device__ inline int plan_policy(int esz, int n, int m, int p, int variant, int lds_limit,
                                           int *lds_bytes) {
    const int base = IpmLayout(n, m, p).end;
    if ((variant == QP_VARIANT_AUTO || variant == QP_VARIANT_TILED) && p == 0 && n <= kTiledMaxN) {
        const int gl = TiledLayout<true>(base, n, m).end * esz;
        if (gl <= lds_limit) { *lds_bytes = gl; return kPolicyTiledGLds; }
        const int gg = TiledLayout<false>(base, n, m).end * esz;
        if (gg <= lds_limit) { *lds_bytes = gg; return kPolicyTiledGGlobal; }
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

int fwd_plan(int esz, int n, int m, int p, int variant, int lds_limit, int *lds_bytes) {
    return plan_policy(esz, n, m, p, variant, lds_limit, lds_bytes);
}

__global__ void qp_zero_counter_kernel(int *c) { *c = 0; }

template <typename T>
__global__ __launch_bounds__(kFwdThreads) void qp_forward_kernel(FwdLaunch L) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int next_idx;
    T *sm = reinterpret_cast<T *>(smem_raw);
    const T tol = (T)L.tol;
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
        const IpmLayout Lo(P.n, P.m, P.p);
        int bytes = 0;
        const int pol = plan_policy(sizeof(T), P.n, P.m, P.p, P.variant, L.lds_limit, &bytes);
        if (pol == kPolicyTiledGLds) {
            TiledFactor<T, true> f(P, sm, Lo.end);
            ipm_solve<T, kFwdThreads>(P, sm, Lo, f, L.max_iter, tol, L.status, L.iters);
        } else if (pol == kPolicyTiledGGlobal) {
            TiledFactor<T, false> f(P, sm, Lo.end);
            ipm_solve<T, kFwdThreads>(P, sm, Lo, f, L.max_iter, tol, L.status, L.iters);
        } else if (pol == kPolicyGenericLds) {
            GenericFactor<T, kFwdThreads, true> f(P, sm, Lo.end);
            ipm_solve<T, kFwdThreads>(P, sm, Lo, f, L.max_iter, tol, L.status, L.iters);
        } else {
            GenericFactor<T, kFwdThreads, false> f(P, sm, Lo.end);
            ipm_solve<T, kFwdThreads>(P, sm, Lo, f, L.max_iter, tol, L.status, L.iters);
        }
        if (!L.queue) idx += gridDim.x;
    }
}

template <typename T>
static hipError_t launch_fwd_t(const FwdLaunch &L, hipStream_t st) {
    if (L.count <= 0) return hipSuccess;
    auto kern = qp_forward_kernel<T>;
    static bool attr_done = false;
    if (!attr_done) {
        (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  L.lds_limit);
        attr_done = true;
    }
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
static int resident_t(int lds_bytes) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, qp_forward_kernel<T>, kFwdThreads,
                                                     (size_t)lds_bytes) != hipSuccess || per < 1)
        per = 1;
    return cus * per;
}

int fwd_resident_workgroups(qp_dtype dt, int lds_bytes) {
    return dt == QP_F64 ? resident_t<double>(lds_bytes) : resident_t<float>(lds_bytes);
}

hipError_t launch_forward(qp_dtype dt, const FwdLaunch &L, hipStream_t st) {
    return dt == QP_F64 ? launch_fwd_t<double>(L, st) : launch_fwd_t<float>(L, st);
}

}  // namespace qpmi
