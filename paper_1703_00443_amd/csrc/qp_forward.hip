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

template <typename T>
__global__ __launch_bounds__(kFwdThreads) void qp_forward_kernel(FwdLaunch L) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);
    const T tol = (T)L.tol;
    for (int idx = blockIdx.x; idx < L.count; idx += gridDim.x) {
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
    hipLaunchKernelGGL(kern, dim3(L.count), dim3(kFwdThreads), L.lds_bytes, st, L);
    return hipGetLastError();
}

hipError_t launch_forward(qp_dtype dt, const FwdLaunch &L, hipStream_t st) {
    return dt == QP_F64 ? launch_fwd_t<double>(L, st) : launch_fwd_t<float>(L, st);
}

}  // namespace qpmi
