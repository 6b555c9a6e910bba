// Forward entry of the kernels: plan query and dispatch by element type and
// batch kind.  The kernels themselves are compiled in qp_forward_{f32,f64}.hip
// (uniform batches), qp_forward_elim_{f32,f64}.hip (the elimination order) and
// qp_forward_varlen_{f32,f64}.hip (uneven batches).
#include "qp_forward.hpp"

namespace qpmi {

int fwd_plan(int esz, int n, int m, int p, int variant, int lds_limit, int *lds_bytes) {
    return plan_policy(esz, n, m, p, variant, lds_limit, lds_bytes);
}

__global__ void qp_zero_counter_kernel(int *c) { *c = 0; }

extern template hipError_t launch_uniform_t<float>(const FwdLaunch &, hipStream_t);
extern template hipError_t launch_uniform_t<double>(const FwdLaunch &, hipStream_t);
extern template hipError_t launch_varlen_t<float>(const FwdLaunch &, hipStream_t);
extern template hipError_t launch_varlen_t<double>(const FwdLaunch &, hipStream_t);
extern template int resident_t<float>(int, bool);
extern template int resident_t<double>(int, bool);

int fwd_resident_workgroups(qp_dtype dt, int lds_bytes, bool with_elim) {
    return dt == QP_F64 ? resident_t<double>(lds_bytes, with_elim) : resident_t<float>(lds_bytes, with_elim);
}

hipError_t launch_forward(qp_dtype dt, const FwdLaunch &L, hipStream_t st) {
    if (L.desc == nullptr) return dt == QP_F64 ? launch_uniform_t<double>(L, st) : launch_uniform_t<float>(L, st);
    return dt == QP_F64 ? launch_varlen_t<double>(L, st) : launch_varlen_t<float>(L, st);
}

}  // namespace qpmi
