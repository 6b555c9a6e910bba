// Uniform-batch forward kernels instantiated for double (one translation unit per
// element type and kernel family, compiled in parallel).
#include "qp_forward.hpp"

namespace qpmi {
extern template hipError_t launch_elim_t<double>(const FwdLaunch &, hipStream_t, int);
template hipError_t launch_uniform_t<double>(const FwdLaunch &, hipStream_t);
}  // namespace qpmi
