// Uniform-batch forward kernels instantiated for float (one translation unit per
// element type and kernel family, compiled in parallel).
#include "qp_forward.hpp"

namespace qpmi {
extern template hipError_t launch_elim_t<float>(const FwdLaunch &, hipStream_t, int);
template hipError_t launch_uniform_t<float>(const FwdLaunch &, hipStream_t);
}  // namespace qpmi
