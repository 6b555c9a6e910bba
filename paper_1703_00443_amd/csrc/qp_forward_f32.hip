// Forward kernels instantiated for float (one translation unit per element type).
#include "qp_forward.hpp"

namespace qpmi {
template hipError_t launch_fwd_t<float>(const FwdLaunch &, hipStream_t);
template int resident_t<float>(int, bool);
}  // namespace qpmi
