// Forward kernels instantiated for double (one translation unit per element type).
#include "qp_forward.hpp"

namespace qpmi {
template hipError_t launch_fwd_t<double>(const FwdLaunch &, hipStream_t);
template int resident_t<double>(int, bool);
}  // namespace qpmi
