// Uneven-batch persistent forward kernels instantiated for float.
#include "qp_forward.hpp"

namespace qpmi {
template hipError_t launch_varlen_t<float>(const FwdLaunch &, hipStream_t);
template int resident_t<float>(int, bool);
}  // namespace qpmi
