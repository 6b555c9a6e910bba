// Uneven-batch persistent forward kernels instantiated for double.
#include "qp_forward.hpp"

namespace qpmi {
template hipError_t launch_varlen_t<double>(const FwdLaunch &, hipStream_t);
template int resident_t<double>(int, bool);
}  // namespace qpmi
