// Elimination-order forward kernels (uniform batches) instantiated for double.
#include "qp_forward.hpp"

namespace qpmi {
template hipError_t launch_elim_t<double>(const FwdLaunch &, hipStream_t, int);
}  // namespace qpmi
