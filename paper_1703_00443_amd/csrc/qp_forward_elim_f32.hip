// Elimination-order forward kernels (uniform batches) instantiated for float.
#include "qp_forward.hpp"

namespace qpmi {
template hipError_t launch_elim_t<float>(const FwdLaunch &, hipStream_t, int);
}  // namespace qpmi
