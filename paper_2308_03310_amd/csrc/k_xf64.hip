// Explicit instantiation of the transform kernel for KP = 64 (its own
// translation unit so that the widths compile in parallel).
#include "k_xf.h"

namespace letkf {
template hipError_t launch_evd_xf_kp<64>(const BatchMap&, hipStream_t);
}  // namespace letkf
