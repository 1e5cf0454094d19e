// The fused analysis kernels at KP = 64 (all precision forms).
#define LETKF_OPAQUE_LANE 1
#include "k_fused.h"

namespace letkf {
template hipError_t launch_fused_kp<64>(const BatchMap& bm, int prec, hipStream_t s);
}  // namespace letkf
