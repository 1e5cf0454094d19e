// Eigensolve / transform / update kernel instantiated for 32-row matrices
// (one translation unit per size so the unrolled sweeps compile in parallel).
#include "k_evd.h"

namespace letkf {
template hipError_t launch_evd_kp<32>(const BatchMap&, hipStream_t);
}  // namespace letkf
