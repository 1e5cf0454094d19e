// Localized Gram matrix and right-hand side per grid point, FP64 on MFMA:
// the grid and persistent launches of the per-point routine (k_gram.h).
#include "k_gram.h"

namespace letkf {

// Grid form: one wavefront per point, four points per block, blocks remapped
// so that neighbouring points (which share observations) stay on one XCD:
// contiguous eighths of a one-problem launch, interleaved runs of blocks
// when the launch covers several problems (whose cost per point differs).
// Persistent form: a device-filling grid whose wavefronts take points from
// per-XCD work queues over contiguous eighths of the slab and, once their
// own eighth is done, from the others' (load balance when the local
// observation counts differ widely between points).
template <int KQ, bool PERSIST>
__global__ __launch_bounds__(256) void k_gram_f64(BatchMap bm) {
  __shared__ int s_ring[4][kRing];
  __shared__ double w_ring[4][kRing];
  const int wid = threadIdx.x >> 6;
  if constexpr (!PERSIST) {
    const int blk = bm.nprob > 1 ? xcd_remap_runs<kBatchRun>(blockIdx.x, gridDim.x)
                                 : xcd_remap(blockIdx.x, gridDim.x);
    const int pl = blk * 4 + wid;
    if (pl < bm.n) gram_f64_point<KQ>(bm, pl, s_ring[wid], w_ring[wid], gram_c(bm, pl, KQ),
                                      gram_b(bm, pl, KQ));
  } else {
    for_each_queued_point(bm, [&](int pl) {
      gram_f64_point<KQ>(bm, pl, s_ring[wid], w_ring[wid], gram_c(bm, pl, KQ), gram_b(bm, pl, KQ));
    });
  }
}

hipError_t launch_gram_f64(const BatchMap& a, int kp, bool persistent, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (persistent && launch_fill_i32(a.queue, kQueueSlots, 0, s) != hipSuccess)
    return hipErrorLaunchFailure;
  const dim3 grid(persistent ? persistent_blocks(a.n, 4) : ceil_div(a.n, 4)), block(256);
#define LETKF_GRAM_F64(KP_)                                                                   \
  if (kp == KP_) {                                                                           \
    if (persistent)                                                                          \
      hipLaunchKernelGGL((k_gram_f64<KP_, true>), grid, block, 0, s, a);                      \
    else                                                                                     \
      hipLaunchKernelGGL((k_gram_f64<KP_, false>), grid, block, 0, s, a);                     \
    return hipGetLastError();                                                                \
  }
  LETKF_GRAM_F64(16)
  LETKF_GRAM_F64(32)
  LETKF_GRAM_F64(64)
#undef LETKF_GRAM_F64
  return hipErrorInvalidValue;
}

}  // namespace letkf
