// Localized Gram matrix and right-hand side in the reduced-precision forms:
// the grid and persistent launches of the per-point routine (k_gram_lp.h).
#include "k_gram_lp.h"

namespace letkf {

// Grid and persistent forms, as for k_gram_f64.
template <int KQ, int PREC, bool PERSIST>
__global__ __launch_bounds__(256, 2) void k_gram_lp(BatchMap bm) {
  __shared__ int s_ring[4][kRing];
  __shared__ double w_ring[4][kRing];
  const int wid = threadIdx.x >> 6;
  if constexpr (!PERSIST) {
    const int blk = bm.nprob > 1 ? xcd_remap_runs<kBatchRun>(blockIdx.x, gridDim.x)
                                 : xcd_remap(blockIdx.x, gridDim.x);
    const int pl = blk * 4 + wid;
    if (pl < bm.n)
      gram_lp_point<KQ, PREC>(bm, pl, s_ring[wid], w_ring[wid], gram_c(bm, pl, KQ),
                              gram_b(bm, pl, KQ));
  } else {
    for_each_queued_point(bm, [&](int pl) {
      gram_lp_point<KQ, PREC>(bm, pl, s_ring[wid], w_ring[wid], gram_c(bm, pl, KQ),
                              gram_b(bm, pl, KQ));
    });
  }
}

hipError_t launch_gram_lp(const BatchMap& a, int kp, int prec, bool persistent, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (persistent && launch_fill_i32(a.queue, kQueueSlots, 0, s) != hipSuccess)
    return hipErrorLaunchFailure;
  const dim3 grid(persistent ? persistent_blocks(a.n, 4) : ceil_div(a.n, 4)), block(256);
#define LETKF_GRAM_LP(KP_, PR_)                                                               \
  if (kp == KP_ && prec == PR_) {                                                            \
    if (persistent)                                                                          \
      hipLaunchKernelGGL((k_gram_lp<KP_, PR_, true>), grid, block, 0, s, a);                  \
    else                                                                                     \
      hipLaunchKernelGGL((k_gram_lp<KP_, PR_, false>), grid, block, 0, s, a);                 \
    return hipGetLastError();                                                                \
  }
  LETKF_GRAM_LP(16, 1)
  LETKF_GRAM_LP(32, 1)
  LETKF_GRAM_LP(64, 1)
  LETKF_GRAM_LP(16, 2)
  LETKF_GRAM_LP(32, 2)
  LETKF_GRAM_LP(64, 2)
#undef LETKF_GRAM_LP
  return hipErrorInvalidValue;
}

}  // namespace letkf
