// The fused form of an analysis: the localized Gram matrix (k_gram.h,
// k_gram_lp.h), the eigensolve, transform and update (k_xf.h) of every point
// of one or several problems in one persistent launch.
//
// Each block is one wavefront that takes items of 64 / KP consecutive points
// from the per-XCD work queues (neighbouring points share observations, so an
// XCD's L2 keeps serving them), forms the items' C one point after another
// as packed upper triangles in LDS (16.6 KB at KP = 64, within the
// eigensolve's own LDS, which it shares) and b in its own slot of global
// memory, then runs the eigensolve and update on the item, one point per KP
// lanes.  C thus never leaves the CU (separate Gram and eigensolve launches
// send it through HBM and back); at KP = 64 the Householder vectors still
// wait in the block's slot through the divide and conquer, as in the
// separate kernel.  The whole analysis is one launch of device-filling size
// instead of two launches per slab, and the Gram's gathers overlap the FP64
// eigensolve of the other wavefronts on a SIMD.  The arithmetic is that of
// the separate kernels, so results are bitwise the same.
#pragma once
#include "common.h"
#include "launch.h"
#include "k_gram.h"
#include "k_gram_lp.h"
#include "k_xf.h"

namespace letkf {

template <int KP>
struct FusedLds {
  static constexpr int G = 64 / KP;
  static constexpr int NPK = KP * (KP + 1) / 2;   // packed upper triangle
  union {
    struct {                      // the Gram: its ring of local observations and
      int s[kRing];               // the item's C matrices
      double w[kRing];
      double c[G][NPK];
    } gram;
    XfLds<KP> xf;
  };
};

template <int KP, int PREC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_fused(BatchMap bm) {
  constexpr int G = 64 / KP;
  constexpr int NQ = KP / 16, NB = NQ * (NQ + 1) / 2;
  __shared__ FusedLds<KP> sh;
  const int lane = lane_id();
  const int seg = lane / KP, jj = lane % KP;
  double* slot_c = bm.C + (size_t)blockIdx.x * fused_slot_c(KP);
  double* slot_b = bm.b + (size_t)blockIdx.x * fused_slot_b(KP);
  const int nitems = (bm.n + G - 1) / G;
  for_each_queued(bm.queue, nitems, [&](int item) __attribute__((always_inline)) {
    const int p0 = item * G;
#pragma unroll 1
    for (int u = 0; u < G; ++u) {
      if (p0 + u < bm.n) {                     // uniform
        if constexpr (PREC == 0)
          gram_f64_point<KP, true>(bm, p0 + u, sh.gram.s, sh.gram.w, sh.gram.c[u],
                                   slot_b + u * KP);
        else
          gram_lp_point<KP, PREC, true>(bm, p0 + u, sh.gram.s, sh.gram.w, sh.gram.c[u],
                                        slot_b + u * KP);
      }
    }
    // b's stores are complete before any lane reads them, and C's LDS
    // stores are visible to every lane
    __threadfence_block();
    wave_lds_sync();
    // the lane's indices, redefined for every item: nothing derived from
    // them may be hoisted out of the loop (that would keep the eigensolve's
    // address arithmetic live through the Gram).  With one point per
    // wavefront (G = 1) the point and its descriptor are uniform and live in
    // scalar registers.
    const int sg = G == 1 ? 0 : opaque(seg), jl = opaque(jj);
    const int pl = p0 + sg;
    bool valid;
    EvdArgs e;
    if constexpr (G == 1)
      e = evd_args_uniform(bm, pl, valid);
    else
      e = evd_args_of(bm, pl, valid);
    const size_t pt = (size_t)e.pt0 + (valid ? pl : 0);
    XRows xr;
    if (e.xio) {             // the caller's member-major arrays, no point-major copy
      const double* xin = G == 1 ? uniform_copy(e.xio) : e.xio[0];
      const double* xout = G == 1 ? uniform_copy(e.xio + 1) : e.xio[1];
      xr.in = xin + pt;
      xr.out = const_cast<double*>(xout) + pt;
      xr.sc = (size_t)e.npts;
      xr.sj = (size_t)9 * e.npts;
    } else {
      xr.in = xr.out = e.xt + pt * 9 * e.k;
      xr.sc = (size_t)e.k;
      xr.sj = 1;
    }
    xf_body<KP, true>(e, valid, sh.gram.c[sg], slot_c + sg * NB * 256, slot_b + sg * KP, xr, sh.xf,
                      sg, jl);
    // the eigensolve's last reads of the slot and of LDS before the next
    // item's Gram writes them
    __threadfence_block();
    wave_lds_sync();
  });
}

template <int KP>
hipError_t launch_fused_kp(const BatchMap& bm, int prec, hipStream_t s) {
  if (bm.n <= 0) return hipSuccess;
  if (launch_fill_i32(bm.queue, kQueueSlots, 0, s) != hipSuccess) return hipErrorLaunchFailure;
  const int nitems = ceil_div(bm.n, 64 / KP);
  const dim3 grid(nitems < kFusedBlocks ? nitems : kFusedBlocks), block(64);
  if (prec == 0)
    hipLaunchKernelGGL((k_fused<KP, 0>), grid, block, 0, s, bm);
  else if (prec == 1)
    hipLaunchKernelGGL((k_fused<KP, 1>), grid, block, 0, s, bm);
  else if (prec == 2)
    hipLaunchKernelGGL((k_fused<KP, 2>), grid, block, 0, s, bm);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace letkf
