// Localized Gram matrix and right-hand side per grid point in reduced
// precision (the FP32 and BF16 forms): the same computation as k_gram_f64,
//     C = sum_j w_j dy_j dy_j^T,   b = sum_j w_j d_j dy_j,
// with the forecast-observation perturbations dy (rounded after the FP64
// mean subtraction) and the weighted operand w_j dy_j in FP32 or BF16, and
// FP32 accumulation on MFMA:
//   FP32: v_mfma_f32_16x16x4f32      (4 local observations per K-step)
//   BF16: v_mfma_f32_16x16x16bf16_1k (16 local observations per K-step)
// C and b are written as FP64 for the FP64 eigensolve.
#include "common.h"
#include "launch.h"

namespace letkf {

typedef short short4_t __attribute__((ext_vector_type(4)));

// Accumulator element r of lane l of a 16x16 f32 MFMA block holds row
// f32_acc_row(l, r), column l % 16.
__device__ __forceinline__ int f32_acc_row(int l, int r) { return 4 * (l >> 4) + r; }


__device__ __forceinline__ double gc_weight(double r, double invc) {
  const double z = r * invc;
  if (z <= 1.0) return (((-0.25 * z + 0.5) * z + 0.625) * z - 5.0 / 3.0) * z * z + 1.0;
  if (z < 2.0)
    return ((((z / 12.0 - 0.5) * z + 0.625) * z + 5.0 / 3.0) * z - 5.0) * z + 4.0 - 2.0 / (3.0 * z);
  return 0.0;
}

__device__ __forceinline__ int cell_intervals_lp(int c, int R, int n, int cb, int nc, int* lo,
                                                 int* hi) {
  if (R < 0 || 2 * R + 1 >= n) {
    lo[0] = 0;
    hi[0] = nc - 1;
    return 1;
  }
  int a = c - R, b = c + R;
  if (a >= 0 && b < n) {
    lo[0] = a / cb;
    hi[0] = b / cb;
    return 1;
  }
  int lo1, hi2;
  if (a < 0) {
    lo1 = (a + n) / cb;
    hi2 = b / cb;
  } else {
    lo1 = a / cb;
    hi2 = (b - n) / cb;
  }
  if (hi2 + 1 >= lo1) {
    lo[0] = 0;
    hi[0] = nc - 1;
    return 1;
  }
  lo[0] = 0;
  hi[0] = hi2;
  lo[1] = lo1;
  hi[1] = nc - 1;
  return 2;
}

template <int KQ, int PREC>
struct GramAccLp {
  static constexpr int NQ = KQ / 16;
  static constexpr int NB = NQ * (NQ + 1) / 2;
  float4_t c[NB];
  float bacc[NQ];
};

// FP32: four ring entries per step, one per 16-lane group.
template <int KQ>
__device__ __forceinline__ void gram_step_f32(GramAccLp<KQ, 1>& acc, const GramArgs& g,
                                              const int* ring_s, const double* ring_w, int head,
                                              int tail) {
  constexpr int NQ = KQ / 16;
  const int lane = lane_id();
  const int e = lane >> 4, col = lane & 15;
  const int idx = head + e;
  float w = 0.f, dv = 0.f;
  float yv[NQ], av[NQ];
#pragma unroll
  for (int I = 0; I < NQ; ++I) yv[I] = 0.f;
  if (idx < tail) {
    const int s = ring_s[idx & 127];
    w = (float)ring_w[idx & 127];
    dv = (float)g.d[s];
    const float* row = reinterpret_cast<const float*>(g.Ylp) + (size_t)s * KQ + col;
#pragma unroll
    for (int I = 0; I < NQ; ++I) yv[I] = row[16 * I];
  }
#pragma unroll
  for (int I = 0; I < NQ; ++I) {
    av[I] = w * yv[I];
    acc.bacc[I] = fmaf(av[I], dv, acc.bacc[I]);
  }
  int blk = 0;
#pragma unroll
  for (int I = 0; I < NQ; ++I) {
#pragma unroll
    for (int J = I; J < NQ; ++J) {
      acc.c[blk] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[I], yv[J], acc.c[blk], 0, 0, 0);
      ++blk;
    }
  }
}

// BF16: sixteen ring entries per step, four per 16-lane group.
template <int KQ>
__device__ __forceinline__ void gram_step_bf16(GramAccLp<KQ, 2>& acc, const GramArgs& g,
                                               const int* ring_s, const double* ring_w, int head,
                                               int tail) {
  constexpr int NQ = KQ / 16;
  const int lane = lane_id();
  const int q = lane >> 4, col = lane & 15;
  short4_t A[NQ], B[NQ];
  const unsigned short* Yh = reinterpret_cast<const unsigned short*>(g.Ylp);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int idx = head + 4 * q + t;
    float w = 0.f, dv = 0.f;
    unsigned short yb[NQ];
#pragma unroll
    for (int I = 0; I < NQ; ++I) yb[I] = 0;
    if (idx < tail) {
      const int s = ring_s[idx & 127];
      w = (float)ring_w[idx & 127];
      dv = (float)g.d[s];
      const unsigned short* row = Yh + (size_t)s * KQ + col;
#pragma unroll
      for (int I = 0; I < NQ; ++I) yb[I] = row[16 * I];
    }
#pragma unroll
    for (int I = 0; I < NQ; ++I) {
      const unsigned short ab = to_bf16(w * from_bf16(yb[I]));
      A[I][t] = (short)ab;
      B[I][t] = (short)yb[I];
      acc.bacc[I] = fmaf(from_bf16(ab), dv, acc.bacc[I]);
    }
  }
  int blk = 0;
#pragma unroll
  for (int I = 0; I < NQ; ++I) {
#pragma unroll
    for (int J = I; J < NQ; ++J) {
      acc.c[blk] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[I], B[J], acc.c[blk], 0, 0, 0);
      ++blk;
    }
  }
}

template <int KQ, int PREC>
__device__ __forceinline__ void gram_lp_point(const BatchMap& bm, int pl, int* ring_s,
                                              double* ring_w) {
  constexpr int NQ = KQ / 16;
  constexpr int NB = NQ * (NQ + 1) / 2;
  constexpr int STEP = PREC == 1 ? 4 : 16;
  const int lane = lane_id();
  const int gidx = bm.g0 + pl;
  const int prob = find_problem(bm.prefix, bm.nprob, gidx);
  const GramArgs g = bm.g[prob];   // copied once: fields stay in registers
  if (*g.abort_flag) return;
  const int pt = gidx - bm.prefix[prob];
  const int x = pt % g.nx, y = pt / g.nx;

  GramAccLp<KQ, PREC> acc;
#pragma unroll
  for (int b = 0; b < NB; ++b) acc.c[b] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int I = 0; I < NQ; ++I) acc.bacc[I] = 0.f;

  int xlo[2], xhi[2], ylo[2], yhi[2];
  const int nxi = cell_intervals_lp(x, g.R, g.nx, g.cb, g.ncx, xlo, xhi);
  const int nyi = cell_intervals_lp(y, g.R, g.ny, g.cb, g.ncy, ylo, yhi);
  int head = 0, tail = 0;
  for (int yi = 0; yi < nyi; ++yi) {
    for (int cy = ylo[yi]; cy <= yhi[yi]; ++cy) {
      for (int xi = 0; xi < nxi; ++xi) {
        const int s0 = g.cell_start[cy * g.ncx + xlo[xi]];
        const int s1 = g.cell_start[cy * g.ncx + xhi[xi] + 1];
        for (int base = s0; base < s1; base += 64) {
          const int s = base + lane;
          double w = 0.0;
          if (s < s1) {
            int dx = abs(x - g.ox[s]);
            dx = min(dx, g.nx - dx);
            int dy = abs(y - g.oy[s]);
            dy = min(dy, g.ny - dy);
            const double r2d = (double)(dx * dx + dy * dy);
            const double rv = g.rinv[s];
            if (rv > 0.0 && r2d <= g.cut2) {
              const double gl = g.loc == 0 ? exp(-r2d * g.inv2L2)
                                           : (g.loc == 1 ? gc_weight(sqrt(r2d), g.invL) : 1.0);
              w = gl * rv;
            }
          }
          const bool in = w > 0.0;
          const uint64_t mask = __ballot(in);
          const int pos = __popcll(mask & ((1ull << lane) - 1ull));
          if (in) {
            ring_s[(tail + pos) & 127] = s;
            ring_w[(tail + pos) & 127] = w;
          }
          tail += __popcll(mask);
          wave_lds_sync();
          while (tail - head >= STEP) {
            if constexpr (PREC == 1)
              gram_step_f32<KQ>(acc, g, ring_s, ring_w, head, tail);
            else
              gram_step_bf16<KQ>(acc, g, ring_s, ring_w, head, tail);
            head += STEP;
          }
          wave_lds_sync();
        }
      }
    }
  }
  if (tail > head) {
    if constexpr (PREC == 1)
      gram_step_f32<KQ>(acc, g, ring_s, ring_w, head, tail);
    else
      gram_step_bf16<KQ>(acc, g, ring_s, ring_w, head, tail);
  }

#pragma unroll
  for (int I = 0; I < NQ; ++I) {
    double v = (double)acc.bacc[I];
    v += xor_lane<16>(v);
    v += xor_lane<32>(v);
    if (lane < 16) bm.b[(size_t)pl * KQ + 16 * I + lane] = v;
  }
  double* out = bm.C + (size_t)pl * NB * 256;
  const int col = lane & 15;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
#pragma unroll
    for (int r = 0; r < 4; ++r) out[b * 256 + f32_acc_row(lane, r) * 16 + col] = (double)acc.c[b][r];
  }
}

// Grid and persistent forms, as for k_gram_f64.
template <int KQ, int PREC, bool PERSIST>
__global__ __launch_bounds__(256) void k_gram_lp(BatchMap bm) {
  __shared__ int s_ring[4][128];
  __shared__ double w_ring[4][128];
  const int wid = threadIdx.x >> 6;
  if constexpr (!PERSIST) {
    const int pl = xcd_remap(blockIdx.x, gridDim.x) * 4 + wid;
    if (pl < bm.n) gram_lp_point<KQ, PREC>(bm, pl, s_ring[wid], w_ring[wid]);
  } else {
    for_each_queued_point(bm, [&](int pl) { gram_lp_point<KQ, PREC>(bm, pl, s_ring[wid], w_ring[wid]); });
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
