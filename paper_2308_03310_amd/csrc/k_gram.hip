// Localized Gram matrix and right-hand side per grid point, FP64 on MFMA.
//
// For grid point x, with local observations j (R-localization, Sec. II-B):
//     w_j = g(r_xj) / sigma_j^2                     diagonal of G o R^-1
//     C   = sum_j w_j dy_j dy_j^T                   dY^T R_loc^-1 dY   (eq. letkf_q)
//     b   = sum_j w_j (yo_j - ybar_j) dy_j          dY^T R_loc^-1 (yo - ybar) (eq. letkf_wa)
// dy_j is row j of the forecast-observation perturbations (length k).
//
// One wavefront per grid point.  The wavefront walks the observation cells
// that intersect the point's window, tests 64 candidates at a time, and
// appends the local ones (slot, weight) to a small ring in LDS; every four
// ring entries feed one K=4 step of v_mfma_f64_16x16x4f64 per upper 16x16
// block of C.  The local observation set is never materialized in HBM.
#include "common.h"
#include "launch.h"

namespace letkf {

__device__ __forceinline__ double gaspari_cohn(double r, double invc) {
  // Gaspari & Cohn (1999) eq. (4.10), half-width c: zero for r >= 2c.
  const double z = r * invc;
  if (z <= 1.0) {
    return (((-0.25 * z + 0.5) * z + 0.625) * z - 5.0 / 3.0) * z * z + 1.0;
  }
  if (z < 2.0) {
    return ((((z / 12.0 - 0.5) * z + 0.625) * z + 5.0 / 3.0) * z - 5.0) * z + 4.0 - 2.0 / (3.0 * z);
  }
  return 0.0;
}

// Cell intervals (at most two, merged when they touch) covering lattice
// coordinates [c - R, c + R] modulo n.
__device__ __forceinline__ int cell_intervals(int c, int R, int n, int cb, int nc, int* lo, int* hi) {
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

template <int KQ>
struct GramAcc {
  static constexpr int NQ = KQ / 16;
  static constexpr int NB = NQ * (NQ + 1) / 2;
  double4_t c[NB];
  double bacc[NQ];
};

template <int KQ>
__device__ __forceinline__ void gram_step(GramAcc<KQ>& acc, const GramArgs& g, const int* ring_s,
                                          const double* ring_w, int head, int tail) {
  constexpr int NQ = KQ / 16;
  const int lane = lane_id();
  const int e = lane >> 4, col = lane & 15;
  const int idx = head + e;
  // Entries past the tail (last, partial step) contribute exact zeros.
  double w = 0.0, dv = 0.0;
  double yv[NQ], av[NQ];
#pragma unroll
  for (int I = 0; I < NQ; ++I) yv[I] = 0.0;
  if (idx < tail) {
    const int s = ring_s[idx & 127];
    w = ring_w[idx & 127];
    dv = g.d[s];
    const double* row = g.Yb + (size_t)s * KQ + col;
#pragma unroll
    for (int I = 0; I < NQ; ++I) yv[I] = row[16 * I];
  }
#pragma unroll
  for (int I = 0; I < NQ; ++I) {
    av[I] = w * yv[I];
    acc.bacc[I] = fma(av[I], dv, acc.bacc[I]);
  }
  int blk = 0;
#pragma unroll
  for (int I = 0; I < NQ; ++I) {
#pragma unroll
    for (int J = I; J < NQ; ++J) {
      acc.c[blk] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[I], yv[J], acc.c[blk], 0, 0, 0);
      ++blk;
    }
  }
}

// The localized Gram matrix and right-hand side of slab-local point pl, by
// one wavefront; ring_s / ring_w are its LDS ring of local observations.
template <int KQ>
__device__ __forceinline__ void gram_f64_point(const BatchMap& bm, int pl, int* ring_s,
                                               double* ring_w) {
  constexpr int NQ = KQ / 16;
  constexpr int NB = NQ * (NQ + 1) / 2;
  const int lane = lane_id();
  const int gidx = bm.g0 + pl;
  const int prob = find_problem(bm.prefix, bm.nprob, gidx);
  const GramArgs g = bm.g[prob];   // copied once: fields stay in registers
  if (*g.abort_flag) return;
  const int pt = gidx - bm.prefix[prob];  // point within its problem
  const int x = pt % g.nx, y = pt / g.nx;

  GramAcc<KQ> acc;
#pragma unroll
  for (int b = 0; b < NB; ++b) acc.c[b] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int I = 0; I < NQ; ++I) acc.bacc[I] = 0.0;

  int xlo[2], xhi[2], ylo[2], yhi[2];
  const int nxi = cell_intervals(x, g.R, g.nx, g.cb, g.ncx, xlo, xhi);
  const int nyi = cell_intervals(y, g.R, g.ny, g.cb, g.ncy, ylo, yhi);
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
            const int r2 = dx * dx + dy * dy;
            const double rv = g.rinv[s];
            const double r2d = (double)r2;
            if (rv > 0.0 && r2d <= g.cut2) {
              double gl;
              if (g.loc == 0) {
                gl = exp(-r2d * g.inv2L2);
              } else if (g.loc == 1) {
                gl = gaspari_cohn(sqrt(r2d), g.invL);
              } else {
                gl = 1.0;
              }
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
          while (tail - head >= 4) {
            gram_step<KQ>(acc, g, ring_s, ring_w, head, tail);
            head += 4;
          }
          wave_lds_sync();
        }
      }
    }
  }
  if (tail > head) gram_step<KQ>(acc, g, ring_s, ring_w, head, tail);

  // b: sum the four K-groups (lanes col, col+16, col+32, col+48).
#pragma unroll
  for (int I = 0; I < NQ; ++I) {
    double v = acc.bacc[I];
    v += xor_lane<16>(v);
    v += xor_lane<32>(v);
    if (lane < 16) bm.b[(size_t)pl * KQ + 16 * I + lane] = v;
  }
  // C blocks: the f64 16x16x4 accumulator gives lane l, element r the entry
  // (row 4*r + l/16, column l%16) of each block.
  double* out = bm.C + (size_t)pl * NB * 256;
  const int e = lane >> 4, col = lane & 15;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
#pragma unroll
    for (int r = 0; r < 4; ++r) out[b * 256 + (4 * r + e) * 16 + col] = acc.c[b][r];
  }
}

// Grid form: one wavefront per point, four points per block, blocks remapped
// so that neighbouring points (which share observations) stay on one XCD.
// Persistent form: a device-filling grid whose wavefronts take points from
// per-XCD work queues over contiguous eighths of the slab and, once their
// own eighth is done, from the others' (load balance when the local
// observation counts differ widely between points).
template <int KQ, bool PERSIST>
__global__ __launch_bounds__(256) void k_gram_f64(BatchMap bm) {
  __shared__ int s_ring[4][128];
  __shared__ double w_ring[4][128];
  const int wid = threadIdx.x >> 6;
  if constexpr (!PERSIST) {
    const int pl = xcd_remap(blockIdx.x, gridDim.x) * 4 + wid;
    if (pl < bm.n) gram_f64_point<KQ>(bm, pl, s_ring[wid], w_ring[wid]);
  } else {
    for_each_queued_point(bm, [&](int pl) { gram_f64_point<KQ>(bm, pl, s_ring[wid], w_ring[wid]); });
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
