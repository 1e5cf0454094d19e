// Localized Gram matrix and right-hand side per grid point in reduced
// precision (the FP32 and BF16 forms): the same computation as k_gram_f64,
//     C = sum_j w_j dy_j dy_j^T,   b = sum_j w_j d_j dy_j,
// with the forecast-observation perturbations dy (rounded after the FP64
// mean subtraction) and the weighted operand w_j dy_j in FP32 or BF16, and
// FP32 accumulation on MFMA:
//   FP32: v_mfma_f32_16x16x4f32      (4 local observations per K-step)
//   BF16: v_mfma_f32_16x16x32_bf16   (32 local observations per K-step, the
//         double-K form of gfx950)
// C and b are written as FP64 for the FP64 eigensolve.
#pragma once
#include <type_traits>

#include "common.h"
#include "k_window.h"
#include "launch.h"

namespace letkf {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// Ring entries per lane and step: FP32 1 (K = 4 over the four 16-lane
// groups), BF16 8 (K = 32).
template <int PREC>
constexpr int lp_entries() {
  return PREC == 1 ? 1 : 8;
}

// Accumulator element r of lane l of a 16x16 f32 MFMA block holds row
// f32_acc_row(l, r), column l % 16.
__device__ __forceinline__ int f32_acc_row(int l, int r) { return 4 * (l >> 4) + r; }

template <int KQ, int PREC>
struct GramAccLp {
  static constexpr int NQ = KQ / 16;
  static constexpr int NB = NQ * (NQ + 1) / 2;
  float4_t c[NB];
  float bacc[NQ];
};

// Ring entries of one step: R per lane (FP32: entry head + lane / 16; BF16:
// entries head + 8 (lane / 16) + t, t < 8).  Every ring slot holds a valid
// observation index and a finite weight (cleared when a point starts), so
// the reads need no branch; entries past the tail get weight 0.
template <int R>
struct RingRefs {
  int s[R];
  float w[R], live[R];
};

template <int R>
__device__ __forceinline__ RingRefs<R> ring_refs(const int* ring_s, const double* ring_w,
                                                 int head, int tail) {
  RingRefs<R> r;
  const int base = head + R * (lane_id() >> 4);
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int idx = base + t;
    const int slot = idx & (kRing - 1);
    r.s[t] = ring_s[slot];
    r.w[t] = (float)ring_w[slot];
    r.live[t] = idx < tail ? 1.f : 0.f;
  }
  return r;
}

// Raw operands of one step as loaded: weights, innovations and the lane's
// entries of the dy rows (FP32 values or BF16 bit patterns).
template <int KQ, int R, typename E>
struct GramStepLp {
  float w[R], dv[R];
  E y[R][KQ / 16];
};

template <int KQ, int R, typename E>
__device__ __forceinline__ GramStepLp<KQ, R, E> gram_load_lp(const GramArgs& g,
                                                             const RingRefs<R>& r) {
  constexpr int NQ = KQ / 16;
  const E* Y = reinterpret_cast<const E*>(g.Ylp);
  const int col = lane_id() & 15;
  GramStepLp<KQ, R, E> st;
#pragma unroll
  for (int t = 0; t < R; ++t) {
    st.w[t] = r.w[t] * r.live[t];
    st.dv[t] = (float)ldg(g.d, r.s[t]);
    const E* row = Y + (size_t)r.s[t] * KQ + col;
#pragma unroll
    for (int I = 0; I < NQ; ++I) st.y[t][I] = ldg(row, 16 * I);
  }
  return st;
}

// FP32: one entry per 16-lane group, K = 4.
template <int KQ>
__device__ __forceinline__ void gram_accumulate_lp(GramAccLp<KQ, 1>& acc,
                                                   const GramStepLp<KQ, 1, float>& st) {
  constexpr int NQ = KQ / 16;
  float av[NQ];
#pragma unroll
  for (int I = 0; I < NQ; ++I) {
    av[I] = st.w[0] * st.y[0][I];
    acc.bacc[I] = fmaf(av[I], st.dv[0], acc.bacc[I]);
  }
  int blk = 0;
#pragma unroll
  for (int I = 0; I < NQ; ++I) {
#pragma unroll
    for (int J = I; J < NQ; ++J) {
      acc.c[blk] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[I], st.y[0][J], acc.c[blk], 0, 0, 0);
      ++blk;
    }
  }
}

// BF16: eight entries per 16-lane group, K = 32; the weighted operand is
// rounded to BF16 and the right-hand side accumulates that rounded value.
// A and B take the lane's entries in the same order, so the sum over K is
// the same whatever order the instruction gives the eight.
template <int KQ>
__device__ __forceinline__ void gram_accumulate_lp(GramAccLp<KQ, 2>& acc,
                                                   const GramStepLp<KQ, 8, unsigned short>& st) {
  constexpr int NQ = KQ / 16;
  bf16x8_t A[NQ], B[NQ];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
#pragma unroll
    for (int I = 0; I < NQ; ++I) {
      const unsigned short ab = to_bf16(st.w[t] * from_bf16(st.y[t][I]));
      A[I][t] = __builtin_bit_cast(__bf16, ab);
      B[I][t] = __builtin_bit_cast(__bf16, st.y[t][I]);
      acc.bacc[I] = fmaf(from_bf16(ab), st.dv[t], acc.bacc[I]);
    }
  }
  int blk = 0;
#pragma unroll
  for (int I = 0; I < NQ; ++I) {
#pragma unroll
    for (int J = I; J < NQ; ++J) {
      acc.c[blk] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[I], B[J], acc.c[blk], 0, 0, 0);
      ++blk;
    }
  }
}

// Every full step in the ring, pipelined as in the FP64 kernel: ring entries
// two steps ahead, dy rows one step ahead, MFMAs of the current step.
template <int KQ, int PREC>
__device__ __forceinline__ void gram_drain_lp(GramAccLp<KQ, PREC>& acc, const GramArgs& g,
                                              const int* ring_s, const double* ring_w, int& head,
                                              int tail) {
  constexpr int R = lp_entries<PREC>();
  constexpr int STEP = 4 * R;
  typedef typename std::conditional<PREC == 1, float, unsigned short>::type E;
  const int n = (tail - head) / STEP;
  if (n == 0) return;
  GramStepLp<KQ, R, E> sa = gram_load_lp<KQ, R, E>(g, ring_refs<R>(ring_s, ring_w, head, tail)), sb;
  RingRefs<R> ra = ring_refs<R>(ring_s, ring_w, head + STEP, tail), rb;
  for (int i = 0; i + 1 < n; i += 2) {
    sb = gram_load_lp<KQ, R, E>(g, ra);
    rb = ring_refs<R>(ring_s, ring_w, head + 2 * STEP, tail);
    __builtin_amdgcn_sched_barrier(0);
    gram_accumulate_lp<KQ>(acc, sa);
    head += STEP;
    sa = gram_load_lp<KQ, R, E>(g, rb);
    ra = ring_refs<R>(ring_s, ring_w, head + 2 * STEP, tail);
    __builtin_amdgcn_sched_barrier(0);
    gram_accumulate_lp<KQ>(acc, sb);
    head += STEP;
  }
  if (n & 1) {
    gram_accumulate_lp<KQ>(acc, sa);
    head += STEP;
  }
}

// The point routine of k_gram_f64 (k_gram.h) in reduced precision: slab-local
// point pl by one wavefront, into Cp (NB upper blocks, or with PACKED the
// packed upper triangle) and bp (KQ entries).
template <int KQ, int PREC, bool PACKED = false>
__device__ __forceinline__ void gram_lp_point(const BatchMap& bm, int pl, int* ring_s,
                                              double* ring_w, double* Cp, double* bp) {
  constexpr int NQ = KQ / 16;
  constexpr int NB = NQ * (NQ + 1) / 2;
  constexpr int R = lp_entries<PREC>();
  typedef typename std::conditional<PREC == 1, float, unsigned short>::type E;
  const int lane = lane_id();
  // the point is the wavefront's: uniform (scalar registers and loads)
  const int gidx = __builtin_amdgcn_readfirstlane(bm.g0 + pl);
  const int prob = bm.prefix ? __builtin_amdgcn_readfirstlane(find_problem(bm.prefix, bm.nprob, gidx))
                             : 0;
  // the problem's descriptor, copied once into scalar registers (or the
  // launch's inline one when there is no table)
  const GramArgs g = bm.g ? uniform_copy(bm.g + prob) : bm.g_inline;
  if (*g.abort_flag) return;
  const int pt = gidx - (bm.prefix ? bm.prefix[prob] : 0);
  const int x = pt % g.nx, y = pt / g.nx;

  GramAccLp<KQ, PREC> acc;
#pragma unroll
  for (int b = 0; b < NB; ++b) acc.c[b] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int I = 0; I < NQ; ++I) acc.bacc[I] = 0.f;

  ring_s[lane] = 0;
  ring_s[lane + 64] = 0;
  ring_w[lane] = 0.0;
  ring_w[lane + 64] = 0.0;
  wave_lds_sync();

  WindowCursor cur;
  bool ok = window_begin(cur, g, x, y);
  Candidate cand{0, 0, 0.0};
  if (ok) cand = load_candidate(g, cur.s, cur.s1);
  int head = 0, tail = 0;
  while (ok) {
    const int s = cur.s + lane;
    const double w = candidate_weight(cand, g, x, y, s < cur.s1);
    WindowCursor nx = cur;
    const bool ok2 = window_next_batch(nx, g);
    cand = ok2 ? load_candidate(g, nx.s, nx.s1) : load_candidate(g, cur.s, cur.s1);
    tail = ring_append(ring_s, ring_w, tail, s, w);
    wave_lds_sync();
    gram_drain_lp<KQ, PREC>(acc, g, ring_s, ring_w, head, tail);
    wave_lds_sync();
    cur = nx;
    ok = ok2;
  }
  if (tail > head)
    gram_accumulate_lp<KQ>(acc, gram_load_lp<KQ, R, E>(g, ring_refs<R>(ring_s, ring_w, head, tail)));

#pragma unroll
  for (int I = 0; I < NQ; ++I) {
    double v = (double)acc.bacc[I];
    v += xor_lane<16>(v);
    v += xor_lane<32>(v);
    if (lane < 16) bp[16 * I + lane] = v;
  }
  const int col = lane & 15;
  store_gram_blocks<KQ, PACKED>(
      Cp, [&](int b, int r) { return (double)acc.c[b][r]; },
      [&](int r) { return f32_acc_row(lane, r); }, col);
}

}  // namespace letkf
