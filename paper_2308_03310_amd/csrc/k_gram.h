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
#pragma once
#include "common.h"
#include "k_window.h"
#include "launch.h"

namespace letkf {

template <int KQ>
struct GramAcc {
  static constexpr int NQ = KQ / 16;
  static constexpr int NB = NQ * (NQ + 1) / 2;
  double4_t c[NB];
  double bacc[NQ];
};

// Ring entry head + lane / 16 of one K = 4 step.  Every slot of the ring
// always holds a valid observation index and a finite weight (the ring is
// cleared when a point starts), so the reads need no branch; entries past the
// tail get weight 0 and contribute exact zeros.
struct RingRef {
  int s;
  double w, live;   // live: 1 for an entry before the tail, else 0
};

__device__ __forceinline__ RingRef ring_ref(const int* ring_s, const double* ring_w, int head,
                                            int tail) {
  const int idx = head + (lane_id() >> 4);
  const int slot = idx & (kRing - 1);
  RingRef r;
  r.s = ring_s[slot];
  r.w = ring_w[slot];
  r.live = idx < tail ? 1.0 : 0.0;
  return r;
}

// Operands of one step: the weight, the innovation and the lane's entries of
// the dy row of its ring entry.
template <int KQ>
struct GramStepF64 {
  double w, dv;
  double yv[KQ / 16];
};

template <int KQ>
__device__ __forceinline__ GramStepF64<KQ> gram_load(const GramArgs& g, const RingRef& r) {
  constexpr int NQ = KQ / 16;
  GramStepF64<KQ> st;
  st.w = r.w * r.live;
  st.dv = ldg(g.d, r.s);
  const double* row = g.Yb + (size_t)r.s * KQ + (lane_id() & 15);
#pragma unroll
  for (int I = 0; I < NQ; ++I) st.yv[I] = ldg(row, 16 * I);
  return st;
}

template <int KQ>
__device__ __forceinline__ void gram_accumulate(GramAcc<KQ>& acc, const GramStepF64<KQ>& st) {
  constexpr int NQ = KQ / 16;
  double av[NQ];
#pragma unroll
  for (int I = 0; I < NQ; ++I) {
    av[I] = st.w * st.yv[I];
    acc.bacc[I] = fma(av[I], st.dv, acc.bacc[I]);
  }
  int blk = 0;
#pragma unroll
  for (int I = 0; I < NQ; ++I) {
#pragma unroll
    for (int J = I; J < NQ; ++J) {
      acc.c[blk] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[I], st.yv[J], acc.c[blk], 0, 0, 0);
      ++blk;
    }
  }
}

// Every full step in the ring, software-pipelined over three stages: the
// ring entries of step h + 8 are read from LDS and the dy rows of step h + 4
// requested from memory while the MFMAs of step h run.  Two register sets
// are used in turn (a copy from one to the other would wait for the loads in
// flight); the sets read past the last full step are dropped.
template <int KQ>
__device__ __forceinline__ void gram_drain(GramAcc<KQ>& acc, const GramArgs& g, const int* ring_s,
                                           const double* ring_w, int& head, int tail) {
  const int n = (tail - head) >> 2;   // full steps
  if (n == 0) return;
  GramStepF64<KQ> sa = gram_load<KQ>(g, ring_ref(ring_s, ring_w, head, tail)), sb;
  RingRef ra = ring_ref(ring_s, ring_w, head + 4, tail), rb;
  // pairs of steps, one loop exit (exits between the two halves would give
  // the accumulators two homes and copies between them); the scheduling
  // barriers keep the compiler from moving the loads down to their use
  for (int i = 0; i + 1 < n; i += 2) {
    sb = gram_load<KQ>(g, ra);
    rb = ring_ref(ring_s, ring_w, head + 8, tail);
    __builtin_amdgcn_sched_barrier(0);
    gram_accumulate<KQ>(acc, sa);
    head += 4;
    sa = gram_load<KQ>(g, rb);
    ra = ring_ref(ring_s, ring_w, head + 8, tail);
    __builtin_amdgcn_sched_barrier(0);
    gram_accumulate<KQ>(acc, sb);
    head += 4;
  }
  if (n & 1) {
    gram_accumulate<KQ>(acc, sa);
    head += 4;
  }
}

// The localized Gram matrix and right-hand side of slab-local point pl, by
// one wavefront, into Cp (the point's NB upper blocks of 256, or with PACKED
// its packed upper triangle) and bp (KQ entries); ring_s / ring_w are its LDS
// ring of local observations.
// The loads of each candidate batch are issued before the ring filled by the
// previous batch is drained.
template <int KQ, bool PACKED = false>
__device__ __forceinline__ void gram_f64_point(const BatchMap& bm, int pl, int* ring_s,
                                               double* ring_w, double* Cp, double* bp) {
  constexpr int NQ = KQ / 16;
  constexpr int NB = NQ * (NQ + 1) / 2;
  const int lane = lane_id();
  // the point is the wavefront's: uniform, so its descriptor, window and
  // cell table go through scalar registers and scalar loads
  const int gidx = __builtin_amdgcn_readfirstlane(bm.g0 + pl);
  const int prob = bm.prefix ? __builtin_amdgcn_readfirstlane(find_problem(bm.prefix, bm.nprob, gidx))
                             : 0;
  // the problem's descriptor, copied once into scalar registers (or the
  // launch's inline one when there is no table)
  const GramArgs g = bm.g ? uniform_copy(bm.g + prob) : bm.g_inline;
  if (*g.abort_flag) return;
  const int pt = gidx - (bm.prefix ? bm.prefix[prob] : 0);  // point within its problem
  const int x = pt % g.nx, y = pt / g.nx;

  GramAcc<KQ> acc;
#pragma unroll
  for (int b = 0; b < NB; ++b) acc.c[b] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int I = 0; I < NQ; ++I) acc.bacc[I] = 0.0;

  // clear the ring: every slot then holds a valid observation index (0; the
  // walk below only runs when there are observations) and a finite weight
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
    // the next batch's loads (this batch's again when there is none)
    cand = ok2 ? load_candidate(g, nx.s, nx.s1) : load_candidate(g, cur.s, cur.s1);
    tail = ring_append(ring_s, ring_w, tail, s, w);
    wave_lds_sync();
    gram_drain<KQ>(acc, g, ring_s, ring_w, head, tail);
    wave_lds_sync();
    cur = nx;
    ok = ok2;
  }
  if (tail > head) gram_accumulate<KQ>(acc, gram_load<KQ>(g, ring_ref(ring_s, ring_w, head, tail)));

  // b: sum the four K-groups (lanes col, col+16, col+32, col+48).
#pragma unroll
  for (int I = 0; I < NQ; ++I) {
    double v = acc.bacc[I];
    v += xor_lane<16>(v);
    v += xor_lane<32>(v);
    if (lane < 16) bp[16 * I + lane] = v;
  }
  // C blocks: the f64 16x16x4 accumulator gives lane l, element r the entry
  // (row 4*r + l/16, column l%16) of each block.
  const int e = lane >> 4, col = lane & 15;
  store_gram_blocks<KQ, PACKED>(
      Cp, [&](int b, int r) { return acc.c[b][r]; }, [&](int r) { return 4 * r + e; }, col);
}

}  // namespace letkf
