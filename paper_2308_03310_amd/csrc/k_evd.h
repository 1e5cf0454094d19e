// Batched symmetric eigensolve of the k x k ensemble-space matrices and the
// LETKF transform / update, FP64, for gfx950.
//
// Per grid point (Sec. II-B):
//     Q     = ((k-1)/rho) I + C                      eq. (letkf_q), inflated
//     Q     = V diag(lam) V^T                         EVD of Q (Sec. II-B, Sec. III)
//     wbar  = V diag(1/lam) V^T b                     eq. (letkf_wa)
//     W     = sqrt(k-1) V diag(lam^-1/2) V^T          eq. (letkf_dwa)
//     X^a   = xbar 1^T + dX (wbar 1^T + W)            eq. (letkf_xa), 9 components share W
//
// Eigensolver (the batched EVD of Sec. III, one matrix per KP lanes of a
// wavefront, 64/KP matrices per wavefront):
//   1. Householder reduction to tridiagonal form T = H^T Q H (Golub & Van
//      Loan, Matrix Computations, Sec. 8.3.1), one matrix row per lane in
//      registers; the reflector of step i and p = tau A v are broadcast
//      through LDS and the symmetric rank-2 update runs in-lane;
//   2. eigenpairs of T by divide and conquer (k_dc.h): T = Q_T diag(lam) Q_T^T;
//   3. back-transformation V = H Q_T = H_0 (H_1 (.. H_{n-3} Q_T)), one column
//      of V per lane.
// Sizes below KP are padded with decoupled rows (unit rows in mode 0, where
// every eigenvalue is at least alpha; zero rows in mode 1): their couplings in
// T are exactly zero, so every merge that involves them is trivial or deflates
// them.
#pragma once
#include "common.h"
#include "launch.h"
#include "k_dc.h"

namespace letkf {

// Target waves per SIMD for the register allocator of the eigensolve kernel.
#ifndef LETKF_EVD_WAVES
#define LETKF_EVD_WAVES 2
#endif

// LDS per block: the matrix area (input staging, then the merge matrices of
// the divide and conquer, then the Householder vectors with row stride KP,
// then V in natural layout with row stride KP+1) and a union of the
// tridiagonalization's broadcast vectors, the divide-and-conquer work arrays
// and the transform's 5 x KP area (Lambda^-1 V^T b, then dX and dX V for up
// to five of the nine components at a time).  The tridiagonal (d, e) stays
// in lane registers, and each reflector's tau is recovered from its vector.
constexpr int kCompGroup = 5;

#ifndef LETKF_REFL_REG_MAX
#define LETKF_REFL_REG_MAX 32
#endif
template <int KP>
struct EvdLds {
  static constexpr int G = 64 / KP;
  static constexpr int S = KP + 1;   // row stride: 16 consecutive rows hit distinct banks
  double mat[G][KP * S];
  union {
    struct {                         // tridiagonalization: broadcast vectors
      double vb[G][KP];
      double wb[G][KP];
    };
    DcLds<KP> dc[G];                 // divide and conquer
    double dxu[G][kCompGroup][KP];   // transform and update
  };
};

// Value of x held by lane SRC (compile-time) of this lane's KP-lane group.
// With one or two groups per wavefront it comes from v_readlane (a VALU read
// into scalar registers, no LDS round trip), the group's copy picked per
// lane; with more, from a lane shuffle.
template <int KP, int SRC>
__device__ __forceinline__ double group_read_c(double x) {
  static_assert(SRC >= 0 && SRC < KP, "group_read_c: source lane");
  if constexpr (KP == 64) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), SRC),
                            __builtin_amdgcn_readlane(__double2loint(x), SRC));
  } else if constexpr (KP == 32) {
    const double v0 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), SRC),
                                       __builtin_amdgcn_readlane(__double2loint(x), SRC));
    const double v1 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), 32 + SRC),
                                       __builtin_amdgcn_readlane(__double2loint(x), 32 + SRC));
    return lane_id() < 32 ? v0 : v1;
  } else {
    return __shfl(x, SRC, KP);
  }
}

// Marks the n values of x (n a multiple of 8) as redefined at this point, so
// that the arithmetic producing them cannot be moved below it.  Instruction
// selection otherwise places side-effect-free arithmetic anywhere in a long
// straight-line region (the unrolled Householder steps are one basic block),
// and sinking a step's updates or selects towards their last use keeps one
// copy per step live.
template <int N>
__device__ __forceinline__ void pin_regs(double* x) {
  static_assert(N % 8 == 0, "pin_regs: multiple of 8");
#pragma unroll
  for (int c = 0; c < N; c += 8)
    asm volatile("" : "+v"(x[c]), "+v"(x[c + 1]), "+v"(x[c + 2]), "+v"(x[c + 3]), "+v"(x[c + 4]),
                 "+v"(x[c + 5]), "+v"(x[c + 6]), "+v"(x[c + 7]));
}

// An integer the compiler cannot see through: LDS addresses derived from it
// are recomputed after each use point instead of being hoisted out of the
// unrolled loops (where every one of them would hold a VGPR).
__device__ __forceinline__ int opaque(int x) {
  asm volatile("v_mov_b32 %0, %1" : "=v"(x) : "v"(x));
  return x;
}

// Q = alpha I + C (mode 0, upper blocks mirrored; padded rows unit) or A
// (mode 1; padded rows zero, scaled by 2^-ex) into the matrix area; this
// lane's entry of b into bj (mode 0).  ex is 0 in mode 0.
template <int KP>
__device__ __forceinline__ void stage_matrix(const EvdArgs& e, EvdLds<KP>& sh, int seg, int jj,
                                             int pl, bool valid, double& bj, int& ex) {
  ex = 0;
  constexpr int NQ = KP / 16;
  constexpr int NB = NQ * (NQ + 1) / 2;
  constexpr int S = EvdLds<KP>::S;
  const int k = e.k;
  double* M = sh.mat[seg];
  if (e.mode == 0) {
    for (int c = 0; c < KP; ++c) M[jj * S + c] = 0.0;
    wave_lds_sync();
    if (valid) {
      // all of this lane's loads first (NB * 256 / KP values), then the LDS writes
      constexpr int PER = 256 / KP;
      const double* Cp = e.C + (size_t)pl * NB * 256 + jj;
      double val[NB * PER];
#pragma unroll
      for (int q = 0; q < NB * PER; ++q) val[q] = Cp[(q / PER) * 256 + (q % PER) * KP];
      int blk = 0;
#pragma unroll
      for (int I = 0; I < NQ; ++I) {
#pragma unroll
        for (int J = I; J < NQ; ++J) {
#pragma unroll
          for (int q = 0; q < PER; ++q) {
            const int t = jj + q * KP;
            const int r = t >> 4, c = t & 15;
            M[(16 * I + r) * S + 16 * J + c] = val[blk * PER + q];
            if (I != J) M[(16 * J + c) * S + 16 * I + r] = val[blk * PER + q];
          }
          ++blk;
        }
      }
    }
    wave_lds_sync();
    if (valid && jj < k)
      M[jj * S + jj] += e.alpha;
    else
      M[jj * S + jj] = 1.0;
    bj = (valid && jj < k) ? e.b[(size_t)pl * KP + jj] : 0.0;
  } else {
    // padded rows stay zero: their eigenvalue 0 never exceeds the largest
    // |eigenvalue| of the matrix, so it leaves the deflation tolerance of
    // every merge (which scales with that) at the matrix's own scale
    double amax = 0.0;
    for (int c = 0; c < KP; ++c) {
      double val = 0.0;
      if (valid && jj < k && c < k) {
        const int r0 = jj < c ? jj : c, c0 = jj < c ? c : jj;
        val = e.A[((size_t)pl * k + r0) * k + c0];
      }
      amax = fmax(amax, fabs(val));
      M[jj * S + c] = val;
    }
    // An exact power-of-two scaling brings the largest entry into [0.5, 1):
    // the hardware reciprocal and square-root estimates of the reduction and
    // the merges then see operands of moderate size whatever the matrix's
    // scale, and the eigenvalues are scaled back on output.  (Each lane
    // rescales only its own row, so no barrier is needed.)
    amax = group_max<KP>(amax);
    if (amax > 0.0 && __builtin_isfinite(amax)) {
      (void)frexp(amax, &ex);
      for (int c = 0; c < KP; ++c) M[jj * S + c] = ldexp(M[jj * S + c], -ex);
    }
  }
}


template <int KP>
__device__ __forceinline__ void load_rows(const double* M, int jj, double (&a)[KP]) {
  constexpr int S = KP + 1;
#pragma unroll
  for (int u = 0; u < KP; ++u) a[u] = M[jj * S + u];
}

constexpr int cmin(int x, int y) { return x < y ? x : y; }
constexpr int cmax(int x, int y) { return x > y ? x : y; }

// Entries [C0, C1) of an LDS vector (C0 even, 16-byte aligned base) into v[],
// two per read.
template <int KP, int C0, int C1>
__device__ __forceinline__ void load_pairs(double (&v)[KP], const double* src) {
#pragma unroll
  for (int c = C0; c < C1; c += 2) {
    const double2 t2 = *reinterpret_cast<const double2*>(src + c);
    v[c] = t2.x;
    v[c + 1] = t2.y;
  }
}

// Streaming forms for rows too long to hold beside a second vector in
// registers (KP = 64): the vector comes from LDS in chunks of CH entries,
// chunk CS + CH being read while chunk CS (already requested) is used, and no
// instruction crosses a chunk boundary, so at most two chunks are live.
//   pc[c % 4] += x[c] v[c] for c in [LO, KP)
template <int KP, int LO, int CS, int CH>
__device__ __forceinline__ void dot_stream(const double (&x)[KP], const double* vsrc,
                                           double (&v)[KP], double (&pc)[4]) {
  if constexpr (CS < KP) {
    constexpr int NS = CS + CH;
    if constexpr (NS < KP) load_pairs<KP, NS, cmin(NS + CH, KP)>(v, vsrc);
#pragma unroll
    for (int c = cmax(CS, LO); c < cmin(NS, KP); ++c) pc[c & 3] = fma(x[c], v[c], pc[c & 3]);
    __builtin_amdgcn_sched_barrier(0);
    dot_stream<KP, LO, NS, CH>(x, vsrc, v, pc);
  }
}

//   pc[c % 4] += x[c] v[c] for c in [LO, KP), nc[c % 4] += v[c]^2 for c in (LO, KP)
template <int KP, int LO, int CS, int CH>
__device__ __forceinline__ void dotn_stream(const double (&x)[KP], const double* vsrc,
                                            double (&v)[KP], double (&pc)[4], double (&nc)[4]) {
  if constexpr (CS < KP) {
    constexpr int NS = CS + CH;
    if constexpr (NS < KP) load_pairs<KP, NS, cmin(NS + CH, KP)>(v, vsrc);
#pragma unroll
    for (int c = cmax(CS, LO); c < cmin(NS, KP); ++c) pc[c & 3] = fma(x[c], v[c], pc[c & 3]);
#pragma unroll
    for (int c = cmax(CS, LO + 1); c < cmin(NS, KP); ++c) nc[c & 3] = fma(v[c], v[c], nc[c & 3]);
    __builtin_amdgcn_sched_barrier(0);
    dotn_stream<KP, LO, NS, CH>(x, vsrc, v, pc, nc);
  }
}

//   x[c] -= f v[c] for c in [LO, KP)
template <int KP, int LO, int CS, int CH>
__device__ __forceinline__ void axpy_stream(double (&x)[KP], const double* vsrc, double (&v)[KP],
                                            double f) {
  if constexpr (CS < KP) {
    constexpr int NS = CS + CH;
    if constexpr (NS < KP) load_pairs<KP, NS, cmin(NS + CH, KP)>(v, vsrc);
#pragma unroll
    for (int c = cmax(CS, LO); c < cmin(NS, KP); ++c) x[c] = fma(-f, v[c], x[c]);
    __builtin_amdgcn_sched_barrier(0);
    axpy_stream<KP, LO, NS, CH>(x, vsrc, v, f);
  }
}

//   x[c] -= vj w[c] + wj v[c] for c in [LO, KP)
template <int KP, int LO, int CS, int CH>
__device__ __forceinline__ void rank2_stream(double (&x)[KP], const double* vsrc,
                                             const double* wsrc, double (&v)[KP],
                                             double (&w)[KP], double vj, double wj) {
  if constexpr (CS < KP) {
    constexpr int NS = CS + CH;
    if constexpr (NS < KP) {
      load_pairs<KP, NS, cmin(NS + CH, KP)>(v, vsrc);
      load_pairs<KP, NS, cmin(NS + CH, KP)>(w, wsrc);
    }
#pragma unroll
    for (int c = cmax(CS, LO); c < cmin(NS, KP); ++c) x[c] = fma(-wj, v[c], fma(-vj, w[c], x[c]));
    __builtin_amdgcn_sched_barrier(0);
    rank2_stream<KP, LO, NS, CH>(x, vsrc, wsrc, v, w, vj, wj);
  }
}

// Householder tridiagonalization of the symmetric matrix whose row jj this
// lane holds in a[].  Step i annihilates A[i+2:, i] with H_i = I - tau v v^T,
// v = (0,..,0, 1, v_{i+2}, .., v_{n-1}); afterwards
//   d_j = T[j][j] and e_j = T[j+1][j] in registers of lane j (dj, ej),
//   a[i] = v_jj of step i for i < jj (the lane's entries of the reflectors).
// With p = tau A v and K = (tau/2) p.v the update A - v w^T - w v^T,
// w = p - K v, is A - v p^T - (p - 2K v) v^T: p is broadcast as soon as it
// is known and the reduction for K runs while it travels through LDS.
// Column i+1 of the updated row (the next step's x) is updated first and the
// next step's two column reductions (alpha, sigma) are started before the
// rest of the row, so their latency hides behind it.
// Step i of the reduction (a compile-time index so that a[] stays in
// registers at every size); alpha = A[i+1][i] and sig = sum_{j>i+1} A[j][i]^2
// come in from the step before and go out for the step after.
template <int KP, int i, bool STREAM, bool UNIT, class Sh>
__device__ __forceinline__ void tridiag_step(double (&a)[KP], Sh& sh, int seg, int jj,
                                             double& alpha, double& sig, double& ej,
                                             double* taus) {
  const int so = opaque(seg * KP);
  double* vb = &sh.vb[0][0] + so;
  double* pb = &sh.wb[0][0] + so;
  const double x = a[i];                                   // A[jj][i]
  const bool refl = sig != 0.0;                             // uniform per matrix
  // |x| = sqrt(alpha^2 + sig) with its reciprocal (refined estimates, for
  // column norms between 1e-154 and 1e154; a zero column takes no
  // reflection and the values are not used), beta = -sign(alpha) |x|.
  // UNIT: v = x / (alpha - beta), v_{i+1} = 1, tau = 1 + |alpha| / |x|
  // (1 / (alpha - beta) = sign(alpha) / (|alpha| + |x|)).  Otherwise v is
  // the column itself below i+1 and v_{i+1} = alpha - beta, tau = 2 / v^T v:
  // all of v but one entry is known before the norm, so v is broadcast and
  // A v formed (but for that entry's term) while the norm is computed.
  double rn, nrm, tau, vj, v1 = 1.0;
  if constexpr (UNIT) {
    rsqrt_sqrt(fma(alpha, alpha, sig), rn, nrm);
    tau = refl ? fma(fabs(alpha), rn, 1.0) : 0.0;
    const double inv = refl ? (alpha >= 0.0 ? 1.0 : -1.0) * frcp(fabs(alpha) + nrm) : 0.0;
    vj = jj == i + 1 ? 1.0 : (jj > i + 1 ? x * inv : 0.0);
    vb[jj] = vj;
  } else {
    vj = jj > i + 1 ? x : 0.0;
    vb[jj] = vj;                       // entry i+1 is 0 in LDS: its term is added apart
  }
  wave_lds_sync();
  if constexpr (!UNIT) {
    rsqrt_sqrt(fma(alpha, alpha, sig), rn, nrm);
    v1 = refl ? (alpha >= 0.0 ? 1.0 : -1.0) * (fabs(alpha) + nrm) : 0.0;   // alpha - beta
    tau = refl ? 2.0 * frcp(fma(v1, v1, sig)) : 0.0;
    vj = jj == i + 1 ? v1 : vj;
  }
  const double beta = refl ? (alpha >= 0.0 ? -nrm : nrm) : alpha;
  if (taus != nullptr && jj == 0) taus[i] = tau;
  constexpr int c0 = (i + 1) & ~1;
  constexpr bool more = i + 1 < KP - 2;                     // a step follows
  if constexpr (!STREAM) {
    // the trailing parts of v and p go to registers in one burst of LDS
    // reads each (one wait per vector instead of one per few products)
    double vv[KP], pp[KP];
    load_pairs<KP, c0, KP>(vv, vb);
    if constexpr (!UNIT) vv[i + 1] = v1;
    double pc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = i + 1; c < KP; ++c) pc[c & 3] = fma(a[c], vv[c], pc[c & 3]);
    const double p = jj > i ? ((pc[0] + pc[1]) + (pc[2] + pc[3])) * tau : 0.0;
    pb[jj] = p;
    wave_lds_sync();
    // p is requested before the reduction for K, which hides the read
    load_pairs<KP, c0, KP>(pp, pb);
    const double K = 0.5 * tau * group_sum<KP>(p * vj);
    const double wj = fma(-2.0 * K, vj, p);
    a[i + 1] = fma(-wj, vv[i + 1], fma(-vj, pp[i + 1], a[i + 1]));
    if constexpr (more) {
      alpha = group_read_c<KP, i + 2>(a[i + 1]);
      sig = group_sum<KP>(jj > i + 2 ? a[i + 1] * a[i + 1] : 0.0);
    }
#pragma unroll
    for (int c = i + 2; c < KP; ++c) a[c] = fma(-wj, vv[c], fma(-vj, pp[c], a[c]));
  } else {
    double vv[KP], pp[KP];
    constexpr int CH = 16;
    load_pairs<KP, c0, cmin(c0 + CH, KP)>(vv, vb);
    double pc[4] = {0.0, 0.0, 0.0, 0.0};
    dot_stream<KP, i + 1, c0, CH>(a, vb, vv, pc);
    double dot = (pc[0] + pc[1]) + (pc[2] + pc[3]);
    if constexpr (!UNIT) dot = fma(a[i + 1], v1, dot);       // the term of v_{i+1}
    const double p = jj > i ? dot * tau : 0.0;
    pb[jj] = p;
    wave_lds_sync();
    // the next column's entries and the first chunk of the rank-2 update's
    // operands are requested before the reduction for K, which hides the reads
    constexpr int CH2 = 8;
    constexpr int c2 = (i + 2) & ~1;
    if constexpr (UNIT) v1 = vb[i + 1];
    const double p1 = pb[i + 1];
    load_pairs<KP, c2, cmin(c2 + CH2, KP)>(vv, vb);
    load_pairs<KP, c2, cmin(c2 + CH2, KP)>(pp, pb);
    const double K = 0.5 * tau * group_sum<KP>(p * vj);
    const double wj = fma(-2.0 * K, vj, p);
    a[i + 1] = fma(-wj, v1, fma(-vj, p1, a[i + 1]));
    if constexpr (more) {
      alpha = group_read_c<KP, i + 2>(a[i + 1]);
      sig = group_sum<KP>(jj > i + 2 ? a[i + 1] * a[i + 1] : 0.0);
    }
    rank2_stream<KP, i + 2, c2, CH2>(a, vb, pb, vv, pp, vj, wj);
  }
  // nothing of the next step may be scheduled into this one (the
  // interleaving would keep two copies of the row live)
  __builtin_amdgcn_sched_barrier(0);
  wave_lds_sync();
  if (jj > i) a[i] = vj;
  if (jj == i) ej = beta;
  // the row and the coupling are final for this step (see pin_regs)
  pin_regs<KP>(a);
  asm volatile("" : "+v"(ej));
}

template <int KP, bool STREAM, bool UNIT, class Sh, int... Is>
__device__ __forceinline__ void tridiag_steps(double (&a)[KP], Sh& sh, int seg, int jj,
                                              double& ej, double* taus,
                                              std::integer_sequence<int, Is...>) {
  double alpha = group_read_c<KP, 1>(a[0]);
  double sig = group_sum<KP>(jj > 1 ? a[0] * a[0] : 0.0);
  (tridiag_step<KP, Is, STREAM, UNIT>(a, sh, seg, jj, alpha, sig, ej, taus), ...);
}

// The reduction; lane jj ends with dj = T[jj][jj] and ej = T[jj+1][jj]
// (e_{KP-1} = 0).  UNIT: the reflectors are scaled to v_{i+1} = 1 and their
// tau values are not kept (the back-transformation recovers each from its
// vector, tau = 2 / v^T v); otherwise they are left unscaled and taus (this
// matrix's KP - 2 values, written to LDS by its first lane) must be given.
// STREAM: the broadcast vectors come from LDS in chunks (fewer registers)
// rather than in one burst.
template <int KP, bool STREAM = (KP > 32), bool UNIT = true, class Sh>
__device__ __forceinline__ void tridiagonalize(double (&a)[KP], Sh& sh, int seg, int jj,
                                               double& dj, double& ej, double* taus = nullptr) {
  ej = 0.0;
  tridiag_steps<KP, STREAM, UNIT>(a, sh, seg, jj, ej, taus,
                                  std::make_integer_sequence<int, KP - 2>{});
  double dg = 0.0;
#pragma unroll
  for (int u = 0; u < KP; ++u) dg = u == jj ? a[u] : dg;
  dj = dg;
  if (jj == KP - 2) ej = a[KP - 1];
  wave_lds_sync();
}

// Whether the Householder vectors stay in registers (a[]) through the divide
// and conquer; beyond that size they wait in global scratch, which leaves
// the registers to the merges.
template <int KP>
constexpr bool kReflInRegisters = KP <= LETKF_REFL_REG_MAX;

// Packed position of reflector i's entry on row r (0 <= i < r < k): the
// reflectors' entries below their unit element, reflector by reflector.
__device__ __forceinline__ int refl_pos(int i, int r, int k) {
  return i * k - i * (i + 1) / 2 + (r - i - 1);
}

// This lane's entries of the reflectors (a[i] = v_jj of step i, i < jj) to
// global scratch rv (k (k - 1) / 2 doubles); rows >= k carry none.
template <int KP>
__device__ __forceinline__ void store_reflectors(const double (&a)[KP], double* rv, int k, int jj,
                                                 bool valid) {
  if (!valid || jj >= k) return;
#pragma unroll
  for (int i = 0; i < KP - 2; ++i)
    if (i < jj) rv[refl_pos(i, jj, k)] = a[i];
}

// Entries i+1 .. KP-1 of reflector i (row i of the matrix area, stride KP)
// into registers, two per LDS read (from the even entry at or below i+1).
template <int KP, int i>
__device__ __forceinline__ void load_reflector(double (&v)[KP], const double* rows) {
  constexpr int c0 = (i + 1) & ~1;
#pragma unroll
  for (int r = c0; r < KP; r += 2) {
    const double2 t2 = *reinterpret_cast<const double2*>(rows + i * KP + r);
    v[r] = t2.x;
    v[r + 1] = t2.y;
  }
}

// tau of a Householder vector v (v_{i+1} = 1) from s = sum_{r > i+1} v_r^2:
// the reduction's tau = (beta - alpha) / beta equals 2 / v^T v = 2 / (1 + s),
// and a step that reflected nothing has v = e_{i+1} (s = 0) and tau = 0.
// (s is summed apart from the unit entry: 1 + s rounds to 1 long before the
// reflection becomes negligible, when it is close to a sign flip, tau = 2.)
__device__ __forceinline__ double tau_of(double s) { return s > 0.0 ? 2.0 * frcp(1.0 + s) : 0.0; }

// H_i applied to this lane's column q, the reflector streamed from LDS (KP = 64).
template <int KP, int i>
__device__ __forceinline__ void apply_reflector_stream(double (&q)[KP], const double* rows) {
  constexpr int c0 = (i + 1) & ~1;
  constexpr int CH = 16;
  const double* v = rows + i * KP;
  double vv[KP];
  load_pairs<KP, c0, cmin(c0 + CH, KP)>(vv, v);
  double pc[4] = {0.0, 0.0, 0.0, 0.0}, nc[4] = {0.0, 0.0, 0.0, 0.0};
  dotn_stream<KP, i + 1, c0, CH>(q, v, vv, pc, nc);
  const double f = tau_of((nc[0] + nc[1]) + (nc[2] + nc[3])) * ((pc[0] + pc[1]) + (pc[2] + pc[3]));
  load_pairs<KP, c0, cmin(c0 + CH, KP)>(vv, v);
  axpy_stream<KP, i + 1, c0, CH>(q, v, vv, f);
}

template <int KP, int... Is>
__device__ __forceinline__ void apply_reflectors_stream(double (&q)[KP], const double* rows,
                                                        std::integer_sequence<int, Is...>) {
  (apply_reflector_stream<KP, KP - 3 - Is>(q, rows), ...);
}

// H_i .. H_0 applied to this lane's column q (KP <= 32), reflector i taken
// from registers (cur) while reflector i-1 is read into the other set: the
// LDS latency of a reflector hides behind the products of the one before.
template <int KP, int i>
__device__ __forceinline__ void apply_reflectors_pipelined(double (&q)[KP], double (&cur)[KP],
                                                           const double* rows) {
  double nxt[KP];
  if constexpr (i > 0) load_reflector<KP, i - 1>(nxt, rows);
  double dc[4] = {0.0, 0.0, 0.0, 0.0}, nc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int r = i + 1; r < KP; ++r) dc[r & 3] = fma(q[r], cur[r], dc[r & 3]);
#pragma unroll
  for (int r = i + 2; r < KP; ++r) nc[r & 3] = fma(cur[r], cur[r], nc[r & 3]);
  const double f = tau_of((nc[0] + nc[1]) + (nc[2] + nc[3])) * ((dc[0] + dc[1]) + (dc[2] + dc[3]));
#pragma unroll
  for (int r = i + 1; r < KP; ++r) q[r] = fma(-f, cur[r], q[r]);
  // no instruction of the next reflector ahead of this point (it would keep
  // a third reflector's registers live)
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (i > 0) apply_reflectors_pipelined<KP, i - 1>(q, nxt, rows);
}

// V = H Q_T with H = H_0 H_1 .. H_{n-3}: q holds row jj of Q_T on entry.
// Q_T goes through the matrix area to give this lane column jj; the
// reflectors follow it there as rows (stride KP), from this lane's registers
// (a[i] = v_jj of step i, KP <= 32) or from the global scratch rv (KP = 64,
// where the registers were needed during the divide and conquer); each lane
// then applies H_{n-3} .. H_0 to its column.  V leaves in the matrix area in
// natural layout (row stride KP+1).
template <int KP>
__device__ __forceinline__ void back_transform(double (&q)[KP], const double (&a)[KP],
                                               const double* rv, int k, EvdLds<KP>& sh, int seg,
                                               int jj) {
  constexpr int S = KP + 1;
  double* M = sh.mat[seg];
#pragma unroll
  for (int u = 0; u < KP; ++u) M[jj * S + u] = q[u];
  wave_lds_sync();
#pragma unroll
  for (int r = 0; r < KP; ++r) q[r] = M[r * S + jj];
  wave_lds_sync();
  if constexpr (kReflInRegisters<KP>) {
#pragma unroll
    for (int i = 0; i < KP - 2; ++i) M[i * KP + jj] = jj > i ? a[i] : 0.0;
  } else {
    double v[KP - 2];
#pragma unroll
    for (int i = 0; i < KP - 2; ++i) v[i] = (i < jj && jj < k) ? rv[refl_pos(i, jj, k)] : 0.0;
#pragma unroll
    for (int i = 0; i < KP - 2; ++i) M[i * KP + jj] = v[i];
  }
  wave_lds_sync();
  if constexpr (KP <= 32) {
    const double* rows = &sh.mat[0][0] + opaque(seg * KP * (KP + 1));
    double cur[KP];
    load_reflector<KP, KP - 3>(cur, rows);
    apply_reflectors_pipelined<KP, KP - 3>(q, cur, rows);
  } else {
    const double* rows = &sh.mat[0][0] + opaque(seg * KP * (KP + 1));
    apply_reflectors_stream<KP>(q, rows, std::make_integer_sequence<int, KP - 2>{});
  }
  wave_lds_sync();
#pragma unroll
  for (int r = 0; r < KP; ++r) M[r * S + jj] = q[r];
  wave_lds_sync();
}

// Mode 1 output: eigenvalues and eigenvectors (V natural layout in M).  For
// k < KP the KP - k padding eigenpairs (unit vectors on the padded rows, which
// the merges never couple to the matrix) are dropped and the k others are
// written in column order.
template <int KP>
__device__ __forceinline__ void write_eig(const EvdArgs& e, const double* M, int seg, int jj,
                                          int pl, bool valid, double lam) {
  const int k = e.k;
  bool real = true;
  for (int r = k; r < KP; ++r) real = real && M[r * (KP + 1) + jj] == 0.0;
  const uint64_t lowmask = KP == 64 ? ~0ull : ((1ull << KP) - 1ull);
  const uint64_t mask = (__ballot(real) >> (seg * KP)) & lowmask;
  const int slot = __popcll(mask & ((1ull << jj) - 1ull));
  if (valid && real && slot < k) {
    e.lam[(size_t)pl * k + slot] = lam;
    for (int r = 0; r < k; ++r) e.vec[((size_t)pl * k + r) * k + slot] = M[r * (KP + 1) + jj];
  }
}

// Mode 0: transform and in-place update of the point's nine components,
// from V (rows from the natural layout in M, row stride KP+1, bank-conflict
// free; this lane's column jj from q[]), this lane's eigenvalue lam and this
// lane's entry of b.
// T = double: FP64 contractions.  T = float: the reduced-precision forms —
// V, b, dX, U and the weights are rounded to FP32 or BF16 (e.prec) as
// contraction operands and accumulated in FP32; the ensemble mean, its
// subtraction and the eigenvalue scaling stay FP64.
template <typename T>
__device__ __forceinline__ T opnd(double x, int prec);
template <>
__device__ __forceinline__ double opnd<double>(double x, int) { return x; }
template <>
__device__ __forceinline__ float opnd<float>(double x, int prec) { return round_operand(x, prec); }

template <int KP, typename T>
__device__ __forceinline__ void transform_update(const EvdArgs& e, EvdLds<KP>& sh, int seg, int jj,
                                                 int pl, bool valid, double lam, double bj,
                                                 const double (&q)[KP]) {
  const int prec = e.prec;
  constexpr int S = KP + 1;
  const int k = e.k;
  const double* M = sh.mat[seg];
  const double* Mrow = M + jj * S;
  // z = Lambda^-1 V^T b  (lane jj = column jj)
  double* bz = sh.dxu[seg][0];
  bz[jj] = bj;
  wave_lds_sync();
  // (column jj of V is this lane's q[] from the back-transformation)
  T z = 0;
#pragma unroll
  for (int r = 0; r < KP; ++r) z = fma(opnd<T>(q[r], prec), opnd<T>(bz[r], prec), z);
  const double z1 = (double)z / lam;
  wave_lds_sync();
  bz[jj] = z1;
  wave_lds_sync();
  // wbar = V z  (lane jj = row jj)
  T wbt = 0;
#pragma unroll 4
  for (int c = 0; c < KP; ++c) wbt = fma(opnd<T>(Mrow[c], prec), opnd<T>(bz[c], prec), wbt);
  const T wb = opnd<T>((double)wbt, prec);
  wave_lds_sync();

  // the point's nine components: mean and perturbations (eqs. xmean, xspread)
  const bool mine = valid && jj < k;
  double* xp = e.xt + (size_t)(e.pt0 + (valid ? pl : 0)) * 9 * k + jj;
  const double inv_k = 1.0 / (double)k;
  const double d2 = e.sqrt_km1 / sqrt(lam);
  bool finite = true;
#pragma unroll
  for (int i0 = 0; i0 < 9; i0 += kCompGroup) {
    constexpr int CG = kCompGroup;
    const int nc = 9 - i0 < CG ? 9 - i0 : CG;
    double dx[CG], xbar[CG];
    T sm[CG];
#pragma unroll
    for (int i = 0; i < CG; ++i) {
      if (i >= nc) break;
      dx[i] = mine ? xp[(i0 + i) * k] : 0.0;
      xbar[i] = group_sum<KP>(dx[i]) * inv_k;
      dx[i] = mine ? dx[i] - xbar[i] : 0.0;
      const T dxo = opnd<T>(dx[i], prec);
      sm[i] = (T)group_sum<KP>((double)(dxo * wb));  // (dX wbar)_i
      sh.dxu[seg][i][jj] = (double)dxo;
    }
    wave_lds_sync();
    // U = dX V diag(sqrt(k-1) lam^-1/2)   (lane jj = column jj)
    T U[CG];
#pragma unroll
    for (int i = 0; i < CG; ++i) U[i] = 0;
#pragma unroll
    for (int m = 0; m < KP; ++m) {
      const T vm = opnd<T>(q[m], prec);
#pragma unroll
      for (int i = 0; i < CG; ++i)
        if (i < nc) U[i] = fma((T)sh.dxu[seg][i][m], vm, U[i]);
    }
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < CG; ++i)
      if (i < nc) sh.dxu[seg][i][jj] = (double)opnd<T>((double)U[i] * d2, prec);
    wave_lds_sync();
    // X^a = xbar + dX wbar + U V^T   (lane jj = member jj)
    T acc[CG];
#pragma unroll
    for (int i = 0; i < CG; ++i) acc[i] = 0;
#pragma unroll 2
    for (int c = 0; c < KP; ++c) {
      const T vr = opnd<T>(Mrow[c], prec);
#pragma unroll
      for (int i = 0; i < CG; ++i)
        if (i < nc) acc[i] = fma((T)sh.dxu[seg][i][c], vr, acc[i]);
    }
#pragma unroll
    for (int i = 0; i < CG; ++i) {
      if (i >= nc) break;
      const double xa = xbar[i] + (double)(sm[i] + acc[i]);
      finite = finite && __builtin_isfinite(xa);
      if (mine) xp[(i0 + i) * k] = xa;
    }
    wave_lds_sync();
  }
  if (mine && !finite) atomicOr(e.status, kStatNonfinite);
}

template <int KP>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(LETKF_EVD_WAVES))) void k_evd(BatchMap bm) {
  constexpr int G = 64 / KP;
  __shared__ EvdLds<KP> sh;
  const int lane = lane_id();
  const int seg = lane / KP, jj = lane % KP;
  const int pl = blockIdx.x * G + seg;
  bool valid;
  const EvdArgs e = evd_args_of(bm, pl, valid);
  double bj = 0.0;
  int ex;
  stage_matrix<KP>(e, sh, seg, jj, pl, valid, bj, ex);
  wave_lds_sync();
  // Scratch for the reflectors when they do not stay in registers through
  // the divide and conquer: this point's Gram output (mode 0, consumed by the
  // staging above) or its eigenvector output (mode 1, written last).
  double* rv = e.mode == 0 ? e.C + (size_t)pl * ((KP / 16) * (KP / 16 + 1) / 2) * 256 : e.vec + (size_t)pl * e.k * e.k;
  double a[KP];
  load_rows<KP>(sh.mat[seg], jj, a);
  wave_lds_sync();
  double dj, ej;   // this lane's diagonal and coupling of T
  tridiagonalize<KP>(a, sh, seg, jj, dj, ej);
  if constexpr (!kReflInRegisters<KP>) store_reflectors<KP>(a, rv, e.k, jj, valid);

  double q[KP];
  double lam;
  const bool conv =
      dc_tridiagonal<KP>(q, lam, sh.dc[seg], dj, ej, sh.mat[seg], jj, e.defl_eps);
  // any lane of the matrix whose secular root ran out of iterations
  const uint64_t segmask = KP == 64 ? ~0ull : (((1ull << KP) - 1ull) << (seg * KP));
  const bool all_conv = (__ballot(!conv) & segmask) == 0;
  if (!all_conv && jj == 0 && valid && e.status) atomicOr(e.status, kStatNotconv);
  wave_lds_sync();
  back_transform<KP>(q, a, rv, e.k, sh, seg, jj);
  if (e.mode != 0) {
    write_eig<KP>(e, sh.mat[seg], seg, jj, pl, valid, ldexp(lam, ex));
    return;
  }
  if (e.prec == 0)
    transform_update<KP, double>(e, sh, seg, jj, pl, valid, lam, bj, q);
  else
    transform_update<KP, float>(e, sh, seg, jj, pl, valid, lam, bj, q);
}

template <int KP>
hipError_t launch_evd_kp(const BatchMap& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const dim3 grid(ceil_div(a.n, 64 / KP));
  hipLaunchKernelGGL(k_evd<KP>, grid, dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace letkf
