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
//      registers; the reflector of step i is broadcast through LDS and the
//      symmetric rank-2 update A -= v w^T + w v^T runs in-lane.
//   2. H = H_0 H_1 ... H_{n-3} accumulated row by row in registers, then
//      stored to LDS (natural layout, row stride KP+1).
//   3. Implicit QL iterations with Wilkinson's shift on T (Bowdler, Martin,
//      Reinsch & Wilkinson 1968, "The QR and QL algorithms for symmetric
//      matrices"), each plane rotation applied to the columns of H in LDS, so
//      that H ends as the eigenvector matrix V.  Every lane of a matrix runs
//      the same scalar rotation chain (the chain is uniform per matrix); the
//      lane owns one row of V.  Deflation is tested lane-parallel (lane j
//      tests the subdiagonal entry e_j) and resolved with a ballot.
// Sizes below KP are padded with decoupled unit rows; their subdiagonal
// entries are exactly zero, so no rotation ever couples them to the matrix.
#pragma once
#include "common.h"
#include "launch.h"

namespace letkf {

// Target waves per SIMD for the register allocator of the eigensolve kernel.
#ifndef LETKF_EVD_WAVES
#define LETKF_EVD_WAVES 2
#endif

// LDS per block: the matrix area (input staging, then the Householder vectors
// with row stride KP, then V in natural layout with row stride KP+1), a
// 5 x KP area per matrix that holds b, then Lambda^-1 V^T b, then dX and dX V
// for up to five of the nine components at a time, and the tridiagonal
// (d, e), the reflector scalars tau and two broadcast vectors.
constexpr int kCompGroup = 5;
template <int KP>
struct EvdLds {
  static constexpr int G = 64 / KP;
  static constexpr int S = KP + 1;   // row stride: 16 consecutive rows hit distinct banks
  double mat[G][KP * S];
  double dxu[G][kCompGroup][KP];
  double d[G][KP];
  double e[G][KP];
  double tau[G][KP];
  double vb[G][KP];
  double wb[G][KP];
};

// Value of x held by lane `src` of this lane's KP-lane group.
template <int KP>
__device__ __forceinline__ double group_read(double x, int src) {
  return __shfl(x, src, KP);
}

// An integer the compiler cannot see through: LDS addresses derived from it
// are recomputed after each use point instead of being hoisted out of the
// unrolled loops (where every one of them would hold a VGPR).
__device__ __forceinline__ int opaque(int x) {
  asm volatile("v_mov_b32 %0, %1" : "=v"(x) : "v"(x));
  return x;
}

// Maximum over aligned groups of G lanes (every lane of a group gets it).
template <int G>
__device__ __forceinline__ double group_max(double x) {
  if constexpr (G >= 64) x = fmax(x, xor_lane<32>(x));
  if constexpr (G >= 32) x = fmax(x, xor_lane<16>(x));
  if constexpr (G >= 16) x = fmax(x, xor_lane<8>(x));
  if constexpr (G >= 8) x = fmax(x, xor_lane<4>(x));
  if constexpr (G >= 4) x = fmax(x, xor_lane<2>(x));
  if constexpr (G >= 2) x = fmax(x, xor_lane<1>(x));
  return x;
}

// 1/sqrt(x) for x > 0: hardware estimate and one Newton-Raphson step.
__device__ __forceinline__ double rsqrt_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x * y;
  return fma(y, fma(-h, y, 0.5), y);
}

// Q = alpha I + C (mode 0, upper blocks mirrored) or A (mode 1) into the
// matrix area, padded rows = unit; b into dxu[0] (mode 0).
template <int KP>
__device__ __forceinline__ void stage_matrix(const EvdArgs& e, EvdLds<KP>& sh, int seg, int jj,
                                             int pl, bool valid) {
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
    sh.dxu[seg][0][jj] = (valid && jj < k) ? e.b[(size_t)pl * KP + jj] : 0.0;
  } else {
    for (int c = 0; c < KP; ++c) {
      double val = c == jj ? 1.0 : 0.0;
      if (valid && jj < k && c < k) {
        const int r0 = jj < c ? jj : c, c0 = jj < c ? c : jj;
        val = e.A[((size_t)pl * k + r0) * k + c0];
      }
      M[jj * S + c] = val;
    }
  }
}


template <int KP>
__device__ __forceinline__ void load_rows(const double* M, int jj, double (&a)[KP]) {
  constexpr int S = KP + 1;
#pragma unroll
  for (int u = 0; u < KP; ++u) a[u] = M[jj * S + u];
}

// Householder tridiagonalization of the symmetric matrix whose row jj this
// lane holds in a[].  Step i annihilates A[i+2:, i] with H_i = I - tau v v^T,
// v = (0,..,0, 1, v_{i+2}, .., v_{n-1}); afterwards
//   d_j = T[j][j] -> sh.d,  e_j = T[j+1][j] -> sh.e,  tau_i -> sh.tau,
//   v of step i -> row i of the matrix area (row stride KP).
template <int KP>
__device__ __forceinline__ void tridiagonalize(double (&a)[KP], EvdLds<KP>& sh, int seg, int jj) {
#pragma unroll
  for (int i = 0; i < KP - 2; ++i) {
    const int so = opaque(seg * KP);
    double* vb = &sh.vb[0][0] + so;
    double* wb = &sh.wb[0][0] + so;
    const double x = a[i];                                   // A[jj][i]
    const double alpha = group_read<KP>(x, i + 1);            // A[i+1][i]
    const double sig = group_sum<KP>(jj > i + 1 ? x * x : 0.0);
    const bool refl = sig != 0.0;                             // uniform per matrix
    const double nrm = sqrt(fma(alpha, alpha, sig));
    const double beta = refl ? (alpha >= 0.0 ? -nrm : nrm) : alpha;
    const double tau = refl ? (beta - alpha) / beta : 0.0;
    const double inv = refl ? 1.0 / (alpha - beta) : 0.0;
    const double vj = jj == i + 1 ? 1.0 : (jj > i + 1 ? x * inv : 0.0);
    vb[jj] = vj;
    wave_lds_sync();
    // p = tau A v over the trailing block, w = p - (tau/2)(p.v) v
    double p0 = 0.0, p1 = 0.0;
#pragma unroll
    for (int c = i + 1; c < KP; ++c) {
      if ((c & 1) == 0)
        p0 = fma(a[c], vb[c], p0);
      else
        p1 = fma(a[c], vb[c], p1);
      if ((c & 7) == 7) asm volatile("" ::: "memory");
    }
    const double p = jj > i ? (p0 + p1) * tau : 0.0;
    const double K = 0.5 * tau * group_sum<KP>(p * vj);
    const double w = fma(-K, vj, p);
    wb[jj] = w;
    wave_lds_sync();
    // A <- A - v w^T - w v^T on rows/columns > i (rows <= i have v = w = 0);
    // v is read again through a fresh offset rather than kept live from above
    const int so2 = opaque(so);
    const double* vb2 = &sh.vb[0][0] + so2;
    const double* wb2 = &sh.wb[0][0] + so2;
#pragma unroll
    for (int c = i + 1; c < KP; ++c) {
      a[c] -= fma(vj, wb2[c], w * vb2[c]);
      if ((c & 7) == 7) asm volatile("" ::: "memory");
    }
    // nothing of the next step may be scheduled into this one (the
    // interleaving would keep two copies of the row live)
    __builtin_amdgcn_sched_barrier(0);
    wave_lds_sync();
    if (jj > i) a[i] = vj;
    if (jj == i) {
      sh.e[seg][i] = beta;
      sh.tau[seg][i] = tau;
    }
  }
  double dg = 0.0;
#pragma unroll
  for (int u = 0; u < KP; ++u) dg = u == jj ? a[u] : dg;
  sh.d[seg][jj] = dg;
  if (jj == KP - 2) sh.e[seg][KP - 2] = a[KP - 1];
  if (jj == KP - 1) sh.e[seg][KP - 1] = 0.0;
  double* Vr = sh.mat[seg];
#pragma unroll
  for (int i = 0; i < KP - 2; ++i) Vr[i * KP + jj] = jj > i ? a[i] : 0.0;
  wave_lds_sync();
}

// Row jj of H = H_0 H_1 ... H_{n-3} (so that Q = H T H^T), accumulated in
// registers from the reflectors in the matrix area, then stored to the
// matrix area in natural layout.
template <int KP>
__device__ __forceinline__ void form_reflector_product(double (&z)[KP], EvdLds<KP>& sh, int seg,
                                                       int jj) {
  constexpr int S = KP + 1;
  double* M = sh.mat[seg];
#pragma unroll
  for (int u = 0; u < KP; ++u) {
    double one = u == jj ? 1.0 : 0.0;
    z[u] = one;
  }
#pragma unroll
  for (int i = 0; i < KP - 2; ++i) {
    const double t = sh.tau[seg][i];
    const double* v = &sh.mat[0][0] + opaque(seg * KP * (KP + 1)) + i * KP;
    double d0 = 0.0, d1 = 0.0;
#pragma unroll
    for (int c = i + 1; c < KP; ++c) {
      if ((c & 1) == 0)
        d0 = fma(z[c], v[c], d0);
      else
        d1 = fma(z[c], v[c], d1);
      if ((c & 7) == 7) asm volatile("" ::: "memory");
    }
    const double f = t * (d0 + d1);
#pragma unroll
    for (int c = i + 1; c < KP; ++c) {
      z[c] = fma(-f, v[c], z[c]);
      if ((c & 7) == 7) asm volatile("" ::: "memory");
    }
  }
  wave_lds_sync();
#pragma unroll
  for (int u = 0; u < KP; ++u) M[jj * S + u] = z[u];
  wave_lds_sync();
}

// Implicit QL with Wilkinson's shift on (d, e), rotations applied to the
// columns of V (natural layout in the matrix area).  On return d holds the
// eigenvalues and column j of V the eigenvector of d_j.  Returns false if the
// matrix needed more than max_its QL iterations in total (the remaining
// subdiagonal entries are then deflated one by one as they are).
template <int KP>
__device__ __forceinline__ bool ql_implicit(EvdLds<KP>& sh, int seg, int jj, int max_its) {
  constexpr int S = KP + 1;
  double* d = sh.d[seg];
  double* e = sh.e[seg];
  double* V = sh.mat[seg] + jj * S;      // this lane's row of V
  const int sh0 = seg * KP;
  const uint64_t lowmask = KP == 64 ? ~0ull : ((1ull << KP) - 1ull);
  constexpr double kHalfEps = 0x1p-53;
  // Deflation threshold relative to the norm of T, max_j |d_j| + |e_j| (as in
  // EISPACK's tql2): the rounding noise that the reduction leaves in the
  // subdiagonal of a tight eigenvalue cluster is of order eps |T|, so a test
  // against the neighbouring diagonal entries alone can stall there.
  double tn = fabs(d[jj]) + fabs(e[jj]);
  tn = group_max<KP>(tn);
  const double tol = kHalfEps * tn;
  int l = 0, its = 0;
  bool ok = true;
  for (;;) {
    wave_lds_sync();
    // lane-parallel deflation test of e_jj (NaN counts as negligible so that
    // a non-finite matrix still terminates)
    const double ej = e[jj];
    const bool small = jj == KP - 1 || !(fabs(ej) > tol);
    const uint64_t sm = (__ballot(small) >> sh0) & lowmask;
    const uint64_t ge = l < 64 ? ~0ull << l : 0ull;
    const uint64_t ns = ~sm & ge & lowmask;
    l = ns ? __builtin_ctzll(ns) : KP;
    bool act = l < KP;
    if (__ballot(act) == 0) break;
    int m = act ? __builtin_ctzll(sm & (~0ull << l)) : 0;
    if (act && ++its > max_its) {
      ok = false;
      e[l] = 0.0;                                          // out of iterations: deflate as is
      act = false;
    }
    double dl = 0.0, g = 0.0;
    if (act) {
      dl = d[l];
      const double dl1 = d[l + 1], el = e[l], dm = d[m];
      g = (dl1 - dl) / (2.0 * el);
      const double r = sqrt(fma(g, g, 1.0));
      g = dm - dl + el / (g + (g >= 0.0 ? r : -r));
    }
    // sweep i = m-1 .. l: carries d[i+1] and the updated V[jj][i+1]
    int i = m - 1;
    double s = 1.0, c = 1.0, p = 0.0;
    double di1 = act ? d[m] : 0.0;
    double vi1 = act ? V[m] : 0.0;
    double ei_n = act ? e[i] : 0.0, di_n = act ? d[i] : 0.0, vi_n = act ? V[i] : 0.0;
    bool sw = act, under = false;
    while (__ballot(sw)) {
      if (sw) {
        const double ei = ei_n, di = di_n, vi = vi_n;
        const int ip = i > 0 ? i - 1 : 0;                 // prefetch the next step's operands
        ei_n = e[ip];
        di_n = d[ip];
        vi_n = V[ip];
        const double f = s * ei, b = c * ei;
        const double rr = fma(f, f, g * g);
        if (rr == 0.0) {
          // f = g = 0: the sweep cannot continue; deflate at m and retry
          d[i + 1] = di1 - p;
          e[i + 1] = 0.0;
          e[m] = 0.0;
          V[i + 1] = vi1;
          under = true;
          sw = false;
        } else {
          const double ir = rsqrt_nr(rr);
          e[i + 1] = rr * ir;
          s = f * ir;
          c = g * ir;
          const double gg = di1 - p;
          const double t = fma(di - gg, s, 2.0 * c * b);
          p = s * t;
          d[i + 1] = gg + p;
          g = fma(c, t, -b);
          V[i + 1] = fma(s, vi, c * vi1);
          vi1 = fma(c, vi, -s * vi1);
          di1 = di;
          if (--i < l) sw = false;
        }
      }
    }
    if (act && !under) {
      V[l] = vi1;
      d[l] = dl - p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  wave_lds_sync();
  return ok;
}

// Mode 1 output: eigenvalues and eigenvectors (V natural layout in M).
template <int KP>
__device__ __forceinline__ void write_eig(const EvdArgs& e, const double* M, int jj, int pl,
                                          bool valid, double lam) {
  const int k = e.k;
  if (valid && jj < k) {
    e.lam[(size_t)pl * k + jj] = lam;
    for (int r = 0; r < k; ++r) e.vec[((size_t)pl * k + r) * k + jj] = M[r * (KP + 1) + jj];
  }
}

// Mode 0: transform and in-place update of the point's nine components,
// from V (natural layout in M, row stride KP+1), this lane's eigenvalue lam
// and b (in dxu[0]).  Row reads M[jj][c] and column reads M[m][jj] are both
// bank-conflict free within 16-lane groups.
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
                                                 int pl, bool valid, double lam) {
  const int prec = e.prec;
  constexpr int S = KP + 1;
  const int k = e.k;
  const double* M = sh.mat[seg];
  const double* Mrow = M + jj * S;
  // z = Lambda^-1 V^T b  (lane jj = column jj)
  double* bz = sh.dxu[seg][0];
  T z = 0;
#pragma unroll 4
  for (int r = 0; r < KP; ++r) z = fma(opnd<T>(M[r * S + jj], prec), opnd<T>(bz[r], prec), z);
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
#pragma unroll 2
    for (int m = 0; m < KP; ++m) {
      const T vm = opnd<T>(M[m * S + jj], prec);
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

// The descriptor of the problem that owns slab-local point pl, with C and b
// pointed at the slab and pt0 set so that pt0 + pl is the point within its
// problem (every helper indexes C, b by pl and the ensemble by pt0 + pl).
__device__ __forceinline__ EvdArgs evd_args_of(const BatchMap& bm, int pl, bool& valid) {
  valid = pl < bm.n;
  const int gidx = bm.g0 + (valid ? pl : 0);
  const int prob = bm.prefix ? find_problem(bm.prefix, bm.nprob, gidx) : 0;
  EvdArgs e = bm.e ? bm.e[prob] : bm.e_inline;
  e.C = bm.C;
  e.b = bm.b;
  e.pt0 = gidx - (bm.prefix ? bm.prefix[prob] : 0) - (valid ? pl : 0);
  if (e.abort_flag && *e.abort_flag) valid = false;
  return e;
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
  stage_matrix<KP>(e, sh, seg, jj, pl, valid);
  wave_lds_sync();
  {
    double a[KP];
    load_rows<KP>(sh.mat[seg], jj, a);
    wave_lds_sync();
    tridiagonalize<KP>(a, sh, seg, jj);
    form_reflector_product<KP>(a, sh, seg, jj);
  }
  const bool conv = ql_implicit<KP>(sh, seg, jj, e.max_its * KP);
  if (!conv && jj == 0 && valid && e.status) atomicOr(e.status, kStatNotconv);
  const double lam = sh.d[seg][jj];
  wave_lds_sync();
  if (e.mode != 0) {
    write_eig<KP>(e, sh.mat[seg], jj, pl, valid, lam);
    return;
  }
  if (e.prec == 0)
    transform_update<KP, double>(e, sh, seg, jj, pl, valid, lam);
  else
    transform_update<KP, float>(e, sh, seg, jj, pl, valid, lam);
}

template <int KP>
hipError_t launch_evd_kp(const BatchMap& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const dim3 grid(ceil_div(a.n, 64 / KP));
  hipLaunchKernelGGL(k_evd<KP>, grid, dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace letkf
