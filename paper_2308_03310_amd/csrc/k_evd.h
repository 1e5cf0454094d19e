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
// Eigensolver: cyclic two-sided Jacobi (Golub & Van Loan, Matrix
// Computations, Sec. 8.5 "Jacobi methods": sym.schur2 rotation, cyclic
// sweeps).  Within a sweep the k(k-1)/2 index pairs are ordered in KP-1
// rounds; round m pairs row p with row p XOR m, so each round is k/2
// disjoint rotations that run in parallel, one matrix row per lane.  A KP-row
// matrix occupies KP lanes of a wavefront (KP = 16, 32, 64), so 64/KP
// matrices share one wavefront.  Sizes below KP are padded with decoupled
// unit diagonal rows, which no rotation ever touches.
//
// Register layout ("diagonal layout"): lane j holds a[u] = A[j][j^u] and
// v[u] = V[j][j^u] for u = 0..KP-1, so the diagonal is a[0], the pivot of
// round m is a[m], and both the row exchange (partner row, xor-m lane
// shuffle) and the column rotation (slots u, u^m) use compile-time register
// indices.
#pragma once
#include "common.h"
#include "launch.h"

namespace letkf {

template <int M>
__host__ __device__ constexpr int high_bit() {
  int h = 1;
  while ((h << 1) <= M) h <<= 1;
  return h;
}

// Slot of the R-th pair representative of mask M: R with a zero bit inserted
// at the position of M's highest set bit (so slot < slot ^ M).
template <int M, int R>
__host__ __device__ constexpr int rep_slot() {
  constexpr int HB = high_bit<M>();
  return ((R & ~(HB - 1)) << 1) | (R & (HB - 1));
}

#ifndef LETKF_JACOBI_PAIR_GROUP
#define LETKF_JACOBI_PAIR_GROUP 0
#endif

template <int R>
__device__ __forceinline__ void pair_group_fence() {
  constexpr int G = LETKF_JACOBI_PAIR_GROUP;
  if constexpr (G > 0 && R % G == G - 1) __builtin_amdgcn_sched_barrier(0);
}

// Row exchange + column rotation of the slot pair (U, U^M) of this lane's row.
template <int KP, int M, int U>
__device__ __forceinline__ void jacobi_pair(double (&a)[KP], double (&v)[KP], int jj, double c,
                                            double sr, const double2* cb) {
  constexpr int UM = U ^ M;
  const double pu = xor_lane<M>(a[UM]);   // partner row, column jj^U
  const double pum = xor_lane<M>(a[U]);   // partner row, column jj^U^M
  const double x0 = fma(sr, pu, c * a[U]);
  const double x1 = fma(sr, pum, c * a[UM]);
  const double2 cf = cb[jj ^ U];          // rotation of column jj^U
  a[U] = fma(cf.y, x1, cf.x * x0);
  a[UM] = fma(-cf.y, x0, cf.x * x1);
  const double v0 = v[U], v1 = v[UM];
  v[U] = fma(cf.y, v1, cf.x * v0);
  v[UM] = fma(-cf.y, v0, cf.x * v1);
}

template <int KP, int M, int... Rs>
__device__ __forceinline__ void jacobi_pairs(double (&a)[KP], double (&v)[KP], int jj, double c,
                                             double sr, const double2* cb,
                                             std::integer_sequence<int, Rs...>) {
  ((jacobi_pair<KP, M, rep_slot<M, Rs>()>(a, v, jj, c, sr, cb), pair_group_fence<Rs>()), ...);
}

// One round: rotations (j, j^M) for every lane j.  cb is this matrix's
// coefficient buffer in LDS (KP entries of (c, signed s)).
template <int KP, int M>
__device__ __forceinline__ void jacobi_round(double (&a)[KP], double (&v)[KP], int jj, double2* cb) {
  constexpr int HB = high_bit<M>();
  const bool lo = (jj & HB) == 0;  // this lane is p (the smaller index) of its pair
  const double d_self = a[0];
  const double d_oth = xor_lane<M>(d_self);
  const double o_self = a[M];
  const double o_oth = xor_lane<M>(o_self);
  // Both lanes of a pair use the p-lane's copies, so they agree bitwise.
  const double app = lo ? d_self : d_oth;
  const double aqq = lo ? d_oth : d_self;
  const double apq = lo ? o_self : o_oth;
  // Branch-free sym.schur2: t = sign(zeta)/(|zeta| + sqrt(1 + zeta^2)) is the
  // smaller root of t^2 + 2 zeta t - 1 = 0; apq = 0 gives the identity.  When
  // zeta^2 overflows, t rounds to 0 and the (negligible) pivot is dropped.
  const bool nz = apq != 0.0;
  const double zeta = (aqq - app) / (2.0 * (nz ? apq : 1.0));
  const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(fma(zeta, zeta, 1.0)));
  const double t = nz ? tt : 0.0;
  const double c = rsqrt(fma(t, t, 1.0));
  const double s = t * c;
  // J restricted to (p,q) is [[c, s], [-s, c]]; row j of J^T A is
  // c*A[j,:] + sr*A[j^M,:] with sr = -s on p and +s on q, and the same
  // (c, sr) of lane l rotates column l.
  const double sr = lo ? -s : s;
  cb[jj] = make_double2(c, sr);
  wave_lds_sync();
  // Opaque copy of the lane index: keeps the per-slot LDS addresses jj^U
  // from being hoisted out of the sweep loop (they would stay live in VGPRs).
  int jr;
  asm volatile("v_mov_b32 %0, %1" : "=v"(jr) : "v"(jj));
  jacobi_pairs<KP, M>(a, v, jr, c, sr, cb, std::make_integer_sequence<int, KP / 2>{});
  a[0] = lo ? fma(-t, apq, app) : fma(t, apq, aqq);
  a[M] = 0.0;
}

template <int KP, int... Ms>
__device__ __forceinline__ void jacobi_sweep_impl(double (&a)[KP], double (&v)[KP], int jj,
                                                  double2* cb0, double2* cb1,
                                                  std::integer_sequence<int, Ms...>) {
  (jacobi_round<KP, Ms + 1>(a, v, jj, (Ms & 1) ? cb1 : cb0), ...);
}

template <int KP>
__device__ __forceinline__ void jacobi_sweep(double (&a)[KP], double (&v)[KP], int jj,
                                             double2* cb0, double2* cb1) {
  jacobi_sweep_impl<KP>(a, v, jj, cb0, cb1, std::make_integer_sequence<int, KP - 1>{});
}

// Runs sweeps until every matrix of the wavefront has a relative squared
// off-diagonal Frobenius norm <= tol2; returns false if max_sweeps ran out.
template <int KP>
__device__ __forceinline__ bool jacobi_solve(double (&a)[KP], double (&v)[KP], int jj,
                                             double2* cb0, double2* cb1, double tol2,
                                             int max_sweeps) {
  for (int sweep = 0;; ++sweep) {
    double off = 0.0;
#pragma unroll
    for (int u = 1; u < KP; ++u) off = fma(a[u], a[u], off);
    const double dg = a[0] * a[0];
    const double off_s = group_sum<KP>(off), dg_s = group_sum<KP>(dg);
    const bool conv = off_s <= tol2 * dg_s;
    if (__ballot(!conv) == 0) return true;
    if (sweep >= max_sweeps) return false;
    jacobi_sweep<KP>(a, v, jj, cb0, cb1);
  }
}

// ---- split solve: wavefront 0 holds A and computes the rotations, wavefront
// 1 holds V and applies them; one workgroup barrier per round publishes the
// coefficient buffer.  Used for 64-row matrices, whose A and V rows (2 x 128
// VGPRs) do not fit one wavefront's registers.
__device__ __forceinline__ void block_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ int opaque_lane(int jj) {
  int jr;
  asm volatile("v_mov_b32 %0, %1" : "=v"(jr) : "v"(jj));
  return jr;
}

template <int KP, int M, int U>
__device__ __forceinline__ void jacobi_pair_a(double (&a)[KP], int jj, double c, double sr,
                                              const double2* cb) {
  constexpr int UM = U ^ M;
  const double pu = xor_lane<M>(a[UM]);
  const double pum = xor_lane<M>(a[U]);
  const double x0 = fma(sr, pu, c * a[U]);
  const double x1 = fma(sr, pum, c * a[UM]);
  const double2 cf = cb[jj ^ U];
  a[U] = fma(cf.y, x1, cf.x * x0);
  a[UM] = fma(-cf.y, x0, cf.x * x1);
}

template <int R>
__device__ __forceinline__ void v_pair_fence() {
  if constexpr (R % 8 == 7) __builtin_amdgcn_sched_barrier(0);
}

template <int KP, int M, int U>
__device__ __forceinline__ void jacobi_pair_v(double (&v)[KP], int jj, const double2* cb) {
  constexpr int UM = U ^ M;
  const double2 cf = cb[jj ^ U];
  const double v0 = v[U], v1 = v[UM];
  v[U] = fma(cf.y, v1, cf.x * v0);
  v[UM] = fma(-cf.y, v0, cf.x * v1);
}

template <int KP, int M, int... Rs>
__device__ __forceinline__ void jacobi_round_a(double (&a)[KP], int jj, double2* cb,
                                               std::integer_sequence<int, Rs...>) {
  constexpr int HB = high_bit<M>();
  const bool lo = (jj & HB) == 0;
  const double d_self = a[0];
  const double d_oth = xor_lane<M>(d_self);
  const double o_self = a[M];
  const double o_oth = xor_lane<M>(o_self);
  const double app = lo ? d_self : d_oth;
  const double aqq = lo ? d_oth : d_self;
  const double apq = lo ? o_self : o_oth;
  const bool nz = apq != 0.0;
  const double zeta = (aqq - app) / (2.0 * (nz ? apq : 1.0));
  const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(fma(zeta, zeta, 1.0)));
  const double t = nz ? tt : 0.0;
  const double c = rsqrt(fma(t, t, 1.0));
  const double s = t * c;
  const double sr = lo ? -s : s;
  cb[jj] = make_double2(c, sr);
  block_sync();
  const int jr = opaque_lane(jj);
  (jacobi_pair_a<KP, M, rep_slot<M, Rs>()>(a, jr, c, sr, cb), ...);
  a[0] = lo ? fma(-t, apq, app) : fma(t, apq, aqq);
  a[M] = 0.0;
}

template <int KP, int M, int... Rs>
__device__ __forceinline__ void jacobi_round_v(double (&v)[KP], int jj, const double2* cb,
                                               std::integer_sequence<int, Rs...>) {
  block_sync();
  const int jr = opaque_lane(jj);
  // fences every 8 pairs: otherwise all KP/2 coefficient loads of the round
  // are hoisted and live next to V's own 2*KP registers
  ((jacobi_pair_v<KP, M, rep_slot<M, Rs>()>(v, jr, cb), v_pair_fence<Rs>()), ...);
}

template <int KP, int... Ms>
__device__ __forceinline__ void jacobi_sweep_a(double (&a)[KP], int jj, double2* cb0, double2* cb1,
                                               std::integer_sequence<int, Ms...>) {
  (jacobi_round_a<KP, Ms + 1>(a, jj, (Ms & 1) ? cb1 : cb0,
                              std::make_integer_sequence<int, KP / 2>{}), ...);
}

template <int KP, int... Ms>
__device__ __forceinline__ void jacobi_sweep_v(double (&v)[KP], int jj, const double2* cb0,
                                               const double2* cb1,
                                               std::integer_sequence<int, Ms...>) {
  (jacobi_round_v<KP, Ms + 1>(v, jj, (Ms & 1) ? cb1 : cb0,
                              std::make_integer_sequence<int, KP / 2>{}), ...);
}

// LDS per block: matrix area (input staging, rotation coefficients during
// the sweeps, then V in natural layout, row stride KP+1) and a 5 x KP area
// per matrix that holds b, then Lambda^-1 V^T b, then dX and dX V for up to
// five of the nine components at a time.  One-wavefront blocks at KP = 32
// use 19 KiB, so eight fit in a CU's 160 KiB.
constexpr int kCompGroup = 5;
template <int KP>
struct EvdLds {
  static constexpr int G = 64 / KP;
  static constexpr int S = KP + 1;   // row stride: 16 consecutive rows hit distinct banks
  double mat[G][KP * S];
  double dxu[G][kCompGroup][KP];
  double lam[64];
  int flag;
};

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
      const double* Cp = e.C + (size_t)pl * NB * 256;
      int blk = 0;
#pragma unroll
      for (int I = 0; I < NQ; ++I) {
#pragma unroll
        for (int J = I; J < NQ; ++J) {
          for (int t = jj; t < 256; t += KP) {
            const int r = t >> 4, c = t & 15;
            const double val = Cp[blk * 256 + t];
            M[(16 * I + r) * S + 16 * J + c] = val;
            if (I != J) M[(16 * J + c) * S + 16 * I + r] = val;
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
  for (int u = 0; u < KP; ++u) a[u] = M[jj * S + (jj ^ u)];
}

// Diagonal-layout rows (v[u] = V[jj][jj^u]) into the natural layout in LDS.
template <int KP>
__device__ __forceinline__ void store_rows(double* M, int jj, const double (&v)[KP]) {
  constexpr int S = KP + 1;
#pragma unroll
  for (int u = 0; u < KP; ++u) M[jj * S + (jj ^ u)] = v[u];
}

template <int KP>
__device__ __forceinline__ void init_identity(double (&v)[KP]) {
#pragma unroll
  for (int u = 0; u < KP; ++u) {
    // opaque constants: the compiler must not specialize the first sweep for V = I
    double x = u == 0 ? 1.0 : 0.0;
    asm volatile("" : "+v"(x));
    v[u] = x;
  }
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

// One wavefront holds both A and V rows of 64/KP matrices (KP = 16, 32).
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
__global__ __launch_bounds__(64) void k_evd(BatchMap bm) {
  constexpr int G = 64 / KP;
  __shared__ EvdLds<KP> sh;
  const int lane = lane_id();
  const int seg = lane / KP, jj = lane % KP;
  const int pl = blockIdx.x * G + seg;
  bool valid;
  const EvdArgs e = evd_args_of(bm, pl, valid);
  double* M = sh.mat[seg];
  stage_matrix<KP>(e, sh, seg, jj, pl, valid);
  wave_lds_sync();
  double a[KP], v[KP];
  load_rows<KP>(M, jj, a);
  init_identity<KP>(v);
  wave_lds_sync();
  double2* cb0 = reinterpret_cast<double2*>(M);
  const bool conv = jacobi_solve<KP>(a, v, jj, cb0, cb0 + KP, e.tol2, e.max_sweeps);
  if (!conv && jj == 0 && valid && e.status) atomicOr(e.status, kStatNotconv);
  wave_lds_sync();
  const double lam = a[0];
  store_rows<KP>(M, jj, v);
  wave_lds_sync();
  if (e.mode != 0) {
    write_eig<KP>(e, M, jj, pl, valid, lam);
    return;
  }
  if (e.prec == 0)
    transform_update<KP, double>(e, sh, seg, jj, pl, valid, lam);
  else
    transform_update<KP, float>(e, sh, seg, jj, pl, valid, lam);
}

// Two wavefronts per block: wavefront 0 holds A (and ends with the
// eigenvalues), wavefront 1 holds V and does the transform.
template <int KP>
__global__ __launch_bounds__(128) void k_evd_split(BatchMap bm) {
  constexpr int G = 64 / KP;
  __shared__ EvdLds<KP> sh;
  // wave-uniform role (readfirstlane makes the branch provably uniform, so A
  // and V never share one wavefront's registers)
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = lane_id();
  const int seg = lane / KP, jj = lane % KP;
  const int pl = blockIdx.x * G + seg;
  bool valid;
  const EvdArgs e = evd_args_of(bm, pl, valid);
  if (!valid) return;   // G = 1: the whole block shares one point (uniform exit, before any barrier)
  double* M = sh.mat[seg];
  if (wid == 0) stage_matrix<KP>(e, sh, seg, jj, pl, valid);
  block_sync();
  double2* cb0 = reinterpret_cast<double2*>(M);
  double2* cb1 = cb0 + KP;
  double lam = 1.0;
  if (wid == 0) {
    double a[KP];
    load_rows<KP>(M, jj, a);
    block_sync();                                  // matrix area becomes the coefficient buffers
    for (int sweep = 0;; ++sweep) {
      double off = 0.0;
#pragma unroll
      for (int u = 1; u < KP; ++u) off = fma(a[u], a[u], off);
      const double dg = a[0] * a[0];
      const bool conv = group_sum<KP>(off) <= e.tol2 * group_sum<KP>(dg);
      const bool all = __ballot(!conv) == 0;
      const bool stop = all || sweep >= e.max_sweeps;
      if (stop && !all && jj == 0 && valid && e.status) atomicOr(e.status, kStatNotconv);
      if (lane == 0) sh.flag = stop ? 1 : 0;
      block_sync();
      if (stop) break;
      jacobi_sweep_a<KP>(a, jj, cb0, cb1, std::make_integer_sequence<int, KP - 1>{});
    }
    lam = a[0];
    sh.lam[lane] = lam;
    block_sync();                                  // V written by wavefront 1
    block_sync();                                  // eigenvalues published
    if (e.mode != 0) write_eig<KP>(e, M, jj, pl, valid, lam);
  } else {
    double v[KP];
    init_identity<KP>(v);
    block_sync();
    for (;;) {
      block_sync();
      if (sh.flag) break;
      jacobi_sweep_v<KP>(v, jj, cb0, cb1, std::make_integer_sequence<int, KP - 1>{});
    }
    store_rows<KP>(M, jj, v);
    block_sync();
    block_sync();
    lam = sh.lam[lane];
    if (e.mode == 0) {
      if (e.prec == 0)
        transform_update<KP, double>(e, sh, seg, jj, pl, valid, lam);
      else
        transform_update<KP, float>(e, sh, seg, jj, pl, valid, lam);
    }
  }
}

template <int KP>
hipError_t launch_evd_kp(const BatchMap& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const dim3 grid(ceil_div(a.n, 64 / KP));
  if constexpr (KP == 64) {
    hipLaunchKernelGGL(k_evd_split<KP>, grid, dim3(128), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_evd<KP>, grid, dim3(64), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace letkf
