// Batched inverse square root of symmetric positive definite matrices by the
// coupled Newton-Schulz iteration, FP64 on MFMA: the direct route to the
// symmetric square-root transform W = sqrt(k-1) Q^-1/2 of the LETKF (eq.
// letkf_dwa) that avoids the eigendecomposition of Q (the alternative the
// paper's batched-EVD section leaves for future work).
//
// With A scaled by s = min(||A||_F, ||A||_inf) >= lambda_max(A), the
// eigenvalues of B = A / s lie in (0, 1], and (Higham, Functions of Matrices,
// Sec. 6.7, the Newton-Schulz form of the Denman-Beavers pair)
//     Y_0 = B,  Z_0 = I,  T_i = (3 I - Z_i Y_i) / 2,
//     Y_{i+1} = Y_i T_i,  Z_{i+1} = T_i Z_i
// takes Y to B^1/2 and Z to B^-1/2: each eigenvalue pair follows
// y <- y t, z <- t z with t = (3 - z y) / 2, which grows z y by 9/4 per step
// while it is small and converges quadratically near 1.  Then
// A^-1/2 = Z / sqrt(s).  In exact arithmetic every iterate is a symmetric
// polynomial in B; in floating point the products are formed in full and in
// this order, because the one-matrix form X <- X (3 I - B X^2) / 2 amplifies
// rounding once cond(B) > 9, and forcing each product symmetric does the same
// to the coupled pair.  Accuracy: about 1e-17 cond(A) relative (rounding in the
// steps of the growth phase), which the residual does not show; for the LETKF
// matrix cond(Q) <= 1 + rho lambda_max(C) / (k - 1).
//
// Two kernels share the iteration: k_nsqrt (matrices in, A^-1/2 out) and
// k_nsqrt_xf, the transform-and-update step of an analysis in its place of
// the eigensolve: Q = C + ((k-1)/rho) I from the Gram blocks, then
// wbar = Q^-1 b = Z (Z b) / s, W = sqrt(k-1) Z / sqrt(s) (eqs. letkf_wa,
// letkf_dwa) and X^a = xbar + dX (wbar 1^T + W) (eq. letkf_xa), in place.
//
// One matrix per block, padded to KP = 16 ceil(k / 16) with B = 1 on the
// padding diagonal (an exact fixed point: the padding stays 1 and never mixes
// with the rest), held in LDS as three full KP x KP matrices Y, Z, T with an
// odd row stride; the 16 x 16 tiles of each product are shared out over the
// block's wavefronts and formed on v_mfma_f64_16x16x4f64.  A step ends after
// the one that finds ||Z Y - I||_F <= 1e-12 KP (its update takes the error,
// quadratically, below the rounding level of the products), or when that
// residual stops falling fourfold per step at or below 1e-6 KP (its rounding
// floor); a stall above it after step 48, or 64 steps, sets the status bit of
// LETKF_ENOTCONV (a matrix that is not positive definite diverges and ends
// there).
#include "common.h"
#include "launch.h"

namespace letkf {

constexpr int kNsMaxSteps = 64;

// Tile (I, J) of the product P = X Z of two LDS matrices (row stride LD), in
// the accumulator layout: lane l, element r holds P[16I + 4r + l/16][16J + l%16].
template <int NQ, int LD>
__device__ __forceinline__ double4_t ns_tile(const double* X, const double* Z, int I, int J, int g,
                                             int c) {
  double4_t acc = {0.0, 0.0, 0.0, 0.0};
  const double* xr = X + (16 * I + c) * LD + g;
  const double* zc = Z + g * LD + 16 * J + c;
#pragma unroll
  for (int K = 0; K < NQ; ++K) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xr[16 * K + 4 * r], zc[(16 * K + 4 * r) * LD], acc,
                                                 0, 0, 0);
  }
  return acc;
}

__device__ __forceinline__ void ns_put(double* S, int LD, int I, int J, const double4_t& t, int g,
                                       int c) {
#pragma unroll
  for (int r = 0; r < 4; ++r) S[(16 * I + 4 * r + g) * LD + 16 * J + c] = t[r];
}

template <int NQ>
struct NsLds {
  static constexpr int KP = 16 * NQ, LD = KP + 1;
  double Y[KP * LD];
  double Z[KP * LD];
  double T[KP * LD];
  double red[2][8];
};

// Block sum (op 0) or maximum (op 1) of one value per lane.
template <int NW>
__device__ __forceinline__ double ns_block_reduce(double v, double* red, int op) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  v = op == 0 ? group_sum<64>(v) : group_max<64>(v);
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = op == 0 ? 0.0 : red[0];
#pragma unroll
  for (int i = 0; i < NW; ++i) t = op == 0 ? t + red[i] : fmax(t, red[i]);
  __syncthreads();
  return t;
}

// With Y holding the symmetric A (k x k of the KP x KP array, unscaled),
// scales it to B = A / s, pads it, sets Z = I and runs the iteration; Z then
// holds B^-1/2.  Returns s; conv and taken report the ending.
template <int NQ, int NW>
__device__ double ns_run(NsLds<NQ>& sh, int k, bool& conv, int& taken) {
  constexpr int KP = 16 * NQ, LD = KP + 1, TPW = NQ * NQ / NW;
  static_assert(TPW * NW == NQ * NQ, "tiles must divide over the wavefronts");
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, c = lane & 15;
  // s = min(||A||_F, ||A||_inf)
  double ss = 0.0, rowmax = 0.0;
  for (int i = w; i < k; i += NW) {
    double rs = 0.0;
    for (int j = lane; j < k; j += 64) {
      const double v = sh.Y[i * LD + j];
      ss += v * v;
      rs += fabs(v);
    }
    rowmax = fmax(rowmax, group_sum<64>(rs));
  }
  const double fro2 = ns_block_reduce<NW>(ss, sh.red[0], 0);
  const double inf = ns_block_reduce<NW>(rowmax, sh.red[1], 1);
  const double s = fmin(sqrt(fro2), inf);
  const double inv_s = 1.0 / s;
  for (int e = tid; e < KP * KP; e += 64 * NW) {
    const int i = e / KP, j = e - i * KP;
    const bool real = i < k && j < k;
    sh.Y[i * LD + j] = real ? sh.Y[i * LD + j] * inv_s : (i == j ? 1.0 : 0.0);
    sh.Z[i * LD + j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  conv = false;
  taken = kNsMaxSteps;
  double prev = 1e300;
  constexpr double kTol2 = 1e-24 * KP * KP;
  constexpr double kFloor2 = 1e-12 * KP * KP;
  for (int it = 0; it < kNsMaxSteps; ++it) {
    // T = (3 I - Z Y) / 2 and ||Z Y - I||_F^2
    double e2 = 0.0;
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int u = w + NW * q, I = u / NQ, J = u - I * NQ;
      const double4_t n = ns_tile<NQ, LD>(sh.Z, sh.Y, I, J, g, c);
      double4_t t;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double d = (I == J && 4 * r + g == c) ? 1.0 : 0.0;
        const double e = n[r] - d;
        e2 += e * e;
        t[r] = 1.5 * d - 0.5 * n[r];
      }
      ns_put(sh.T, LD, I, J, t, g, c);
    }
    e2 = group_sum<64>(e2);
    if (lane == 0) sh.red[0][w] = e2;
    __syncthreads();
    double err = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) err += sh.red[0][i];
    // Y <- Y T, Z <- T Z (formed in registers, written after every read)
    double4_t yn[TPW], zn[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int u = w + NW * q, I = u / NQ, J = u - I * NQ;
      yn[q] = ns_tile<NQ, LD>(sh.Y, sh.T, I, J, g, c);
      zn[q] = ns_tile<NQ, LD>(sh.T, sh.Z, I, J, g, c);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int u = w + NW * q, I = u / NQ, J = u - I * NQ;
      ns_put(sh.Y, LD, I, J, yn[q], g, c);
      ns_put(sh.Z, LD, I, J, zn[q], g, c);
    }
    __syncthreads();
    if (err <= kTol2) {          // this step was the last one needed (uniform)
      conv = true;
      taken = it + 1;
      break;
    }
    if (!(err < 0.25 * prev)) {  // no longer falling quadratically
      if (err <= kFloor2) {      // the rounding floor of the residual
        conv = true;
        taken = it + 1;
        break;
      }
      if (it >= 48) {            // stalled far from I: not converged
        taken = it + 1;
        break;
      }
    }
    prev = err;
  }
  return s;
}

// Wavefronts per block for NQ x NQ tiles (NQ^2 / NW tiles of each product per
// wavefront; the LDS of three KP x KP matrices allows 1 to 24 blocks per CU).
template <int NQ>
constexpr int ns_waves() {
  return NQ == 1 ? 1 : NQ == 2 ? 2 : NQ == 3 ? 3 : 8;
}

template <int NQ>
__global__ __launch_bounds__(64 * ns_waves<NQ>()) void k_nsqrt(const double* __restrict__ a,
                                                               int batch, int k,
                                                               double* __restrict__ x, int* status,
                                                               int* __restrict__ steps) {
  constexpr int NW = ns_waves<NQ>(), KP = 16 * NQ, LD = KP + 1;
  __shared__ NsLds<NQ> sh;
  const int tid = threadIdx.x;
  const int m = blockIdx.x;
  const double* am = a + (size_t)m * k * k;
  for (int e = tid; e < k * k; e += 64 * NW) {
    const int i = e / k, j = e - i * k;
    sh.Y[i * LD + j] = ldg(am, e);
  }
  __syncthreads();
  bool conv;
  int taken;
  const double s = ns_run<NQ, NW>(sh, k, conv, taken);
  if (!conv && tid == 0 && status) atomicOr(status, kStatNotconv);
  if (tid == 0 && steps) steps[m] = taken;
  const double r_s = 1.0 / sqrt(s);
  double* xm = x + (size_t)m * k * k;
  for (int e = tid; e < k * k; e += 64 * NW) {
    const int i = e / k, j = e - i * k;
    xm[e] = sh.Z[i * LD + j] * r_s;
  }
}

// One grid point of an analysis slab per block: Q from the Gram output
// (upper 16 x 16 blocks of C, KPC = the launch's padded order), the
// iteration on it, then the transform and update of the point's nine
// components in place (the point-major ensemble, [9][k] per point).
template <int NQ, int KPC>
__global__ __launch_bounds__(64 * ns_waves<NQ>()) void k_nsqrt_xf(BatchMap bm) {
  constexpr int NW = ns_waves<NQ>(), KP = 16 * NQ, LD = KP + 1;
  constexpr int NQC = KPC / 16, NB = NQC * (NQC + 1) / 2;
  static_assert(KP <= KPC, "the iteration's order may not exceed the Gram's");
  __shared__ NsLds<NQ> sh;
  __shared__ double wb[KP];
  __shared__ double xbar[9];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int pl = blockIdx.x;
  bool valid;
  const EvdArgs e = evd_args_of(bm, pl, valid);
  if (!valid) return;                       // uniform over the block
  const int k = e.k;
  const double* Cp = e.C + (size_t)pl * NB * 256;
  // Q = C + alpha I, entry (i, j) from block (min(I,J), max(I,J)); diagonal
  // blocks hold both triangles
  for (int u = tid; u < k * k; u += 64 * NW) {
    const int i = u / k, j = u - i * k;
    const int I = i >> 4, J = j >> 4;
    const int lo = I < J ? I : J, hi = I < J ? J : I;
    const int blk = lo * NQC - lo * (lo - 1) / 2 + (hi - lo);
    const int off = I <= J ? (i & 15) * 16 + (j & 15) : (j & 15) * 16 + (i & 15);
    sh.Y[i * LD + j] = ldg(Cp + blk * 256, off) + (i == j ? e.alpha : 0.0);
  }
  __syncthreads();
  bool conv;
  int taken;
  const double s = ns_run<NQ, NW>(sh, k, conv, taken);
  if (!conv && tid == 0 && e.status) atomicOr(e.status, kStatNotconv);
  // v = Z b (into the first row of T), then wbar = Z v / s
  const double* bp = e.b + (size_t)pl * KPC;
  for (int i = tid; i < k; i += 64 * NW) {
    double acc = 0.0;
    for (int j = 0; j < k; ++j) acc = fma(sh.Z[i * LD + j], ldg(bp, j), acc);
    sh.T[i] = acc;
  }
  __syncthreads();
  const double inv_s = 1.0 / s;
  for (int i = tid; i < k; i += 64 * NW) {
    double acc = 0.0;
    for (int j = 0; j < k; ++j) acc = fma(sh.Z[i * LD + j], sh.T[j], acc);
    wb[i] = acc * inv_s;
  }
  // dX: the nine components of the point's members, mean removed (rows of
  // Y, which the iteration no longer needs)
  double* xp = e.xt + (size_t)(e.pt0 + pl) * 9 * k;
  for (int u = tid; u < 9 * k; u += 64 * NW) sh.Y[(u / k) * LD + (u % k)] = ldg(xp, u);
  __syncthreads();
  for (int cpt = w; cpt < 9; cpt += NW) {
    double t = 0.0;
    for (int j = lane; j < k; j += 64) t += sh.Y[cpt * LD + j];
    t = group_sum<64>(t);
    if (lane == 0) xbar[cpt] = t / (double)k;
  }
  __syncthreads();
  for (int u = tid; u < 9 * k; u += 64 * NW) sh.Y[(u / k) * LD + (u % k)] -= xbar[u / k];
  __syncthreads();
  // X^a[c][j] = xbar_c + sum_i dX[c][i] (wbar_i + f Z[i][j]), f = sqrt(k-1) / sqrt(s)
  const double f = e.sqrt_km1 / sqrt(s);
  bool finite = true;
  for (int u = tid; u < 9 * k; u += 64 * NW) {
    const int cpt = u / k, j = u - cpt * k;
    const double* dx = sh.Y + cpt * LD;
    double acc = 0.0;
    for (int i = 0; i < k; ++i) acc = fma(dx[i], fma(f, sh.Z[i * LD + j], wb[i]), acc);
    const double xa = xbar[cpt] + acc;
    finite = finite && __builtin_isfinite(xa);
    xp[u] = xa;
  }
  if (!finite) atomicOr(e.status, kStatNonfinite);
}

hipError_t launch_nsqrt(const double* a, int batch, int k, double* x, int* status, int* steps,
                        hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  switch ((k + 15) / 16) {
    case 1:
      hipLaunchKernelGGL(k_nsqrt<1>, dim3(batch), dim3(64 * ns_waves<1>()), 0, s, a, batch, k, x,
                         status, steps);
      break;
    case 2:
      hipLaunchKernelGGL(k_nsqrt<2>, dim3(batch), dim3(64 * ns_waves<2>()), 0, s, a, batch, k, x,
                         status, steps);
      break;
    case 3:
      hipLaunchKernelGGL(k_nsqrt<3>, dim3(batch), dim3(64 * ns_waves<3>()), 0, s, a, batch, k, x,
                         status, steps);
      break;
    case 4:
      hipLaunchKernelGGL(k_nsqrt<4>, dim3(batch), dim3(64 * ns_waves<4>()), 0, s, a, batch, k, x,
                         status, steps);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The launch's problems share the Gram's padded order kp (16, 32 or 64); the
// iteration runs at that order too (entries past a problem's k are padding).
hipError_t launch_nsqrt_xf(const BatchMap& bm, int kp, hipStream_t s) {
  if (bm.n <= 0) return hipSuccess;
  if (kp == 16)
    hipLaunchKernelGGL((k_nsqrt_xf<1, 16>), dim3(bm.n), dim3(64 * ns_waves<1>()), 0, s, bm);
  else if (kp == 32)
    hipLaunchKernelGGL((k_nsqrt_xf<2, 32>), dim3(bm.n), dim3(64 * ns_waves<2>()), 0, s, bm);
  else if (kp == 64)
    hipLaunchKernelGGL((k_nsqrt_xf<4, 64>), dim3(bm.n), dim3(64 * ns_waves<4>()), 0, s, bm);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace letkf
