// Eigenpairs of the symmetric tridiagonal matrix T (diagonal d, subdiagonal
// e) by Cuppen's divide and conquer, for one matrix per KP lanes of a
// wavefront (KP a power of two).  Used after the Householder reduction of the
// LETKF ensemble-space matrix (Sec. II-B, the batched EVD of Sec. III).
//
// Method (Cuppen 1981; Dongarra & Sorensen 1987; stable eigenvectors from
// Gu & Eisenstat 1995):
//   * T is torn at every coupling e_i, leaving 1 x 1 leaves d_i - e_{i-1} - e_i;
//   * levels S = 2, 4, .., KP merge two children of size S/2 at the split
//     m = a + S/2:  T_block = diag(Q1 D1 Q1^T, Q2 D2 Q2^T) + beta u u^T with
//     beta = e_{m-1}, u = e_{m-1} + e_m, so the block's eigenproblem is the
//     rank-one update D + beta z z^T of the children's eigenvalues, with
//     z = (last row of Q1, first row of Q2);
//   * poles are sorted; negligible z entries and (rotated) pairs of nearly
//     equal poles are deflated; every other eigenvalue is the root of the
//     secular equation 1/rho + sum_j w_j^2 / (d_j - lambda) = 0 in its own
//     pole interval, found by one lane with a two-pole rational model
//     safeguarded by bisection, in the shifted form lambda = d_org + tau;
//   * the weights are recomputed from the roots (Loewner) so that the
//     eigenvectors (D - lambda I)^-1 zhat are numerically orthogonal;
//   * lane r keeps row r of the tridiagonal eigenvector matrix restricted to
//     its current block (qs[]); the merge matrix W (rows block-local, one
//     column per eigenvalue) is built column-per-lane in LDS.
#pragma once
#include "common.h"

namespace letkf {

template <int KP>
struct DcLds {
  double lam[KP];   // eigenvalues of the current blocks, by position
  double dt[KP];    // signed poles of a merge, block-local original order
  double zb[KP];    // merge vector z
  double ds[KP];    // poles sorted ascending
  double ws[KP];    // weights in sorted order
  double dk[KP];    // non-deflated poles (ascending)
  double wk[KP];    // non-deflated weights
  double rt[KP];    // secular roots: offset tau from the origin pole
  double zh[KP];    // recomputed weights zhat
  double rc[KP];    // deflation rotations: cosine
  double rs[KP];    //                       sine
  int pm[KP];       // sorted position -> block-local original index
  int kp[KP];       // non-deflated index -> sorted position
  int inv[KP];      // sorted position -> non-deflated index, -1 if deflated
  int ro[KP];       // secular roots: origin pole (non-deflated index)
  int rp[KP];       // deflation rotations: first sorted position
  int rj[KP];       //                       second sorted position
  int nk[KP];       // per block (at its base): non-deflated count
  int nr[KP];       //                          rotation count
};

constexpr double kDcEps = 0x1p-52;
constexpr int kSecularMaxIts = 64;

// The root in (lo, hi) of  c0 + B1/(p1 - t) + B2/(p2 - t) = 0  with p1 < p2,
// B1, B2 >= 0 (the function rises from -inf to +inf between the poles);
// NaN if the quadratic gives none.
__device__ __forceinline__ double two_pole_root(double c0, double B1, double B2, double p1,
                                                double p2) {
  const double a = c0;
  const double b = -(c0 * (p1 + p2) + B1 + B2);
  const double c = c0 * p1 * p2 + B1 * p2 + B2 * p1;
  if (a == 0.0) return c / -b;
  const double disc = fmax(b * b - 4.0 * a * c, 0.0);
  const double q = -0.5 * (b + (b >= 0.0 ? sqrt(disc) : -sqrt(disc)));
  const double r1 = q / a;
  const double r2 = q != 0.0 ? c / q : __builtin_nan("");
  return (r1 > p1 && r1 < p2) ? r1 : r2;
}

// Root i (0-based) of 1/rho + sum_{j<K} w_j^2/(d_j - lambda) = 0, d ascending
// (LDS, K entries), rho > 0, every w_j != 0.  Returns the origin pole index
// and tau with lambda = d[org] + tau; *its receives the iteration count.
__device__ __forceinline__ int secular_root(const double* d, const double* w, int K, int i,
                                            double rho, double& tau_out, int& its) {
  const double irho = 1.0 / rho;
  double lo, hi;
  int org;
  if (i < K - 1) {
    const double di = d[i];
    const double mid = 0.5 * (d[i + 1] - di);
    double f = irho;
    for (int j = 0; j < K; ++j) f += w[j] * w[j] / ((d[j] - di) - mid);
    if (f >= 0.0) {
      org = i;
      lo = 0.0;
      hi = mid;
    } else {
      org = i + 1;
      lo = -mid;
      hi = 0.0;
    }
  } else {
    double s = 0.0;
    for (int j = 0; j < K; ++j) s += w[j] * w[j];
    org = K - 1;
    lo = 0.0;
    hi = rho * s * (1.0 + 8.0 * kDcEps);
  }
  const double dorg = d[org];
  const double pi = d[i] - dorg;                         // pole i, shifted
  const double pi1 = i + 1 < K ? d[i + 1] - dorg : 0.0;  // pole i+1 (interior roots)
  const double pm1 = i > 0 ? d[i - 1] - dorg : 0.0;      // pole i-1 (last root)
  // start: the nearest poles exact, the other terms frozen at the midpoint
  double tau;
  {
    const double tm = 0.5 * (lo + hi);
    double rest = irho;
    const int e1 = i, e2 = i < K - 1 ? i + 1 : i;
    for (int j = 0; j < K; ++j)
      if (j != e1 && j != e2) rest += w[j] * w[j] / ((d[j] - dorg) - tm);
    double t0;
    if (i < K - 1)
      t0 = two_pole_root(rest, w[i] * w[i], w[i + 1] * w[i + 1], pi, pi1);
    else
      t0 = rest > 0.0 ? pi + w[i] * w[i] / rest : __builtin_nan("");
    tau = (t0 > lo && t0 < hi) ? t0 : tm;
  }
  its = 0;
  for (int it = 1; it <= kSecularMaxIts; ++it) {
    its = it;
    // psi: terms j <= i, phi: terms j > i (for the last root psi2 = j < K-1)
    double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0, ps2 = 0.0, dps2 = 0.0;
    for (int j = 0; j < K; ++j) {
      const double r = (d[j] - dorg) - tau;
      const double t = w[j] / r;
      const double tw = t * w[j], t2 = t * t;
      if (j <= i) {
        psi += tw;
        dpsi += t2;
      } else {
        phi += tw;
        dphi += t2;
      }
      if (j < K - 1) {
        ps2 += tw;
        dps2 += t2;
      }
    }
    const double f = irho + psi + phi;
    if (fabs(f) <= 4.0 * kDcEps * K * (irho + fabs(psi) + fabs(phi))) break;
    if (f < 0.0)
      lo = tau;
    else
      hi = tau;
    if (hi - lo <= 2.0 * kDcEps * fmax(fabs(lo), fabs(hi))) break;
    double tn;
    if (i < K - 1) {
      const double g1 = pi - tau, g2 = pi1 - tau;
      const double B1 = dpsi * g1 * g1, A1 = psi - dpsi * g1;
      const double B2 = dphi * g2 * g2, A2 = phi - dphi * g2;
      tn = two_pole_root(irho + A1 + A2, B1, B2, pi, pi1);
    } else if (K == 1) {
      const double g1 = pi - tau;
      const double B1 = dpsi * g1 * g1, A1 = psi - dpsi * g1;
      const double c0 = irho + A1;
      tn = c0 > 0.0 ? pi + B1 / c0 : __builtin_nan("");
    } else {
      // last root: the terms j < K-1 modelled by a pole at pole K-2, the last
      // pole's own term exact; the wanted root is the larger one
      const double g1 = pm1 - tau;
      const double B1 = dps2 * g1 * g1, A1 = ps2 - dps2 * g1;
      const double B2 = w[i] * w[i];
      const double c0 = irho + A1;
      tn = __builtin_nan("");
      if (c0 > 0.0) {
        const double a = c0, b = -(c0 * (pm1 + pi) + B1 + B2), c = c0 * pm1 * pi + B1 * pi + B2 * pm1;
        const double disc = fmax(b * b - 4.0 * a * c, 0.0);
        const double q = -0.5 * (b + (b >= 0.0 ? sqrt(disc) : -sqrt(disc)));
        const double r1 = q / a, r2 = q != 0.0 ? c / q : r1;
        tn = fmax(r1, r2);
      }
    }
    tau = (tn > lo && tn < hi) ? tn : 0.5 * (lo + hi);
  }
  tau_out = tau;
  return org;
}

// One merge level S for every block of the matrix at once.  Lane jj (row jj
// of T) is position t = jj % S of block a = jj - t.  qs[0..S/2) holds, on
// entry, row jj of the child's eigenvector matrix restricted to the child's
// columns; on exit (S < KP) qs[0..S) holds it for the merged block.  At
// S == KP the full row is returned in qs[0..KP).  W is this matrix's LDS
// scratch for the merge matrices (KP * (KP + 1) doubles).
template <int KP, int S>
__device__ __forceinline__ void dc_merge(double (&qs)[KP], DcLds<KP>& L, const double* e_orig,
                                         double* W, int jj, bool& ok) {
  constexpr int H = S / 2;
  constexpr int WS = S + 1;                  // row stride of a block's merge matrix
  const int t = jj & (S - 1);
  const int a = jj - t;
  const int m = a + H;
  double* Wb = W + (a / S) * S * WS;         // this block's merge matrix
  // z: last row of the left child, first row of the right child
  if (jj == m - 1) {
#pragma unroll
    for (int q = 0; q < H; ++q) L.zb[a + q] = qs[q];
  }
  if (jj == m) {
#pragma unroll
    for (int q = 0; q < H; ++q) L.zb[m + q] = qs[q];
  }
  const double beta = e_orig[m - 1];
  const bool flip = beta < 0.0;
  const double D = flip ? -L.lam[jj] : L.lam[jj];
  L.dt[jj] = D;
  wave_lds_sync();
  const double z = L.zb[jj];
  const double nz2 = group_sum<S>(z * z);
  const double rho = fabs(beta) * nz2;
  const bool trivial = !(rho > 0.0);               // uniform per block
  const double w = trivial ? 0.0 : z / sqrt(nz2);
  // sort the poles (ties by index)
  int rank = 0;
  for (int u = 0; u < S; ++u) {
    const double Du = L.dt[a + u];
    rank += (Du < D || (Du == D && u < t)) ? 1 : 0;
  }
  L.ds[a + rank] = D;
  L.ws[a + rank] = w;
  L.pm[a + rank] = t;
  const double tol = 8.0 * kDcEps * fmax(group_max<S>(fabs(D)), rho);
  wave_lds_sync();
  // deflation scan (sequential, one lane per block)
  if (t == 0 && !trivial) {
    int prev = -1, K = 0, nrot = 0;
    for (int k = 0; k < S; ++k) {
      double wk = L.ws[a + k];
      if (fabs(rho * wk) <= tol) {
        L.ws[a + k] = 0.0;
        L.inv[a + k] = -1;
        continue;
      }
      L.inv[a + k] = 0;
      if (prev >= 0) {
        const double wp = L.ws[a + prev];
        const double tt = sqrt(fma(wp, wp, wk * wk));
        const double c = wk / tt, s = wp / tt;
        const double dp = L.ds[a + prev], dj = L.ds[a + k];
        if (fabs((dj - dp) * c * s) <= tol) {
          L.ds[a + prev] = fma(c * c, dp, s * s * dj);
          L.ds[a + k] = fma(s * s, dp, c * c * dj);
          L.ws[a + prev] = 0.0;
          L.ws[a + k] = tt;
          L.inv[a + prev] = -1;
          L.rp[a + nrot] = prev;
          L.rj[a + nrot] = k;
          L.rc[a + nrot] = c;
          L.rs[a + nrot] = s;
          ++nrot;
        }
      }
      prev = k;
    }
    for (int k = 0; k < S; ++k) {
      if (L.inv[a + k] >= 0) {
        L.inv[a + k] = K;
        L.kp[a + K] = k;
        ++K;
      }
    }
    L.nk[a] = K;
    L.nr[a] = nrot;
  }
  wave_lds_sync();
  const int K = trivial ? 0 : L.nk[a];
  if (t < K) {
    const int sp = L.kp[a + t];
    L.dk[a + t] = L.ds[a + sp];
    L.wk[a + t] = L.ws[a + sp];
  }
  wave_lds_sync();
  // secular roots, one per lane
  if (t < K) {
    double tau;
    int its;
    const int org = secular_root(L.dk + a, L.wk + a, K, t, rho, tau, its);
    if (its >= kSecularMaxIts) ok = false;
    L.ro[a + t] = org;
    L.rt[a + t] = tau;
  }
  wave_lds_sync();
  // Loewner: zhat_j^2 = (1/rho) prod_i (lambda_i - d_j) / prod_{i != j} (d_i - d_j)
  if (t < K) {
    const double dj = L.dk[a + t];
    double prod = 1.0 / rho;
    for (int i = 0; i < K; ++i) {
      const double num = (L.dk[a + L.ro[a + i]] - dj) + L.rt[a + i];
      prod *= i == t ? num : num / (L.dk[a + i] - dj);
    }
    const double zr = sqrt(fmax(prod, 0.0));
    L.zh[a + t] = L.wk[a + t] >= 0.0 ? zr : -zr;
  }
  wave_lds_sync();
  // column t of the merge matrix (sorted eigenvalue order; rows block-local)
  double lam_new;
  for (int r = 0; r < S; ++r) Wb[r * WS + t] = 0.0;
  if (trivial) {
    Wb[t * WS + t] = 1.0;
    lam_new = D;
  } else {
    const int ti = L.inv[a + t];
    if (ti < 0) {
      Wb[L.pm[a + t] * WS + t] = 1.0;
      lam_new = L.ds[a + t];
    } else {
      const int org = L.ro[a + ti];
      const double tau = L.rt[a + ti];
      const double dorg = L.dk[a + org];
      double nrm = 0.0;
      for (int u = 0; u < K; ++u) {
        const double v = L.zh[a + u] / ((L.dk[a + u] - dorg) - tau);
        nrm = fma(v, v, nrm);
      }
      const double inrm = 1.0 / sqrt(nrm);
      for (int u = 0; u < K; ++u) {
        const double v = L.zh[a + u] / ((L.dk[a + u] - dorg) - tau);
        Wb[L.pm[a + L.kp[a + u]] * WS + t] = v * inrm;
      }
      lam_new = dorg + tau;
    }
    // deflation rotations, last first, on rows pm[p], pm[j] of this column
    const int nrot = L.nr[a];
    for (int q = nrot - 1; q >= 0; --q) {
      const int rpi = L.pm[a + L.rp[a + q]] * WS + t;
      const int rji = L.pm[a + L.rj[a + q]] * WS + t;
      const double c = L.rc[a + q], s = L.rs[a + q];
      const double xp = Wb[rpi], xj = Wb[rji];
      Wb[rpi] = fma(c, xp, s * xj);
      Wb[rji] = fma(-s, xp, c * xj);
    }
  }
  L.lam[jj] = flip ? -lam_new : lam_new;
  wave_lds_sync();
  // this lane's row of the merged block's eigenvector matrix
  const int h0 = t < H ? 0 : H;              // first W row of this lane's child
  double out[S];
#pragma unroll
  for (int c = 0; c < S; ++c) out[c] = 0.0;
#pragma unroll
  for (int q = 0; q < H; ++q) {
    const double x = qs[q];
    const double* Wr = Wb + (h0 + q) * WS;
#pragma unroll
    for (int c = 0; c < S; ++c) out[c] = fma(x, Wr[c], out[c]);
  }
#pragma unroll
  for (int c = 0; c < S; ++c) qs[c] = out[c];
  wave_lds_sync();
}

template <int KP, int S>
__device__ __forceinline__ void dc_levels(double (&qs)[KP], DcLds<KP>& L, const double* e_orig,
                                          double* W, int jj, bool& ok) {
  if constexpr (S <= KP) {
    dc_merge<KP, S>(qs, L, e_orig, W, jj, ok);
    dc_levels<KP, 2 * S>(qs, L, e_orig, W, jj, ok);
  }
}

// Eigen-decomposition of the tridiagonal (d, e) (LDS, KP entries each; e
// is not modified).  On return L.lam[jj] is the eigenvalue of column jj and
// qs[] is row jj of the eigenvector matrix.  Returns false if a secular root
// ran out of iterations.
template <int KP>
__device__ __forceinline__ bool dc_tridiagonal(double (&qs)[KP], DcLds<KP>& L, const double* d,
                                               const double* e, double* W, int jj) {
  const double el = jj > 0 ? e[jj - 1] : 0.0;
  L.lam[jj] = d[jj] - el - e[jj];            // leaves after tearing every coupling
#pragma unroll
  for (int c = 0; c < KP; ++c) qs[c] = c == 0 ? 1.0 : 0.0;
  wave_lds_sync();
  bool ok = true;
  dc_levels<KP, 2>(qs, L, e, W, jj, ok);
  return ok;
}

}  // namespace letkf
