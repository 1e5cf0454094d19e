// Eigenpairs of the symmetric tridiagonal matrix T (diagonal d, subdiagonal
// e) by Cuppen's divide and conquer, for one matrix per KP lanes of a
// wavefront (KP a power of two).  Used after the Householder reduction of the
// LETKF ensemble-space matrix (Sec. II-B, the batched EVD of Sec. III).
//
// Method (Cuppen 1981; Dongarra & Sorensen 1987; stable eigenvectors from
// Gu & Eisenstat 1995):
//   * T is torn at every fourth coupling (a torn coupling e_i comes off the
//     two diagonal entries next to it), leaving 4 x 4 leaves that cyclic
//     Jacobi diagonalizes on a quad of lanes (jacobi4);
//   * levels S = 8, 16, .., KP merge two children of size S/2 at the split
//     m = a + S/2:  T_block = diag(Q1 D1 Q1^T, Q2 D2 Q2^T) + beta u u^T with
//     beta = e_{m-1}, u = e_{m-1} + e_m, so the block's eigenproblem is the
//     rank-one update D + beta z z^T of the children's eigenvalues, with
//     z = (last row of Q1, first row of Q2);
//   * poles are sorted; negligible z entries and (rotated) pairs of nearly
//     equal poles are deflated; every other eigenvalue is the root of the
//     secular equation 1/rho + sum_j w_j^2 / (d_j - lambda) = 0 in its own
//     pole interval, found by one lane with a two-pole rational model
//     (secular_root) safeguarded by bisection, in the shifted form
//     lambda = d_org + tau;
//   * the weights are recomputed from the roots (Loewner) so that the
//     eigenvectors (D - lambda I)^-1 zhat are numerically orthogonal;
//   * lane r keeps row r of the tridiagonal eigenvector matrix restricted to
//     its current block (qs[]); the merge matrix W (rows block-local, one
//     column per eigenvalue) is built column-per-lane in LDS.
#pragma once
#include "common.h"

namespace letkf {

// Per-matrix LDS of the merges.  Arrays that share storage are never live at
// once: dt, zb and ws are dead once the keep list is built, before the
// secular roots (rt, rd) and the recomputed weights (zh) are written.
template <int KP>
struct DcLds {
  union {
    double dt[KP];  // signed poles of a merge, block-local original order
    double rt[KP];  // secular roots: offset tau from the origin pole
  };
  union {
    double zb[KP];  // merge vector z
    double rd[KP];  // secular roots: origin pole value
  };
  union {
    double ws[KP];  // weights in sorted order
    double zh[KP];  // recomputed weights zhat
  };
  double ds[KP];    // poles sorted ascending
  // non-deflated (pole, squared weight) pairs, ascending, per block of S slots:
  // slots [2a, 2a + K) and again [2a + K, 2a + 2K), so that a walk over the K - 2
  // poles away from a root, starting just above it and wrapping around,
  // reads consecutive slots
  alignas(16) double2 dw[2 * KP];
  double rc[KP];    // deflation rotations: cosine
  double rs[KP];    //                       sine
  int pm[KP];       // sorted position -> block-local original index
  int inv[KP];      // sorted position -> non-deflated index, -1 if deflated
  int rw[KP];       // non-deflated index -> block-local row of its eigenvector
                    // entry (kRowMask), kNegWeight set when its weight is negative
  // deflation rotations: first | second sorted position << 8; slot S - 1 of
  // a block (never a rotation: a block of S poles has at most S - 2) holds
  // the block's rotation count
  int rot[KP];
};

constexpr int kRowMask = 0xFF;
constexpr int kNegWeight = 0x100;

constexpr double kDcEps = 0x1p-52;
constexpr int kSecularMaxIts = 64;   // room for a full bisection to 2 ulps

// 1/x for finite x != 0 of moderate size: hardware estimate and two
// Newton-Raphson steps.
__device__ __forceinline__ double frcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

// 1/sqrt(x) and sqrt(x) for finite x > 0 of moderate size: hardware
// estimate of 1/sqrt(x), two Newton-Raphson steps, then sqrt(x) = x/sqrt(x)
// with one correction.
__device__ __forceinline__ void rsqrt_sqrt(double x, double& r, double& s) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  double q = x * y;
  q = fma(fma(-q, q, x), 0.5 * y, q);
  r = y;
  s = q;
}

// 1/sqrt(x) for x > 0 and 1/x for finite x != 0: the refined estimates in
// the usual range of their argument, else the IEEE forms.
__device__ __forceinline__ double rsqrt_any(double x) {
  if (x > 1e-280 && x < 1e280) {
    double r, q;
    rsqrt_sqrt(x, r, q);
    return r;
  }
  return 1.0 / sqrt(x);
}
__device__ __forceinline__ double rcp_any(double x) {
  const double ax = fabs(x);
  if (ax > 1e-280 && ax < 1e280) return frcp(x);
  return 1.0 / x;
}

// 1/x to about 10 ulps (the estimate carries about 24 bits; one
// Newton-Raphson step): for the far terms of the secular sums, whose
// rounding the convergence test already allows for (4 eps K sum |terms|).
__device__ __forceinline__ double frcp1(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return fma(y, fma(-x, y, 1.0), y);
}

// The root of  c0 + B1/(p1 - t) + B2/(p2 - t) = 0  (p1 < p2, B1, B2 >= 0: the
// function rises from -inf to +inf between the poles) that lies in the
// bracket (lo, hi) inside (p1, p2); NaN if neither root of the quadratic
// does.  (With a tiny B the quadratic's other root sits just outside a pole
// and can round to inside it, so the pole interval cannot pick the root.)
__device__ __forceinline__ double two_pole_root(double c0, double B1, double B2, double p1,
                                                double p2, double lo, double hi) {
  const double a = c0;
  const double b = -(c0 * (p1 + p2) + B1 + B2);
  const double c = c0 * p1 * p2 + B1 * p2 + B2 * p1;
  // (reciprocals to about an ulp: the result is a model step, checked
  // against the bracket and verified by the next evaluation of f)
  if (a == 0.0) return -c * frcp(b);
  const double disc = fmax(b * b - 4.0 * a * c, 0.0);
  const double q = -0.5 * (b + (b >= 0.0 ? sqrt(disc) : -sqrt(disc)));
  const double r1 = q * frcp(a);
  const double r2 = q != 0.0 ? c * frcp(q) : __builtin_nan("");
  return (r1 > lo && r1 < hi) ? r1 : r2;
}


// One model step of the secular iteration at the iterate t (origin-shifted),
// given f = f(t) and the near terms t1 = W1/(P1 - t), t2 = W2/(P2 - t): the
// near terms exact, the far sum (slope Fd, half curvature Fh at t) replaced
// by c + s1/(P1 - x) + s2/(P2 - x) matched to it in value, slope and
// curvature (interior root) or in value and slope on P1 alone (root above
// the last pole).  The model is solved for the step eta = x - t around the
// evaluated f rather than for x from its constant and pole weights: a far
// pole next to a near one puts a large weight on the other model pole, and
// the constant then cancels against that pole's term, which would lose f
// (and stall the iteration short of the root).  Returns the model's root in
// (lo, hi), or NaN.
__device__ __forceinline__ double secular_model_step(double f, double t1, double t2, double Fd,
                                                     double Fh, double P1, double P2, double t,
                                                     double lo, double hi, bool last, int K,
                                                     double irho) {
  const double g1 = P1 - t, g2 = P2 - t;
  // split of F' over the model poles: a1 = s1/g1^2, a2 = s2/g2^2
  double a1, a2;
  if (last) {
    a1 = Fd;
    a2 = 0.0;
  } else {
    const double ig = frcp(g2 - g1);
    a1 = fmax((Fh * g2 - Fd) * g1 * ig, 0.0);
    a2 = fmax((Fd - Fh * g1) * g2 * ig, 0.0);
  }
  // a single pole (no far terms): f(x) = 1/rho + W2/(P2 - x) has its root at
  // P2 + rho W2, with W2 = t2 g2
  if (K == 1) return P2 + t2 * g2 * frcp(irho);
  // the model's pole terms at t, and the model times (g1 - eta)(g2 - eta):
  //   A eta^2 + B eta + C = 0
  const double s1 = t1 + a1 * g1, s2 = t2 + a2 * g2;
  const double A = f - s1 - s2;
  const double B = s1 * g2 + s2 * g1 - f * (g1 + g2);
  const double C = f * g1 * g2;
  if (A == 0.0) return B != 0.0 ? t - C * frcp(B) : __builtin_nan("");
  const double disc = fmax(B * B - 4.0 * A * C, 0.0);
  const double q = -0.5 * (B + (B >= 0.0 ? sqrt(disc) : -sqrt(disc)));
  const double x1 = t + q * frcp(A);
  const double x2 = q != 0.0 ? t + C * frcp(q) : __builtin_nan("");
  return (x1 > lo && x1 < hi) ? x1 : x2;
}

// Root i (0-based) of f(lambda) = 1/rho + sum_j w_j^2/(d_j - lambda) = 0 over
// the K pairs dw[j] = (d_j, w_j^2) (LDS, d ascending, w_j != 0, rho > 0; slots
// K .. 2K-1 repeat slots 0 .. K-1).  Returns the origin pole index with
// lambda = d[org] + tau_out; conv is cleared if the iteration limit was hit.
//
// Every step keeps the terms of the two poles nearest the root (e1 < e2)
// exact and replaces the sum F of the K - 2 others by c + s1/(P1 - t) +
// s2/(P2 - t) on the same two poles, matching F and its first two
// derivatives at the current iterate (Borges & Gragg 1993): cubic
// convergence, and s1, s2 >= 0 for an interior root, so the model rises
// monotonically between its poles.  For the root above the last pole both
// model poles lie below it and the far terms are matched in value and slope
// on P1 alone.  Each model is solved for the step from the iterate (see
// secular_model_step).  A bracket from the signs of f safeguards every step.
__device__ __forceinline__ int secular_root(const double2* dw, int K, int i, double rho,
                                            double& tau_out, bool& conv) {
  const double irho = rcp_any(rho);
  const bool last = i == K - 1;
  const double di = dw[i].x;
  const double di1 = last ? di : dw[i + 1].x;
  double s2 = 0.0;
#pragma unroll 8
  for (int j = 0; j < K; ++j) s2 += dw[j].y;
  // probe point: the interval midpoint (last root: halfway to d + rho |w|^2),
  // evaluated in coordinates shifted to d_i (d_j - d_i is exact for the
  // nearby poles, d_j - (d_i + half) would not be when the gap is tiny)
  const double gap = last ? rho * s2 : di1 - di;
  const double half = 0.5 * gap;
  double fm = irho, ti = 0.0, ti1 = 0.0;
#pragma unroll 8
  for (int j = 0; j < K; ++j) {
    const double2 p = dw[j];
    const double t = p.y * frcp((p.x - di) - half);
    fm += t;
    ti = j == i ? t : ti;
    ti1 = j == i + 1 ? t : ti1;
  }
  // origin: the pole nearer the root (the sign of f at the midpoint); the
  // bracket is that half of the interval (its far end excludes the other
  // pole, next to which the model's second root can round into the interval)
  int org;
  double lo, hi;
  if (last) {
    org = i;
    lo = 0.0;
    hi = gap * (1.0 + 8.0 * kDcEps);
  } else if (fm >= 0.0) {
    org = i;
    lo = 0.0;
    hi = half;
  } else {
    org = i + 1;
    lo = -half;
    hi = 0.0;
  }
  const double dorg = last || fm >= 0.0 ? di : di1;
  const double pi = di - dorg, pi1 = di1 - dorg;
  const double pm1 = i > 0 ? dw[i - 1].x - dorg : 0.0;
  const double wi2 = dw[i].y;
  const double wi12 = last ? 0.0 : dw[i + 1].y;
  // start: the nearest poles exact, the other terms frozen at their value at
  // the probe (a model matched in slope and curvature there as well
  // extrapolates badly to a root that hugs a pole, the common case with
  // small weights)
  double tau;
  {
    const double tm = fm >= 0.0 || last ? half : -half;   // the probe, shifted to the origin
    const double rest = fm - ti - ti1;
    const double t0 = last ? (rest > 0.0 ? pi + wi2 * frcp(rest) : __builtin_nan(""))
                           : two_pole_root(rest, wi2, wi12, pi, pi1, lo, hi);
    tau = (t0 > lo && t0 < hi) ? t0 : tm;
  }
  const int e1 = last ? i - 1 : i;           // the two poles nearest the root; -1 when K == 1
  const int e2 = last ? i : i + 1;
  const double P1 = last ? pm1 : pi, P2 = last ? pi : pi1;
  const double W1 = e1 >= 0 ? dw[e1].y : 0.0, W2 = dw[e2].y;
  // the far poles: e2 + 1, .., K - 1, 0, .., e1 - 1 (the same count on every
  // lane of the block, so the lanes' loops stay in step)
  const double2* far = dw + e2 + 1;
  const int nfar = K - 2;
  conv = false;
  // sum |terms| of the far terms, for the convergence test's rounding bound:
  // taken at the first iterate (it changes little as the iterate converges
  // and only scales the test)
  double A = 0.0;
  for (int it = 0; it < kSecularMaxIts; ++it) {
    // F, F' and F''/2 of the far terms at tau, in two chains
    double F0 = 0.0, D0 = 0.0, E0 = 0.0;
    double F1 = 0.0, D1 = 0.0, E1 = 0.0;
    int o = 0;
    if (it == 0) {
      double A0 = 0.0, A1 = 0.0;
#pragma unroll 4
      for (; o + 1 < nfar; o += 2) {
        const double2 p = far[o], q = far[o + 1];
        const double r0 = frcp1((p.x - dorg) - tau);
        const double r1 = frcp1((q.x - dorg) - tau);
        const double t0 = p.y * r0, t1 = q.y * r1;
        const double u0 = t0 * r0, u1 = t1 * r1;
        F0 += t0;
        A0 += fabs(t0);
        D0 += u0;
        E0 = fma(u0, r0, E0);
        F1 += t1;
        A1 += fabs(t1);
        D1 += u1;
        E1 = fma(u1, r1, E1);
      }
      if (o < nfar) {
        const double2 p = far[o];
        const double r0 = frcp1((p.x - dorg) - tau);
        const double t0 = p.y * r0;
        const double u0 = t0 * r0;
        F0 += t0;
        A0 += fabs(t0);
        D0 += u0;
        E0 = fma(u0, r0, E0);
      }
      A = A0 + A1;
    } else {
#pragma unroll 4
      for (; o + 1 < nfar; o += 2) {
        const double2 p = far[o], q = far[o + 1];
        const double r0 = frcp1((p.x - dorg) - tau);
        const double r1 = frcp1((q.x - dorg) - tau);
        const double t0 = p.y * r0, t1 = q.y * r1;
        const double u0 = t0 * r0, u1 = t1 * r1;
        F0 += t0;
        D0 += u0;
        E0 = fma(u0, r0, E0);
        F1 += t1;
        D1 += u1;
        E1 = fma(u1, r1, E1);
      }
      if (o < nfar) {
        const double2 p = far[o];
        const double r0 = frcp1((p.x - dorg) - tau);
        const double t0 = p.y * r0;
        const double u0 = t0 * r0;
        F0 += t0;
        D0 += u0;
        E0 = fma(u0, r0, E0);
      }
    }
    const double F = F0 + F1, Fd = D0 + D1, Fh = E0 + E1;
    const double g1 = P1 - tau, g2 = P2 - tau;
    const double t1 = e1 >= 0 ? W1 * frcp(g1) : 0.0;
    const double t2 = W2 * frcp(g2);
    const double f = irho + F + t1 + t2;
    if (fabs(f) <= 4.0 * kDcEps * K * (irho + A + fabs(t1) + fabs(t2))) {
      conv = true;
      break;
    }
    if (f < 0.0)
      lo = tau;
    else
      hi = tau;
    if (hi - lo <= 2.0 * kDcEps * fmax(fabs(lo), fabs(hi))) {
      conv = true;
      break;
    }
    const double tn = secular_model_step(f, t1, t2, Fd, Fh, P1, P2, tau, lo, hi, last, K, irho);
    const bool inside = tn > lo && tn < hi;
    const double tnew = inside ? tn : 0.5 * (lo + hi);
    // a model step (not a bisection) this small has converged: the model
    // matches f to second order or better, so the next step would move tau
    // by an ulp
    const bool done = inside && fabs(tnew - tau) <= 2.0 * kDcEps * fabs(tnew);
    tau = tnew;
    if (done) {
      conv = true;
      break;
    }
  }
  tau_out = tau;
  return org;
}

// What a merge of two children leaves to the construction of its
// eigenvectors (per lane; block-uniform fields marked).
struct MergeRoots {
  double D;        // this lane's pole (child eigenvalue, sign-flipped when beta < 0)
  bool flip;       // beta < 0: the rank-one update was solved for -T (block-uniform)
  bool trivial;    // beta z z^T = 0: the block stays decoupled (block-uniform)
  int K;           // non-deflated poles (block-uniform)
};

// The eigenvalue problem of one merge level S for every block of the matrix
// at once: lane jj (column jj of the children's eigenvector matrix, position
// t = jj % S of block a = jj - t) holds the children's eigenvalue lam and the
// entry z of the merge vector at its column (the left child's last row, the
// right child's first row); beta = e_{m-1} is the torn coupling.  Sorts the
// poles, deflates, solves the secular equation (one root per lane) and
// recomputes the weights (Loewner); on return L holds, per block: the sorted
// poles ds and their original positions pm, the deflation map inv, the
// rotations rot/rc/rs, the non-deflated pairs dw with their rows rw, the
// roots (rd, rt) and the recomputed weights zh.
template <int KP, int S>
__device__ __forceinline__ MergeRoots merge_roots(double z, double lam, double beta,
                                                  DcLds<KP>& L, int jj, double deps, bool& ok) {
  const int t = jj & (S - 1);
  const int a = jj - t;
  const int sh0 = (lane_id() & ~(S - 1));    // first lane of this block in the wavefront
  MergeRoots mr;
  const bool flip = beta < 0.0;
  const double D = flip ? -lam : lam;
  mr.D = D;
  mr.flip = flip;
  L.dt[jj] = D;
  wave_lds_sync();
  const double nz2 = group_sum<S>(z * z);
  const double rho = fabs(beta) * nz2;
  const bool trivial = !(rho > 0.0);               // uniform per block
  mr.trivial = trivial;
  const double w = trivial ? 0.0 : z * rsqrt_any(nz2);
  // sort the poles (ties by index)
  int rank = 0;
#pragma unroll 8
  for (int u = 0; u < S; ++u) {
    const double Du = L.dt[a + u];
    rank += (Du < D || (Du == D && u < t)) ? 1 : 0;
  }
  L.ds[a + rank] = D;
  L.ws[a + rank] = w;
  L.pm[a + rank] = t;
  const double tol = 8.0 * deps * fmax(group_max<S>(fabs(D)), rho);
  wave_lds_sync();
  // deflation: negligible weights (lane-parallel), then pairs of close poles
  // (sequential, by one lane per block, over the sorted order).  A pair (p, k)
  // of neighbouring surviving poles is rotated when |(d_k - d_p) c s| <= tol
  // for the rotation (c, s) = (w_k, w_p) / |(w_p, w_k)| that zeroes w_p,
  // i.e. |d_k - d_p| |w_k w_p| <= tol (w_p^2 + w_k^2).  Every pair is first
  // tested with the unrotated values, lane-parallel (the candidates); a
  // rotation changes only the pair it acts on (p is deflated, k takes the
  // rotated values), so only the pair after a rotation can change its
  // answer: the scan goes from candidate to candidate and follows each
  // chain of rotations while the test of the next pair passes.  The
  // decisions, their order and the arithmetic are those of a scan over
  // every position.
  const uint64_t bmask = S == 64 ? ~0ull : ((1ull << S) - 1ull);
  const double wt = L.ws[a + t], dtt = L.ds[a + t];
  const bool small = !(fabs(rho * wt) > tol);
  L.inv[a + t] = small ? -1 : 0;
  if (small) L.ws[a + t] = 0.0;
  const bool live = !trivial && !small;
  const uint64_t lmask = (__ballot(live) >> sh0) & bmask;
  const uint64_t below = lmask & ((1ull << t) - 1ull);
  bool cand = false;
  if (live && below != 0) {
    const int pp = 63 - __clzll(below);
    const double wp = L.ws[a + pp], dp = L.ds[a + pp];
    cand = fabs(dtt - dp) * fabs(wt * wp) <= tol * fma(wp, wp, wt * wt);
  }
  const uint64_t cmask = (__ballot(cand) >> sh0) & bmask;
  if (t == 0) L.rot[a + S - 1] = 0;
  wave_lds_sync();
  if (t == 0 && cmask != 0) {
    uint64_t cm = cmask, lm = lmask;
    int nrot = 0;
    while (cm != 0) {
      int k = __builtin_ctzll(cm);                          // a candidate and
      int prev = 63 - __clzll(lm & ((1ull << k) - 1ull));   // its surviving left neighbour
      double dp = L.ds[a + prev], wp = L.ws[a + prev];
      double wk = L.ws[a + k], dk = L.ds[a + k];
      bool end = false;
      for (;;) {
        // the next surviving position and its values, read before this
        // step's stores (which touch k and the positions below it only)
        const uint64_t above = k == 63 ? 0ull : lm & ~((2ull << k) - 1ull);
        const int kn = above != 0 ? __builtin_ctzll(above) : k;
        const double wn = L.ws[a + kn], dn = L.ds[a + kn];
        const double nn = fma(wp, wp, wk * wk);
        if (!(fabs(dk - dp) * fabs(wk * wp) <= tol * nn)) break;
        double it, tt;
        rsqrt_sqrt(nn, it, tt);
        const double c = wk * it, sn = wp * it;
        L.ds[a + prev] = fma(c * c, dp, sn * sn * dk);
        L.ws[a + prev] = 0.0;
        L.inv[a + prev] = -1;
        L.rot[a + nrot] = prev | (k << 8);
        L.rc[a + nrot] = c;
        L.rs[a + nrot] = sn;
        ++nrot;
        dp = fma(sn * sn, dp, c * c * dk);
        wp = tt;
        L.ds[a + k] = dp;
        L.ws[a + k] = wp;
        lm &= ~(1ull << prev);
        prev = k;
        if (above == 0) {
          end = true;
          break;
        }
        k = kn;
        wk = wn;
        dk = dn;
      }
      // the candidates up to where the chain stopped have been decided
      cm = (end || k == 63) ? 0ull : cm & ~((2ull << k) - 1ull);
    }
    L.rot[a + S - 1] = nrot;
  }
  wave_lds_sync();
  // keep list: non-deflated sorted positions in order
  const bool keep = !trivial && L.inv[a + t] >= 0;
  const uint64_t kmask = (__ballot(keep) >> sh0) & (S == 64 ? ~0ull : ((1ull << S) - 1ull));
  const int K = __popcll(kmask);
  mr.K = K;
  const int kidx = __popcll(kmask & ((1ull << t) - 1ull));
  if (keep) {
    L.inv[a + t] = kidx;
    const double wv = L.ws[a + t];
    L.rw[a + kidx] = L.pm[a + t] | (wv < 0.0 ? kNegWeight : 0);
    const double2 pr = make_double2(L.ds[a + t], wv * wv);
    L.dw[2 * a + kidx] = pr;
    L.dw[2 * a + K + kidx] = pr;
  }
  wave_lds_sync();
  // secular roots, one per lane
  if (t < K) {
    double tau;
    bool conv;
    const int org = secular_root(L.dw + 2 * a, K, t, rho, tau, conv);
    if (!conv) ok = false;
    L.rd[a + t] = L.dw[2 * a + org].x;
    L.rt[a + t] = tau;
  }
  wave_lds_sync();
  // Loewner: zhat_j^2 = (1/rho) prod_i (lambda_i - d_j) / prod_{i != j} (d_i - d_j)
  if (t < K) {
    const double dj = L.dw[2 * a + t].x;
    double prod = rcp_any(rho);
#pragma unroll 8
    for (int i = 0; i < S; ++i) {
      if (i < K) {
        const double num = (L.rd[a + i] - dj) + L.rt[a + i];
        prod *= i == t ? num : num * frcp(L.dw[2 * a + i].x - dj);
      }
    }
    const double zr = sqrt(fmax(prod, 0.0));
    L.zh[a + t] = (L.rw[a + t] & kNegWeight) ? -zr : zr;
  }
  if (t >= K) L.zh[a + t] = 0.0;
  wave_lds_sync();
  return mr;
}

// One merge level S for every block of the matrix at once.  Lane jj (row jj
// of T) is position t = jj % S of block a = jj - t.  qs[0..S/2) holds, on
// entry, row jj of the child's eigenvector matrix restricted to the child's
// columns; on exit it holds row jj of the merged block's eigenvector matrix
// restricted to the block's columns (qs[0..S)); lam is the eigenvalue of
// column jj of the child on entry, of the merged block on exit.  W is this
// matrix's LDS scratch for the merge matrices (KP * (KP + 1) doubles).
template <int KP, int S>
__device__ __forceinline__ void dc_merge(double (&qs)[KP], double& lam, DcLds<KP>& L,
                                         double ej, double* W, int jj, double deps,
                                         bool& ok) {
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
  const double beta = __shfl(ej, m - 1, KP);   // e_{m-1}, held by lane m - 1
  wave_lds_sync();
  const double z = L.zb[jj];
  const MergeRoots mr = merge_roots<KP, S>(z, lam, beta, L, jj, deps, ok);
  const bool trivial = mr.trivial, flip = mr.flip;
  const double D = mr.D;
  const int K = mr.K;
  // column t of the merge matrix (sorted eigenvalue order; rows block-local),
  // left unnormalized: its scale cs goes to the padding column of row t and
  // is applied to the merged rows below (the rotations commute with it)
  double lam_new, cs = 1.0;
#pragma unroll 8
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
      const double tau = L.rt[a + ti];
      const double dorg = L.rd[a + ti];
      double nrm = 0.0;
#pragma unroll 8
      for (int u = 0; u < K; ++u) {
        const double v = L.zh[a + u] * frcp((L.dw[2 * a + u].x - dorg) - tau);
        nrm = fma(v, v, nrm);
        Wb[(L.rw[a + u] & kRowMask) * WS + t] = v;
      }
      cs = rsqrt_any(nrm);
      lam_new = dorg + tau;
    }
    // deflation rotations, last first, on rows pm[p], pm[j] of this column
    const int nrot = L.rot[a + S - 1];
    for (int q = nrot - 1; q >= 0; --q) {
      const int pj = L.rot[a + q];
      const int rpi = L.pm[a + (pj & 255)] * WS + t;
      const int rji = L.pm[a + (pj >> 8)] * WS + t;
      const double c = L.rc[a + q], sn = L.rs[a + q];
      const double xp = Wb[rpi], xj = Wb[rji];
      Wb[rpi] = fma(c, xp, sn * xj);
      Wb[rji] = fma(-sn, xp, c * xj);
    }
  }
  Wb[t * WS + S] = cs;
  lam = flip ? -lam_new : lam_new;
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
  for (int c = 0; c < S; ++c) qs[c] = out[c] * Wb[c * WS + S];
  wave_lds_sync();
}

template <int KP, int S>
__device__ __forceinline__ void dc_levels(double (&qs)[KP], double& lam, DcLds<KP>& L,
                                          double ej, double* W, int jj, double deps,
                                          bool& ok) {
  if constexpr (S <= KP) {
    dc_merge<KP, S>(qs, lam, L, ej, W, jj, deps, ok);
    dc_levels<KP, 2 * S>(qs, lam, L, ej, W, jj, deps, ok);
  }
}

// ---- 4 x 4 leaves of the divide and conquer, one per quad of lanes ----
// Lane t of a quad holds row t of the leaf A and row t of the accumulated
// rotations V (A_0 = V diag(lam) V^T at the end).  Cyclic Jacobi (Golub &
// Van Loan, Sec. 8.5) in the parallel order {(0,1),(2,3)}, {(0,2),(1,3)},
// {(0,3),(1,2)}: the two rotations of a round act on disjoint index pairs,
// so each lane applies both to its row's columns, then the rotation of its
// own pair to the rows (with its partner's row).  Quad exchanges are DPP
// quad permutations: 0xB1 lane ^ 1, 0x4E lane ^ 2, 0x1B lane ^ 3.

__device__ __forceinline__ double sel4(const double (&x)[4], int t) {
  return t == 0 ? x[0] : t == 1 ? x[1] : t == 2 ? x[2] : x[3];
}

// The symmetric Schur rotation of the 2 x 2 block (app, apq; apq, aqq):
// c, s with J = [[c, s], [-s, c]] and J^T A J diagonal (as the 2 x 2 leaves).
__device__ __forceinline__ void schur2(double app, double aqq, double apq, double& c, double& s) {
  c = 1.0;
  s = 0.0;
  const double a2 = 2.0 * apq, diff = aqq - app;
  if (fabs(a2) > 1e-250 && fabs(a2) < 1e250 && fabs(diff) < 1e100 * fabs(a2)) {
    // the usual case, from refined reciprocals and reciprocal square roots
    // (|th| < 1e100, so th^2 + 1 and |th| + sqrt(th^2 + 1) stay in range)
    const double th = diff * frcp(a2);
    double r1, q1;
    rsqrt_sqrt(fma(th, th, 1.0), r1, q1);
    const double t = (th >= 0.0 ? 1.0 : -1.0) * frcp(fabs(th) + q1);
    double q2;
    rsqrt_sqrt(fma(t, t, 1.0), c, q2);
    s = t * c;
  } else if (apq != 0.0) {
    const double th = diff / a2;
    const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(fma(th, th, 1.0)));
    c = 1.0 / sqrt(fma(t, t, 1.0));
    s = t * c;
  }
}

// Columns p, q of a row rotated: (x_p, x_q) <- (c x_p - s x_q, s x_p + c x_q).
template <int P, int Q>
__device__ __forceinline__ void rot_cols(double (&x)[4], double c, double s) {
  const double xp = x[P], xq = x[Q];
  x[P] = fma(c, xp, -s * xq);
  x[Q] = fma(s, xp, c * xq);
}

// One round: pairs (P0, Q0) and (P1, Q1); PART is the DPP pattern of the
// partner in one's own pair, OTHER that of a lane of the other pair.
template <int P0, int Q0, int P1, int Q1, int PART, int OTHER>
__device__ __forceinline__ void jacobi4_round(double (&A)[4], double (&V)[4], int t) {
  const bool first = t == P0 || t == Q0;
  const int p = first ? P0 : P1, q = first ? Q0 : Q1;
  const bool isp = t == p;
  // the pair's entries: a_pp and a_qq from their lanes, a_pq from row p, so
  // that both lanes of the pair compute the same rotation
  const double d = sel4(A, t);
  const double dp = dpp_lane<PART>(d);
  const double o = sel4(A, q);                 // row p: a_pq (row q: unused)
  const double op = dpp_lane<PART>(o);
  double c, s;
  schur2(isp ? d : dp, isp ? dp : d, isp ? o : op, c, s);
  const double co = dpp_lane<OTHER>(c), so = dpp_lane<OTHER>(s);
  const double c0 = first ? c : co, s0 = first ? s : so;
  const double c1 = first ? co : c, s1 = first ? so : s;
  // A <- A J, V <- V J
  rot_cols<P0, Q0>(A, c0, s0);
  rot_cols<P1, Q1>(A, c1, s1);
  rot_cols<P0, Q0>(V, c0, s0);
  rot_cols<P1, Q1>(V, c1, s1);
  // A <- J^T A: row p <- c row_p - s row_q, row q <- s row_p + c row_q
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const double other = dpp_lane<PART>(A[j]);
    A[j] = isp ? fma(c, A[j], -s * other) : fma(s, other, c * A[j]);
  }
}

// Sum over the quad.
__device__ __forceinline__ double quad_sum(double x) {
  x += dpp_lane<0xB1>(x);
  return x + dpp_lane<0x4E>(x);
}

// x[t ^ M] of lane t ^ M, for each lane t (the quad's values of register t
// transposed through lane pairs t, t ^ M).
template <int M>
__device__ __forceinline__ double quad_xchg(const double (&x)[4], int t) {
  constexpr int CTRL = M == 1 ? 0xB1 : M == 2 ? 0x4E : 0x1B;
  return dpp_lane<CTRL>(sel4(x, t ^ M));
}

// The leaf's eigendecomposition: lam = this lane's eigenvalue, Vc = column t
// of V (V[0..3][t]: the eigenvector of lam), Vr = row t of V.  Sweeps until
// every leaf of the wavefront is diagonal to 1e-15 of its norm (at most 8;
// a 4 x 4 symmetric matrix takes 3 or 4 in FP64).
__device__ __forceinline__ void jacobi4(double (&A)[4], double& lam, double (&Vc)[4],
                                        double (&Vr)[4], int t) {
#pragma unroll
  for (int j = 0; j < 4; ++j) Vr[j] = j == t ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 8; ++sweep) {
    double off = 0.0, fro = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double a2 = A[j] * A[j];
      fro += a2;
      off += j == t ? 0.0 : a2;
    }
    off = quad_sum(off);
    fro = quad_sum(fro);
    if (__ballot(off > 1e-30 * fro) == 0) break;         // wave-uniform
    jacobi4_round<0, 1, 2, 3, 0xB1, 0x4E>(A, Vr, t);
    jacobi4_round<0, 2, 1, 3, 0x4E, 0xB1>(A, Vr, t);
    jacobi4_round<0, 3, 1, 2, 0x1B, 0xB1>(A, Vr, t);
  }
  lam = sel4(A, t);
  // column t of V: V[s][t] is lane s's entry t
#pragma unroll
  for (int j = 0; j < 4; ++j) Vc[j] = 0.0;
  const double own = sel4(Vr, t);
  const double x1 = quad_xchg<1>(Vr, t), x2 = quad_xchg<2>(Vr, t), x3 = quad_xchg<3>(Vr, t);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int m = s ^ t;
    Vc[s] = m == 0 ? own : m == 1 ? x1 : m == 2 ? x2 : x3;
  }
}

// Row t = jj % 4 of the 4 x 4 leaf of T at lane jj (d_jj = dj, e_jj = ej =
// T[jj+1][jj]): T torn at every fourth coupling (Cuppen: a torn coupling
// comes off both diagonal entries it joins; e_{KP-1} = 0).
template <int KP>
__device__ __forceinline__ void leaf4(double dj, double ej, int jj, double (&A)[4]) {
  const int t = jj & 3, a4 = jj & ~3;
  const double eabove = __shfl(ej, a4 > 0 ? a4 - 1 : 0, KP);
  const double eleft = dpp_lane<0x90>(ej);       // quad_perm [0,0,1,2]: lane t - 1's coupling
  double dd = dj;
  if (t == 0 && a4 > 0) dd -= eabove;
  if (t == 3) dd -= ej;
#pragma unroll
  for (int j = 0; j < 4; ++j) A[j] = j == t ? dd : (j == t + 1 ? ej : (j == t - 1 ? eleft : 0.0));
}

// Eigen-decomposition of the tridiagonal (d, e), lane jj of the KP-lane group
// holding dj = d_jj and ej = e_jj = T[jj+1][jj] (e_{KP-1} = 0).  Deflation tolerance 8 deps max(|D|, rho) per merge, with
// deps the unit roundoff of the arithmetic that produced the matrix.  On
// return lam is the eigenvalue of column jj and qs[] is row jj of the
// eigenvector matrix.  Returns false if a secular root ran out of iterations.
template <int KP>
__device__ __forceinline__ bool dc_tridiagonal(double (&qs)[KP], double& lam, DcLds<KP>& L,
                                               double dj, double ej, double* W, int jj,
                                               double deps) {
  // 4 x 4 leaves (leaf4), each diagonalized by Jacobi on its quad of lanes;
  // row t of the leaf's eigenvector matrix is the row restricted to the
  // leaf's columns
  const int t = jj & 3;
  double A[4], Vc[4], Vr[4];
  leaf4<KP>(dj, ej, jj, A);
  jacobi4(A, lam, Vc, Vr, t);
#pragma unroll
  for (int q = 0; q < KP; ++q) qs[q] = q < 4 ? Vr[q] : 0.0;
  bool ok = true;
  dc_levels<KP, 8>(qs, lam, L, ej, W, jj, deps, ok);
  return ok;
}

}  // namespace letkf
