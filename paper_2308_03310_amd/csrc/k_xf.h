// LETKF ensemble transform and update without forming the eigenvectors, FP64,
// for gfx950.
//
// Per grid point (Sec. II-B), with Q = ((k-1)/rho) I + C = V diag(lam) V^T:
//     X^a = xbar 1^T + dX (wbar 1^T + W),   wbar = V lam^-1 V^T b,
//     W   = sqrt(k-1) V lam^-1/2 V^T                  eqs. (letkf_wa), (letkf_dwa), (letkf_xa)
// Only ten vectors ever meet V: the nine rows of dX and b.  With the
// Householder reduction Q = H T H^T and the divide and conquer T = Q_T diag(lam)
// Q_T^T, V = H Q_T, and
//     G = dX V,  g = b^T V       (rows of X H carried forward through the merges)
//     X^a - xbar 1^T = (G lam^-1 g^T) 1^T + (G sqrt(k-1) lam^-1/2) Q_T^T H^T
//                                             (carried back through the merges)
// so V is never built: the O(k^3) eigenvector accumulation of the merges and
// the back-transformation become O(k^2) work per level on ten vectors.
//
// Layouts of one matrix on its KP lanes (KP/64 of a wavefront):
//   * Householder reduction: lane j holds row j of Q (k_evd.h);
//   * Householder vectors applied to rows of X: 16 rows x NP = KP/16 parts,
//     lane 16 q + c holds entries q, q + NP, .., q + 15 NP of row c (an entry
//     j is zero in every reflector below j, so reflector i touches only the
//     entries from (i+1)/NP on);
//   * divide and conquer: lane t holds column t of the vectors (its entry of
//     each row) and the eigenvalue of column t.
// Each merge of the divide and conquer (k_dc.h) gives the merged block's
// eigenvectors in terms of its children's as M = G_0 .. G_{r-1} C, deflation
// rotations G_q and C with columns zhat_u / (d_u - lam_t) (normalized) or unit
// columns for deflated poles; the vectors are multiplied by M on the way up
// and by M^T on the way down, from what each lane keeps of its merges.  The
// merge vector z of a block is made of its children's last and first rows of
// Q_T, so two more vectors (the first and last rows of every block) ride
// along on the way up.
#pragma once
#include "common.h"
#include "launch.h"
#include "k_dc.h"
#include "k_evd.h"

namespace letkf {

constexpr int kXfRows = 10;   // rows of X: nine components of dX, then b
constexpr int kXfUp = 12;     // vectors on the way up: X rows, first row, last row
constexpr int kXfDown = 9;    // vectors on the way down
constexpr int kXfRec = 14;    // record of a non-deflated pole on the way up: d, zhat, 12 entries
constexpr int kXfRecB = 12;   // record of a non-deflated root on the way down: dorg, tau, 9 entries

// Register budget of the transform kernel: the Householder vectors stay in
// the lanes' registers through the divide and conquer only up to this width
// (beyond it they wait in the point's consumed Gram output), and the
// reduction streams its broadcast vectors from LDS above this width.
#ifndef LETKF_XF_REFL_REG_MAX
#define LETKF_XF_REFL_REG_MAX 32
#endif
#ifndef LETKF_XF_BURST_MAX
#define LETKF_XF_BURST_MAX 32
#endif
template <int KP>
constexpr bool kXfReflInRegisters = KP <= LETKF_XF_REFL_REG_MAX;
template <int KP>
constexpr bool kXfStream = KP > LETKF_XF_BURST_MAX;

template <int KP>
struct XfLds {
  static constexpr int G = 64 / KP;
  double taus[G][KP];                      // reflector tau values (KP - 2 used)
  union {
    struct {                               // Householder reduction: broadcast vectors
      double vb[G][KP];
      double wb[G][KP];
    };
    struct {                               // Householder vectors on the rows of X
      double refl[G][16][KP];              // 16 reflectors, entries in part-major order
      double tr[G][KP][kXfRows + 1];       // row layout <-> column layout
    };
    struct {                               // divide and conquer
      DcLds<KP> dc[G];
      double vr[G][KP][kXfUp];             // vectors by block-local row (rotations, deflated columns)
      alignas(16) double rec[G][KP][kXfRec];
      int pinv[G][KP];                     // block-local row -> sorted position
    };
  };
};

// Sum over the NP parts of a row (lanes c, c + 16, c + 32, c + 48 of a group).
template <int NP>
__device__ __forceinline__ double part_sum(double x) {
  if constexpr (NP >= 2) {
    double a, b;
    row_pair<16>(x, a, b);
    x = a + b;
  }
  if constexpr (NP >= 4) {
    double a, b;
    row_pair<32>(x, a, b);
    x = a + b;
  }
  return x;
}

// Position of entry j of a reflector in the part-major layout.
template <int KP>
__device__ __forceinline__ int part_pos(int j) {
  constexpr int NP = KP / 16;
  return (j % NP) * 16 + j / NP;
}

// Row jj of Q = alpha I + C from the Gram output (upper 16 x 16 blocks of C;
// an entry below the diagonal block is read from its mirror), padded rows
// unit, and this lane's entry of b.
template <int KP>
__device__ __forceinline__ void xf_load_row(const EvdArgs& e, const double* Cp, int jj, bool valid,
                                            double (&a)[KP]) {
  constexpr int NQ = KP / 16;
  const bool real = valid && jj < e.k;
  const int I = jj >> 4, r = jj & 15;
#pragma unroll
  for (int J = 0; J < NQ; ++J) {
    // block (min(I,J), max(I,J)) in row-major upper order; only the upper
    // triangle of C is read (its diagonal blocks' two triangles differ by
    // rounding), so the row is that of an exactly symmetric matrix, as the
    // packed form gives it
    const int lo = I < J ? I : J, hi = I < J ? J : I;
    const int blk = lo * NQ - lo * (lo - 1) / 2 + (hi - lo);
    const double* B = Cp + blk * 256;
    if (J > I) {
#pragma unroll
      for (int c = 0; c < 16; ++c) a[16 * J + c] = ldg(B, r * 16 + c);
    } else if (J < I) {
#pragma unroll
      for (int c = 0; c < 16; ++c) a[16 * J + c] = ldg(B, c * 16 + r);
    } else {
#pragma unroll
      for (int c = 0; c < 16; ++c) a[16 * J + c] = ldg(B, c >= r ? r * 16 + c : c * 16 + r);
    }
  }
#pragma unroll
  for (int c = 0; c < KP; ++c) {
    const double v = real ? a[c] : 0.0;
    a[c] = c == jj ? (real ? v + e.alpha : 1.0) : v;
  }
}

// Row jj of Q from C held as its packed upper triangle in LDS (the fused
// kernel), as xf_load_row.
template <int KP>
__device__ __forceinline__ void xf_load_row_packed(const EvdArgs& e, const double* Cq, int jj,
                                                   bool valid, double (&a)[KP]) {
  const bool real = valid && jj < e.k;
  const auto* lds = (const __attribute__((address_space(3))) double*)Cq;
#pragma unroll
  for (int c = 0; c < KP; ++c) {
    const double v = c >= jj ? lds[packed_upper(jj, c, KP)] : lds[packed_upper(c, jj, KP)];
    a[c] = c == jj ? (real ? v + e.alpha : 1.0) : (real ? v : 0.0);
  }
}

// Reflectors [I0, I0 + 16) of this matrix into the LDS chunk, entries in
// part-major order, from the lanes' registers (a[i] = entry jj of reflector
// i for i < jj) or from the global copy (rv, packed; entries below the unit
// entry of each reflector are zero).
template <int KP, int I0>
__device__ __forceinline__ void xf_stage_refl_regs(const double (&a)[KP], double* chunk, int jj) {
  const int pos = part_pos<KP>(jj);
#pragma unroll
  for (int i = I0; i < I0 + 16; ++i) {
    if (i < KP - 2) chunk[(i - I0) * KP + pos] = jj > i ? a[i] : 0.0;
  }
}

template <int KP, int I0>
__device__ __forceinline__ void xf_load_refl_global(double (&v)[16], const double* rv, int k, int jj,
                                                    bool valid) {
#pragma unroll
  for (int i = I0; i < I0 + 16; ++i) {
    v[i - I0] = 0.0;
    if (i < KP - 2 && valid && jj > i && jj < k) v[i - I0] = ldg(rv, refl_pos(i, jj, k));
  }
}

template <int KP, int I0>
__device__ __forceinline__ void xf_store_refl_chunk(const double (&v)[16], double* chunk, int jj) {
  const int pos = part_pos<KP>(jj);
#pragma unroll
  for (int i = I0; i < I0 + 16; ++i) {
    if (i < KP - 2) chunk[(i - I0) * KP + pos] = v[i - I0];
  }
}

// Entries u0.. of reflector i (this lane's part) from the LDS chunk.
template <int KP, int i, int I0>
__device__ __forceinline__ void xf_load_refl(double (&v)[16], const double* chunk, int q) {
  constexpr int NP = KP / 16;
  constexpr int u0 = ((i + 1) / NP) & ~1;     // first pair holding an entry >= i + 1
  const double* vrow = chunk + (i - I0) * KP + q * 16;
#pragma unroll
  for (int u = u0; u < 16; u += 2) {
    const double2 t2 = *reinterpret_cast<const double2*>(vrow + u);
    v[u] = t2.x;
    v[u + 1] = t2.y;
  }
}

// x <- x (I - tau v v^T) for reflector i (row-part layout: this lane's part q
// holds entries q + NP u of the row, u = 0..15; entries below (i+1)/NP are
// zero in v and skipped).
template <int KP, int i>
__device__ __forceinline__ void xf_apply_refl(double (&x)[16], const double (&v)[16], double tau) {
  constexpr int NP = KP / 16;
  constexpr int u0 = ((i + 1) / NP) & ~1;
  double s0 = 0.0, s1 = 0.0;
#pragma unroll
  for (int u = u0; u < 16; u += 2) {
    s0 = fma(x[u], v[u], s0);
    s1 = fma(x[u + 1], v[u + 1], s1);
  }
  const double f = tau * part_sum<NP>(s0 + s1);
#pragma unroll
  for (int u = u0; u < 16; ++u) x[u] = fma(-f, v[u], x[u]);
}

// Reflectors of the chunk [I0, I0 + 16) in ascending (UP) or descending
// order, those below KP - 2, software-pipelined: the next reflector's entries
// are requested before the current one is applied; a compiler memory
// barrier keeps the loads of later reflectors from being hoisted further and
// scheduling barriers keep the products of a reflector from sinking below the
// next one's loads (either way every reflector would be held in registers).
template <int KP, int I0, bool UP, int J>
__device__ __forceinline__ void xf_chunk_step(double (&x)[16], double (&cur)[16],
                                              const double* chunk, const double* taus, int q) {
  constexpr int i = UP ? I0 + J : I0 + 15 - J;
  constexpr int inext = UP ? i + 1 : i - 1;
  constexpr bool has_next = J + 1 < 16 && inext >= I0 && inext < KP - 2;
  if constexpr (J < 16) {
    if constexpr (i < KP - 2) {
      double nxt[16];
      if constexpr (has_next) xf_load_refl<KP, (has_next ? inext : I0), I0>(nxt, chunk, q);
      const double tau = taus[i];
      asm volatile("" ::: "memory");
      xf_apply_refl<KP, i>(x, cur, tau);
      pin_regs<16>(x);   // the products of this reflector happen here
      if constexpr (has_next) {
#pragma unroll
        for (int u = 0; u < 16; ++u) cur[u] = nxt[u];
      }
      xf_chunk_step<KP, I0, UP, J + 1>(x, cur, chunk, taus, q);
    } else {
      // (descending order: reflectors past KP - 3 are skipped; load the first real one)
      if constexpr (!UP && has_next) xf_load_refl<KP, inext, I0>(cur, chunk, q);
      xf_chunk_step<KP, I0, UP, J + 1>(x, cur, chunk, taus, q);
    }
  }
}

template <int KP, int I0, bool UP>
__device__ __forceinline__ void xf_apply_chunk(double (&x)[16], const double* chunk,
                                               const double* taus, int q) {
  constexpr int first = UP ? I0 : (I0 + 15 < KP - 3 ? I0 + 15 : KP - 3);
  double cur[16];
  xf_load_refl<KP, first, I0>(cur, chunk, q);
  if constexpr (UP) {
    xf_chunk_step<KP, I0, true, 0>(x, cur, chunk, taus, q);
  } else {
    xf_chunk_step<KP, I0, false, I0 + 15 - first>(x, cur, chunk, taus, q);
  }
}

// X H = X H_0 H_1 .. H_{n-3}: reflectors in ascending order, staged 16 at a
// time from the lanes' registers.
template <int KP, int I0>
__device__ __forceinline__ void xf_reflect_forward(double (&x)[16], const double (&a)[KP],
                                                   XfLds<KP>& sh, int seg, int jj, int q) {
  if constexpr (I0 < KP - 2) {
    double* chunk = &sh.refl[seg][0][0];
    xf_stage_refl_regs<KP, I0>(a, chunk, jj);
    wave_lds_sync();
    xf_apply_chunk<KP, I0, true>(x, chunk, sh.taus[seg], q);
    wave_lds_sync();
    xf_reflect_forward<KP, I0 + 16>(x, a, sh, seg, jj, q);
  }
}

// Z H^T = Z H_{n-3} .. H_0: reflectors in descending order, 16 at a time,
// from the lanes' registers (KP <= LETKF_XF_REFL_REG_MAX) or from the global
// copy, the next chunk's loads in flight while a chunk is applied.
template <int KP, int I0>
__device__ __forceinline__ void xf_reflect_backward_regs(double (&x)[16], const double (&a)[KP],
                                                         XfLds<KP>& sh, int seg, int jj, int q) {
  if constexpr (I0 >= 0) {
    double* chunk = &sh.refl[seg][0][0];
    xf_stage_refl_regs<KP, I0>(a, chunk, jj);
    wave_lds_sync();
    xf_apply_chunk<KP, I0, false>(x, chunk, sh.taus[seg], q);
    wave_lds_sync();
    xf_reflect_backward_regs<KP, I0 - 16>(x, a, sh, seg, jj, q);
  }
}

template <int KP, int I0>
__device__ __forceinline__ void xf_reflect_backward_global(double (&x)[16], double (&nxt)[16],
                                                           const double* rv, int k, bool valid,
                                                           XfLds<KP>& sh, int seg, int jj, int q) {
  if constexpr (I0 >= 0) {
    double* chunk = &sh.refl[seg][0][0];
    xf_store_refl_chunk<KP, I0>(nxt, chunk, jj);
    if constexpr (I0 >= 16) xf_load_refl_global<KP, I0 - 16>(nxt, rv, k, jj, valid);
    wave_lds_sync();
    xf_apply_chunk<KP, I0, false>(x, chunk, sh.taus[seg], q);
    wave_lds_sync();
    xf_reflect_backward_global<KP, I0 - 16>(x, nxt, rv, k, valid, sh, seg, jj, q);
  }
}

// What a lane keeps of one merge for the way down.
struct XfHist {
  double dorg, tau, cs;   // as column t: its root (origin pole, offset) and column scale
  double drow, zrow;      // as row r: pole and weight of its non-deflated index
  double rc, rs;          // the block's rotation number t (if t < nrot)
  int col;                // as column: inv[t] + 1 (0: deflated); as row: source
                          // sorted position << 8 | (non-deflated ? 1 : 0) << 16
  int rot;                // rotation rows rp | rj << 8; nrot << 16; trivial << 24
};

// One merge level S on the way up, for every block of the matrix at once.
// R: this lane's column of the twelve vectors (children's eigenvector basis
// in, merged block's out); lam: the eigenvalue of this column.
template <int KP, int S>
__device__ __forceinline__ void xf_merge_up(double (&R)[kXfUp], double& lam, double ej,
                                            XfLds<KP>& sh, int seg, int jj, double deps, bool& ok,
                                            XfHist& h) {
  constexpr int H = S / 2;
  DcLds<KP>& L = sh.dc[seg];
  const int t = jj & (S - 1);
  const int a = jj - t;
  const double z = t < H ? R[11] : R[10];   // left child's last row | right child's first row
  const double beta = __shfl(ej, a + H - 1, KP);
  const MergeRoots mr = merge_roots<KP, S>(z, lam, beta, L, jj, deps, ok);
  // first row of the block: the left child's on its columns; last row: the right child's
  R[10] = t < H ? R[10] : 0.0;
  R[11] = t < H ? 0.0 : R[11];
  h.rot = mr.trivial ? (1 << 24) : 0;
  h.col = 0;
  h.dorg = h.tau = h.drow = h.zrow = h.rc = h.rs = 0.0;
  h.cs = 1.0;
  const bool any_merge = __ballot(!mr.trivial) != 0;
  if (!any_merge) return;                               // wave-uniform
  const int ti = mr.trivial ? -1 : L.inv[a + t];
  const int pmt = mr.trivial ? t : L.pm[a + t];
  const int nrot = mr.trivial ? 0 : L.rot[a + S - 1];
  double (*vr)[kXfUp] = sh.vr[seg];
#pragma unroll
  for (int v = 0; v < kXfUp; ++v) vr[jj][v] = R[v];
  sh.pinv[seg][a + pmt] = t;
  int rp = 0, rj = 0;
  if (t < nrot) {
    const int pj = L.rot[a + t];
    rp = L.pm[a + (pj & 255)];
    rj = L.pm[a + (pj >> 8)];
    h.rc = L.rc[a + t];
    h.rs = L.rs[a + t];
  }
  h.rot |= rp | (rj << 8) | (nrot << 16);
  wave_lds_sync();
  // deflation rotations R <- R G_0 .. G_{nrot-1} on the block's rows, one
  // sequence per vector
  if (__ballot(nrot > 0) != 0) {
    for (int v = t; v < kXfUp; v += S) {
      for (int qq = 0; qq < nrot; ++qq) {
        const int pj = L.rot[a + qq];
        const int p0 = a + L.pm[a + (pj & 255)], p1 = a + L.pm[a + (pj >> 8)];
        const double c = L.rc[a + qq], sn = L.rs[a + qq];
        const double xp = vr[p0][v], xj = vr[p1][v];
        vr[p0][v] = fma(c, xp, -sn * xj);
        vr[p1][v] = fma(sn, xp, c * xj);
      }
    }
    wave_lds_sync();
  }
  // records of the non-deflated poles: (d_u, zhat_u, the vectors at its row)
  double (*rec)[kXfRec] = sh.rec[seg];
  if (ti >= 0) {
    rec[a + ti][0] = L.dw[2 * a + ti].x;
    rec[a + ti][1] = L.zh[a + ti];
#pragma unroll
    for (int v = 0; v < kXfUp; ++v) rec[a + ti][2 + v] = vr[a + pmt][v];
  }
  wave_lds_sync();
  // this lane as a row: where its entry goes on the way down
  if (!mr.trivial) {
    const int tr = sh.pinv[seg][jj];
    const int ur = L.inv[a + tr];
    h.col = (tr << 8) | (ur >= 0 ? (1 << 16) : 0);
    if (ur >= 0) {
      h.drow = L.dw[2 * a + ur].x;
      h.zrow = L.zh[a + ur];
    }
  }
  double lam_new = lam;
  if (!mr.trivial) {
    if (ti < 0) {
#pragma unroll
      for (int v = 0; v < kXfUp; ++v) R[v] = vr[a + pmt][v];
      lam_new = L.ds[a + t];
    } else {
      const double tau = L.rt[a + ti];
      const double dorg = L.rd[a + ti];
      double acc[kXfUp];
#pragma unroll
      for (int v = 0; v < kXfUp; ++v) acc[v] = 0.0;
      double nrm = 0.0;
      const int K = mr.K;
#pragma unroll 2
      for (int u = 0; u < K; ++u) {
        const double* rr = rec[a + u];
        const double2 dz = *reinterpret_cast<const double2*>(rr);
        const double w = dz.y * frcp((dz.x - dorg) - tau);
        nrm = fma(w, w, nrm);
#pragma unroll
        for (int v = 0; v < kXfUp; v += 2) {
          const double2 x2 = *reinterpret_cast<const double2*>(rr + 2 + v);
          acc[v] = fma(w, x2.x, acc[v]);
          acc[v + 1] = fma(w, x2.y, acc[v + 1]);
        }
      }
      const double cs = rsqrt_any(nrm);
#pragma unroll
      for (int v = 0; v < kXfUp; ++v) R[v] = acc[v] * cs;
      lam_new = dorg + tau;
      h.dorg = dorg;
      h.tau = tau;
      h.cs = cs;
      h.col |= ti + 1;
    }
    lam = mr.flip ? -lam_new : lam_new;
  }
  wave_lds_sync();
}

// The same merge on the way down: Y (this lane's column of the nine vectors
// in the merged block's eigenvector basis) becomes Y M^T in the children's.
template <int KP, int S>
__device__ __forceinline__ void xf_merge_down(double (&Y)[kXfDown], XfLds<KP>& sh, int seg,
                                              int jj, const XfHist& h) {
  const int t = jj & (S - 1);
  const int a = jj - t;
  const bool trivial = (h.rot >> 24) & 1;
  if (__ballot(!trivial) == 0) return;                  // wave-uniform
  const int nrot = (h.rot >> 16) & 0xFF;
  double (*vr)[kXfUp] = sh.vr[seg];
  double (*rec)[kXfRec] = sh.rec[seg];
  int K = 0;
  if (!trivial) {
#pragma unroll
    for (int v = 0; v < kXfDown; ++v) vr[jj][v] = Y[v];
    const int ti = (h.col & 0xFF) - 1;
    if (ti >= 0) {
      rec[a + ti][0] = h.dorg;
      rec[a + ti][1] = h.tau;
#pragma unroll
      for (int v = 0; v < kXfDown; ++v) rec[a + ti][2 + v] = Y[v] * h.cs;
    }
    K = __popcll(__ballot(ti >= 0) >> (lane_id() & ~(S - 1)) &
                 (S == 64 ? ~0ull : ((1ull << S) - 1ull)));
  }
  wave_lds_sync();
  double Yc[kXfDown];
  if (!trivial) {
    const int src = (h.col >> 8) & 0xFF;
    if ((h.col >> 16) & 1) {
      double acc[kXfDown];
#pragma unroll
      for (int v = 0; v < kXfDown; ++v) acc[v] = 0.0;
#pragma unroll 2
      for (int u = 0; u < K; ++u) {
        const double* rr = rec[a + u];
        const double2 dt = *reinterpret_cast<const double2*>(rr);
        const double w = frcp((h.drow - dt.x) - dt.y);
#pragma unroll
        for (int v = 0; v < 8; v += 2) {
          const double2 x2 = *reinterpret_cast<const double2*>(rr + 2 + v);
          acc[v] = fma(w, x2.x, acc[v]);
          acc[v + 1] = fma(w, x2.y, acc[v + 1]);
        }
        acc[8] = fma(w, rr[10], acc[8]);
      }
#pragma unroll
      for (int v = 0; v < kXfDown; ++v) Yc[v] = acc[v] * h.zrow;
    } else {
#pragma unroll
      for (int v = 0; v < kXfDown; ++v) Yc[v] = vr[a + src][v];
    }
  }
  wave_lds_sync();
  // rotations transposed, last first
  if (__ballot(nrot > 0) != 0) {
    if (!trivial) {
#pragma unroll
      for (int v = 0; v < kXfDown; ++v) vr[jj][v] = Yc[v];
    }
    // the block's rotations to LDS (row pair, c, s), from the lanes that kept them
    DcLds<KP>& L = sh.dc[seg];
    if (t < nrot) {
      L.rot[a + t] = h.rot & 0xFFFF;
      L.rc[a + t] = h.rc;
      L.rs[a + t] = h.rs;
    }
    wave_lds_sync();
    for (int v = t; v < kXfDown; v += S) {
      for (int qq = nrot - 1; qq >= 0; --qq) {
        const int pj = L.rot[a + qq];
        const int p0 = a + (pj & 255), p1 = a + (pj >> 8);
        const double c = L.rc[a + qq], sn = L.rs[a + qq];
        const double xp = vr[p0][v], xj = vr[p1][v];
        vr[p0][v] = fma(c, xp, sn * xj);
        vr[p1][v] = fma(-sn, xp, c * xj);
      }
    }
    wave_lds_sync();
    if (!trivial) {
#pragma unroll
      for (int v = 0; v < kXfDown; ++v) Yc[v] = vr[jj][v];
    }
    wave_lds_sync();
  }
  if (!trivial) {
#pragma unroll
    for (int v = 0; v < kXfDown; ++v) Y[v] = Yc[v];
  }
}

// Levels S, 2S, .., KP up, the transform at the top, and back down.  At the
// top (S > KP) lane t holds g_t = (b^T V)_t and G[:, t] = (dX V)[:, t]: the
// analysis-mean increment dX V lam^-1 V^T b = G (g / lam) is summed into mi,
// and the nine vectors leave as Y = G sqrt(k-1) lam^-1/2.
template <int KP, int S>
__device__ __forceinline__ void xf_levels(double (&R)[kXfUp], double lam, double ej, XfLds<KP>& sh,
                                          int seg, int jj, double deps, double sqrt_km1, bool& ok,
                                          double (&Y)[kXfDown], double (&mi)[kXfDown]) {
  if constexpr (S > KP) {
    const double y = R[9] * rcp_any(lam);
    const double d2 = sqrt_km1 * rsqrt_any(lam);
#pragma unroll
    for (int c = 0; c < kXfDown; ++c) {
      mi[c] = group_sum<KP>(R[c] * y);
      Y[c] = R[c] * d2;
    }
  } else {
    XfHist h;
    xf_merge_up<KP, S>(R, lam, ej, sh, seg, jj, deps, ok, h);
    xf_levels<KP, 2 * S>(R, lam, ej, sh, seg, jj, deps, sqrt_km1, ok, Y, mi);
    xf_merge_down<KP, S>(Y, sh, seg, jj, h);
  }
}

// The transform of one matrix: T given by (dj, ej) on lane jj, R = this
// lane's column of X H on entry; Y = this lane's column of Y Q_T^T and mi the
// nine mean increments on exit.  Returns false if a secular root ran out of
// iterations.
template <int KP>
__device__ __forceinline__ bool xf_tridiagonal(double (&R)[kXfUp], double dj, double ej,
                                               XfLds<KP>& sh, int seg, int jj, double deps,
                                               double sqrt_km1, double (&Y)[kXfDown],
                                               double (&mi)[kXfDown]) {
  // 4 x 4 leaves diagonalized by Jacobi (k_dc.h)
  const int t = jj & 3;
  double A[4];
  leaf4<KP>(dj, ej, jj, A);
  double lam, Vc[4], Vr[4];
  jacobi4(A, lam, Vc, Vr, t);
  // R <- R V: entry t of each vector is sum_s R_s V[s][t]
#pragma unroll
  for (int v = 0; v < kXfRows; ++v) {
    const double r1 = dpp_lane<0xB1>(R[v]), r2 = dpp_lane<0x4E>(R[v]), r3 = dpp_lane<0x1B>(R[v]);
    // lane t ^ m holds entry s = t ^ m of the vector, weighted by V[s][t]
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int m = s ^ t;
      acc = fma(m == 0 ? R[v] : m == 1 ? r1 : m == 2 ? r2 : r3, Vc[s], acc);
    }
    R[v] = acc;
  }
  R[10] = Vc[0];             // first row of the leaf's eigenvectors
  R[11] = Vc[3];             // last row
  bool ok = true;
  xf_levels<KP, 8>(R, lam, ej, sh, seg, jj, deps, sqrt_km1, ok, Y, mi);
  // leaves on the way down: Y <- Y V^T, entry t = sum_s Y_s V[t][s]
#pragma unroll
  for (int v = 0; v < kXfDown; ++v) {
    const double y1 = dpp_lane<0xB1>(Y[v]), y2 = dpp_lane<0x4E>(Y[v]), y3 = dpp_lane<0x1B>(Y[v]);
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int m = s ^ t;
      acc = fma(m == 0 ? Y[v] : m == 1 ? y1 : m == 2 ? y2 : y3, Vr[s], acc);
    }
    Y[v] = acc;
  }
  return ok;
}

// Eigensolve, transform and in-place update of the point-major ensemble for
// 64 / KP points per wavefront (mode 0 of EvdArgs).
// One point's ensemble values: component c of member j is in[c sc + j sj]
// before the update and out[c sc + j sj] after it (point-major: sc = k,
// sj = 1, in = out; member-major [k][9][npts]: sc = npts, sj = 9 npts).
struct XRows {
  const double* in;
  double* out;
  size_t sc, sj;
};

// The eigensolve, transform and update of one point on KP lanes (segment
// seg of the wavefront): e its problem's descriptor, Cq its Gram output (the
// upper 16 x 16 blocks of C in global memory, or with PACKED the packed upper
// triangle in LDS, consumed before the eigensolve uses its LDS), rv global
// scratch for the Householder vectors (k (k - 1) / 2 doubles, used when the
// registers cannot keep them), bp its b, xr its ensemble values.  valid
// false: the segment computes on padding and writes nothing.
template <int KP, bool PACKED = false>
__device__ __forceinline__ void xf_body(const EvdArgs& e, bool valid, const double* Cq, double* rv,
                                        const double* bp, const XRows& xr, XfLds<KP>& sh, int seg,
                                        int jj) {
  constexpr int NP = KP / 16;
  const int k = e.k;

  double a[KP];
  if constexpr (PACKED) {
    xf_load_row_packed<KP>(e, Cq, jj, valid, a);
    wave_lds_sync();                 // C is read before the reduction's LDS use
  } else {
    xf_load_row<KP>(e, Cq, jj, valid, a);
  }
  double dj, ej;
  tridiagonalize<KP, kXfStream<KP>, false>(a, sh, seg, jj, dj, ej, sh.taus[seg]);

  // rows of X: dX (nine components, ensemble mean removed) and b, row-part
  // layout; requested before the reflectors' global copy is written, so that
  // the wait for them does not include those stores
  const int q = jj >> 4, c = jj & 15;
  double x[16];
  {
    // row c < 9: component c of the point's members; row 9: b; one load per
    // entry, clamped to the row (entries past k and rows past 9 are zero)
    const double* src = c < 9 ? xr.in + c * xr.sc : bp;
    const size_t sj = c < 9 ? xr.sj : 1;
    const int jmax = c < 9 ? k - 1 : KP - 1;
    const bool row_ok = valid && c < kXfRows;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int j = q + NP * u;
      const double v = ldg(src, (size_t)(j < jmax ? j : jmax) * sj);
      x[u] = (row_ok && j < k) ? v : 0.0;
    }
  }
  if constexpr (!kXfReflInRegisters<KP>) store_reflectors<KP>(a, rv, k, jj, valid);
  double xbar = 0.0;
  {
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) s += x[u];
    xbar = c < 9 ? part_sum<NP>(s) / (double)k : 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) x[u] = (q + NP * u < k) ? x[u] - xbar : 0.0;
  }
  wave_lds_sync();
  xf_reflect_forward<KP, 0>(x, a, sh, seg, jj, q);
  // to the column layout
#pragma unroll
  for (int u = 0; u < 16; ++u)
    if (c < kXfRows) sh.tr[seg][q + NP * u][c] = x[u];
  wave_lds_sync();
  double R[kXfUp];
#pragma unroll
  for (int v = 0; v < kXfRows; ++v) R[v] = sh.tr[seg][jj][v];
  R[10] = R[11] = 0.0;
  wave_lds_sync();

  double Y[kXfDown], mi[kXfDown];
  const bool conv = xf_tridiagonal<KP>(R, dj, ej, sh, seg, jj, e.defl_eps, e.sqrt_km1, Y, mi);
  const uint64_t segmask = KP == 64 ? ~0ull : (((1ull << KP) - 1ull) << (seg * KP));
  if ((__ballot(!conv) & segmask) != 0 && jj == 0 && valid && e.status)
    atomicOr(e.status, kStatNotconv);
  wave_lds_sync();

  // back to the row layout, then the reflectors in reverse order
#pragma unroll
  for (int v = 0; v < kXfDown; ++v) sh.tr[seg][jj][v] = Y[v];
  wave_lds_sync();
#pragma unroll
  for (int u = 0; u < 16; ++u) x[u] = c < kXfDown ? sh.tr[seg][q + NP * u][c] : 0.0;
  // the increment for component c (mean increment of lane c's row)
  double mic = 0.0;
#pragma unroll
  for (int v = 0; v < kXfDown; ++v) mic = v == c ? mi[v] : mic;
  wave_lds_sync();
  constexpr int ILAST = ((KP - 3) / 16) * 16;
  if constexpr (kXfReflInRegisters<KP>) {
    xf_reflect_backward_regs<KP, ILAST>(x, a, sh, seg, jj, q);
  } else {
    double nxt[16];
    xf_load_refl_global<KP, ILAST>(nxt, rv, k, jj, valid);
    xf_reflect_backward_global<KP, ILAST>(x, nxt, rv, k, valid, sh, seg, jj, q);
  }
  // X^a = xbar + mean increment + (Y Q_T^T H^T), this lane's entries of its
  // row.  The entry indices are recomputed here from a laundered part index
  // (kept from the loads instead, they would be live through the whole
  // eigensolve), and the stores are global ones (a flat store would also hold
  // back the next wait for LDS).
  bool finite = true;
  if (valid && c < 9) {
    const int qs = opaque(q);
    double* const row = xr.out + c * xr.sc;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int j = qs + NP * u;
      if (j < k) {
        const double xa = xbar + (mic + x[u]);
        finite = finite && __builtin_isfinite(xa);
        stg(row, (size_t)j * xr.sj, xa);
      }
    }
  }
  if (!finite) atomicOr(e.status, kStatNonfinite);
}

template <int KP>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_evd_xf(BatchMap bm) {
  constexpr int G = 64 / KP;
  __shared__ XfLds<KP> sh;
  const int lane = lane_id();
  const int seg = lane / KP, jj = lane % KP;
  const int pl = blockIdx.x * G + seg;
  bool valid;
  EvdArgs e;
  if constexpr (G == 1)      // one point per wavefront: its descriptor in scalar registers
    e = evd_args_uniform(bm, pl, valid);
  else
    e = evd_args_of(bm, pl, valid);
  const int pv = valid ? pl : 0;
  // the reflectors' global copy goes to the point's consumed Gram output
  double* cp = gram_c(bm, pv, KP);
  double* xp = e.xt + (size_t)(e.pt0 + pv) * 9 * e.k;
  xf_body<KP>(e, valid, cp, cp, gram_b(bm, pv, KP), XRows{xp, xp, (size_t)e.k, 1}, sh, seg, jj);
}

template <int KP>
hipError_t launch_evd_xf_kp(const BatchMap& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const dim3 grid(ceil_div(a.n, 64 / KP));
  hipLaunchKernelGGL(k_evd_xf<KP>, grid, dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace letkf
