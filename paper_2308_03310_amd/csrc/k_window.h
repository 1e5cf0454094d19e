// The local observations of a grid point (R-localization, Sec. II-B), as the
// Gram kernels find them: a walk over the observation cells that intersect
// the point's window, 64 candidates per batch, each with its localization
// weight w_j = g(r_xj) / sigma_j^2, and the accepted ones appended to a small
// per-wavefront ring in LDS.  The walk is a cursor so that a kernel can issue
// the loads of the next batch before it works on the current one.
#pragma once
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

// Position in the walk.  The window's cell ranges (one per cell row and
// x-interval: observations [s, s1) of cells xlo..xhi of row cy, sorted by
// cell) are numbered r = 0, 1, ..; their bounds are read 64 at a time, range
// base + l by lane l in one round of loads, and taken from the lanes as the
// walk reaches them, so the walk waits on memory once per 64 ranges rather
// than once per range.  Every field but vs, vs1 is the same on all lanes (the
// point is the wavefront's).
struct WindowCursor {
  int nxi, n0, nranges;                   // x-intervals, rows of y-interval 0, ranges
  int ylo0, ylo1, xlo0, xhi0, xlo1, xhi1;
  int r, base;                            // current range; first range of the loaded chunk
  int vs, vs1;                            // this lane's range of the chunk (range base + lane)
  int s, s1;                              // current batch start and range end
};

// Bounds of ranges base .. base + 63, range base + l to lane l.
__device__ __forceinline__ void window_load_chunk(WindowCursor& c, const GramArgs& g) {
  const int r = c.base + lane_id();
  c.vs = c.vs1 = 0;
  if (r < c.nranges) {
    const int rr = r / c.nxi, xi = r - rr * c.nxi;
    const int cy = rr < c.n0 ? c.ylo0 + rr : c.ylo1 + (rr - c.n0);
    const int row = cy * g.ncx;
    c.vs = ldg(g.cell_start, row + (xi == 0 ? c.xlo0 : c.xlo1));
    c.vs1 = ldg(g.cell_start, row + (xi == 0 ? c.xhi0 : c.xhi1) + 1);
  }
}

// Moves to the next non-empty range; false when the window is exhausted.
__device__ __forceinline__ bool window_next_range(WindowCursor& c, const GramArgs& g) {
  for (;;) {
    if (++c.r >= c.nranges) return false;
    if (c.r - c.base >= 64) {
      c.base += 64;
      window_load_chunk(c, g);
    }
    c.s = __builtin_amdgcn_readlane(c.vs, c.r - c.base);
    c.s1 = __builtin_amdgcn_readlane(c.vs1, c.r - c.base);
    if (c.s < c.s1) return true;
  }
}

// Starts the walk for point (x, y) (uniform over the wavefront).
__device__ __forceinline__ bool window_begin(WindowCursor& c, const GramArgs& g, int x, int y) {
  int lo[2] = {0, 0}, hi[2] = {0, 0};
  c.nxi = cell_intervals(x, g.R, g.nx, g.cb, g.ncx, lo, hi);
  c.xlo0 = lo[0];
  c.xhi0 = hi[0];
  c.xlo1 = lo[1];
  c.xhi1 = hi[1];
  lo[1] = hi[1] = 0;
  const int nyi = cell_intervals(y, g.R, g.ny, g.cb, g.ncy, lo, hi);
  c.ylo0 = lo[0];
  c.ylo1 = lo[1];
  c.n0 = hi[0] - lo[0] + 1;
  c.nranges = (c.n0 + (nyi > 1 ? hi[1] - lo[1] + 1 : 0)) * c.nxi;
  c.r = -1;
  c.base = 0;
  window_load_chunk(c, g);
  return window_next_range(c, g);
}

__device__ __forceinline__ bool window_next_batch(WindowCursor& c, const GramArgs& g) {
  c.s += 64;
  if (c.s < c.s1) return true;
  return window_next_range(c, g);
}

// This lane's candidate of the batch starting at s0 (range end s1 > s0): the
// raw loads, issued ahead of their use and without a branch (lanes past the
// range read its last observation; candidate_weight ignores them).
struct Candidate {
  int ox, oy;
  double rinv;
};

__device__ __forceinline__ Candidate load_candidate(const GramArgs& g, int s0, int s1) {
  const int s = min(s0 + lane_id(), s1 - 1);
  Candidate c;
  c.ox = ldg(g.ox, s);
  c.oy = ldg(g.oy, s);
  c.rinv = ldg(g.rinv, s);
  return c;
}

// Localization weight of the candidate for point (x, y) (periodic minimum
// image distance); 0 past the cutoff or for an observation with no weight.
__device__ __forceinline__ double candidate_weight(const Candidate& c, const GramArgs& g, int x,
                                                   int y, bool present) {
  int dx = abs(x - c.ox);
  dx = min(dx, g.nx - dx);
  int dy = abs(y - c.oy);
  dy = min(dy, g.ny - dy);
  const double r2d = (double)(dx * dx + dy * dy);
  double w = 0.0;
  if (present && c.rinv > 0.0 && r2d <= g.cut2) {
    double gl;
    if (g.loc == 0) {
      gl = exp(-r2d * g.inv2L2);
    } else if (g.loc == 1) {
      gl = gaspari_cohn(sqrt(r2d), g.invL);
    } else {
      gl = 1.0;
    }
    w = gl * c.rinv;
  }
  return w;
}

constexpr int kRing = 128;   // ring entries per wavefront (a batch adds at most 64)

// Appends the lanes whose w > 0 (observation s) to the ring; returns the new tail.
__device__ __forceinline__ int ring_append(int* ring_s, double* ring_w, int tail, int s, double w) {
  const int lane = lane_id();
  const bool in = w > 0.0;
  const uint64_t mask = __ballot(in);
  const int pos = __popcll(mask & ((1ull << lane) - 1ull));
  if (in) {
    ring_s[(tail + pos) & (kRing - 1)] = s;
    ring_w[(tail + pos) & (kRing - 1)] = w;
  }
  return tail + __popcll(mask);
}

}  // namespace letkf
