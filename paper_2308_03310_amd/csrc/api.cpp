// C-ABI of the LETKF library (include/letkf.h): plans, argument checks,
// workspace ownership and the stream-ordered launch sequence of analyses.
//
// Per analysis (Sec. II-B, Algorithm 1): observation checks + cell binning,
// member-major -> point-major transpose, forecast observations, then the
// localized Gram and the eigensolve/transform/update over slabs of points,
// then the transpose back.  A call that covers every problem of the plan once
// runs the Gram and eigensolve kernels once per slab over the concatenated
// points of all problems of the same eigensolver width and precision.
#include "../../include/letkf.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "launch.h"

using namespace letkf;

namespace {

constexpr int kCell = 8;                       // default observation-cell edge (lattice points)
constexpr int kCellMin = 4;                    // smallest cell edge letkf_tune tries
constexpr int kMaxDim = 32768;                 // keeps squared distances inside int32
constexpr uint64_t kChunkBytes = 1ull << 30;   // Gram output (C, b) per slab

struct ProblemWs {
  letkf_problem p;
  int npts, kp, nb, ncx, ncy, ncells, nobs_alloc;
  int cell;             // observation-cell edge in use (tunable)
  double* xt;
  int* obs_cell;
  int* perm;
  int* cell_count;
  int* cell_start;
  int* cell_fill;
  int* ox;
  int* oy;
  double* Yb;    // FP64 perturbations (FP64 form)
  void* Ylp;     // FP32 / BF16 perturbations (reduced forms)
  double* d;
  double* rinv;
  double* bgk;   // lattice-BGK ping-pong buffer (plans made with LETKF_FLAG_CYCLE)
  int* abort_flag;
  // device copies of host observation arrays (plans made with LETKF_FLAG_OBS_ON_HOST)
  int32_t* h_ix;
  int32_t* h_iy;
  int32_t* h_kind;
  double* h_val;
  double* h_var;
};

// Problems sharing an eigensolver width and precision: the Gram and
// eigensolve kernels of a batched call run over their concatenated points.
struct ProblemClass {
  int kp = 16, prec = 0, nb = 1, slab = 256;
  std::vector<int> members;   // problem indices, in order
  GramArgs* g = nullptr;      // device [members]
  EvdArgs* e = nullptr;       // device [members]
  int* prefix = nullptr;      // device [members + 1]
  int total = 0;              // points over all members
};

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

constexpr int kKnownFlags = LETKF_FLAG_PHASE_TIMING | LETKF_FLAG_CYCLE | LETKF_FLAG_OBS_ON_HOST |
                            LETKF_FLAG_DETERMINISTIC | LETKF_FLAG_GRAPH_CAPTURE | LETKF_FLAG_NSQRT;

int check_problem(const letkf_problem& p) {
  if (p.nx < 1 || p.ny < 1 || p.nx > kMaxDim || p.ny > kMaxDim) return LETKF_EINVAL;
  if ((int64_t)p.nx * p.ny > ((int64_t)1 << 30)) return LETKF_EINVAL;
  if (p.k < 2 || p.k > LETKF_MAX_K) return LETKF_EINVAL;
  if (p.n_obs_max < 0) return LETKF_EINVAL;
  if (!finite_pos(p.loc_len) || !finite_pos(p.infl)) return LETKF_EINVAL;
  if (p.loc != LETKF_LOC_GAUSS && p.loc != LETKF_LOC_GC && p.loc != LETKF_LOC_NONE)
    return LETKF_EINVAL;
  if (p.precision != LETKF_PREC_FP64 && p.precision != LETKF_PREC_FP32 &&
      p.precision != LETKF_PREC_BF16)
    return LETKF_EINVAL;
  return LETKF_OK;
}

int check_device(int* dev_out) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return LETKF_EDEVICE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return LETKF_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return LETKF_EDEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return LETKF_EDEVICE;
  *dev_out = dev;
  return LETKF_OK;
}

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Points per Gram/eigensolve launch so that the slab's C and b stay within
// kChunkBytes (at least 256 points, at most `total`).
int slab_points(int nb, int kp, int total) {
  const uint64_t per_pt = ((uint64_t)nb * 256 + kp) * sizeof(double);
  uint64_t ch = kChunkBytes / per_pt;
  if (ch < 256) ch = 256;
  return (int)(ch < (uint64_t)total ? ch : (uint64_t)total);
}

}  // namespace

struct letkf_plan_s {
  int device = 0;
  int flags = 0;
  std::string cache_path;           // tuning cache (empty: none)
  hipStream_t aux = nullptr;        // the plan's own stream: status reads
  int* host_stat = nullptr;         // pinned host word the status is read into
  std::vector<ProblemWs> probs;
  std::vector<ProblemClass> classes;
  GramArgs* g_one = nullptr;        // device [nprob]: descriptor of each problem
  EvdArgs* e_one = nullptr;         // device [nprob]
  int* prefix_one = nullptr;        // device [2 * nprob]: {0, npts} per problem
  double* slab_C = nullptr;         // Gram output of one slab (shared by all slabs)
  double* slab_b = nullptr;
  int* stat = nullptr;              // device: [1] sticky status bits, [2 + p] abort flag of problem p
  std::vector<void*> allocs;
  uint64_t bytes = 0;
  std::atomic<int> busy{0};
  hipStream_t last_stream = nullptr;
  int form = LETKF_FORM_AUTO;       // kernel form of the Gram -> update steps (tunable)
  int* queue = nullptr;             // device [kQueueSlots]: persistent-launch work counters
  const double** xio = nullptr;     // device [2 nprob]: {xb, xa} of the current call, read by
                                    // the fused form (which works on them in place of xt)
  // Phase timing: a ring of event sets, one set per timed call.
  static constexpr int kSlots = 256;
  bool timing = false;
  int nev = 0;                      // events per slot
  std::vector<hipEvent_t> ev;       // kSlots * nev
  std::vector<int> slot_slabs;      // slabs launched in the slot's call
  int max_pairs = 0;                // launch pairs (Gram, eigensolve) per call, at most
  std::vector<char> pair_fused;     // kSlots * max_pairs: the pair was one fused launch
  int next_slot = 0, recorded = 0;

  template <class T>
  bool alloc(T** p, size_t count) {
    void* q = nullptr;
    const size_t nbytes = count * sizeof(T) > 0 ? count * sizeof(T) : 256;
    if (hipMalloc(&q, nbytes) != hipSuccess) return false;
    allocs.push_back(q);
    bytes += nbytes;
    *p = static_cast<T*>(q);
    return true;
  }
  void release() {
    for (void* q : allocs) (void)hipFree(q);
    allocs.clear();
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
    if (aux) (void)hipStreamDestroy(aux);
    aux = nullptr;
    if (host_stat) (void)hipHostFree(host_stat);
    host_stat = nullptr;
  }
};

namespace {

void set_cell(ProblemWs& w, int cell) {
  w.cell = cell;
  w.ncx = ceil_div(w.p.nx, cell);
  w.ncy = ceil_div(w.p.ny, cell);
  w.ncells = w.ncx * w.ncy;
}

// Cell arrays are sized for the smallest cell edge the tuner may choose.
int max_cells(const ProblemWs& w) { return ceil_div(w.p.nx, kCellMin) * ceil_div(w.p.ny, kCellMin); }

void plan_sizes(ProblemWs& w) {
  const letkf_problem& p = w.p;
  w.npts = p.nx * p.ny;
  w.kp = pow2_at_least16(p.k);
  w.nb = n_upper_blocks(w.kp);
  set_cell(w, kCell);
  w.nobs_alloc = p.n_obs_max > 0 ? p.n_obs_max : 1;
}

uint64_t ws_bytes(const ProblemWs& w, bool cycle, bool host_obs) {
  const uint64_t no = (uint64_t)w.nobs_alloc;
  const uint64_t ystride =
      w.p.precision == LETKF_PREC_FP64 ? 8 : (w.p.precision == LETKF_PREC_FP32 ? 4 : 2);
  const uint64_t state = (uint64_t)w.npts * 9 * w.p.k * sizeof(double);
  uint64_t b = state * (cycle ? 2 : 1);
  b += no * 5 * sizeof(int) + no * w.kp * ystride + no * 2 * sizeof(double);
  b += (uint64_t)(3 * max_cells(w) + 1) * sizeof(int);
  if (host_obs) b += no * (3 * sizeof(int32_t) + 2 * sizeof(double));
  return b;
}

GramArgs gram_desc(const ProblemWs& w) {
  const letkf_problem& p = w.p;
  GramArgs ga{};
  ga.nx = p.nx;
  ga.ny = p.ny;
  ga.k = p.k;
  ga.cb = w.cell;
  ga.ncx = w.ncx;
  ga.ncy = w.ncy;
  ga.loc = p.loc;
  const double L = p.loc_len;
  if (p.loc == LETKF_LOC_NONE) {
    ga.R = -1;
    ga.cut2 = std::numeric_limits<double>::infinity();
  } else {
    const double r = std::floor(2.0 * L);
    ga.R = r >= (double)(p.nx > p.ny ? p.nx : p.ny) ? -1 : (int)r;
    ga.cut2 = 4.0 * L * L;
  }
  ga.inv2L2 = 1.0 / (2.0 * L * L);
  ga.invL = 1.0 / L;
  ga.cell_start = w.cell_start;
  ga.ox = w.ox;
  ga.oy = w.oy;
  ga.Yb = w.Yb;
  ga.Ylp = w.Ylp;
  ga.d = w.d;
  ga.rinv = w.rinv;
  ga.abort_flag = w.abort_flag;
  return ga;
}

EvdArgs evd_desc(const ProblemWs& w, int* status) {
  const letkf_problem& p = w.p;
  EvdArgs ea{};
  ea.mode = 0;
  ea.prec = p.precision;
  ea.k = p.k;
  ea.npts = w.npts;
  ea.alpha = (double)(p.k - 1) / p.infl;
  ea.sqrt_km1 = std::sqrt((double)(p.k - 1));
  // Q carries the rounding of its contractions, and the divide and conquer
  // deflates at a matching level: FP64 unit roundoff for the FP64 form,
  // FP32's for the FP32 form; the BF16 form's operands are rounded to 8 bits,
  // so its C is uncertain at about 2^-8 relative and 2^-16 stays far below
  // that noise (measured: the BF16 error is unchanged against 2^-24).
  ea.defl_eps = p.precision == LETKF_PREC_FP64   ? 0x1p-52
                : p.precision == LETKF_PREC_FP32 ? 0x1p-24
                                                 : 0x1p-16;
  ea.xt = w.xt;
  ea.abort_flag = w.abort_flag;
  ea.status = status;
  return ea;
}

ObsArgs obs_args(const ProblemWs& w, const letkf_io& io, int* status) {
  const letkf_problem& p = w.p;
  ObsArgs oa{};
  oa.nx = p.nx;
  oa.ny = p.ny;
  oa.k = p.k;
  oa.kq = w.kp;
  oa.npts = w.npts;
  oa.n_obs = io.n_obs;
  oa.cb = w.cell;
  oa.ncx = w.ncx;
  oa.ncy = w.ncy;
  oa.ncells = w.ncells;
  oa.ix = io.obs_ix;
  oa.iy = io.obs_iy;
  oa.kind = io.obs_kind;
  oa.val = io.obs_val;
  oa.var = io.obs_var;
  oa.obs_cell = w.obs_cell;
  oa.cell_count = w.cell_count;
  oa.cell_start = w.cell_start;
  oa.cell_fill = w.cell_fill;
  oa.perm = w.perm;
  oa.ox = w.ox;
  oa.oy = w.oy;
  oa.Yb = w.Yb;
  oa.Ylp = w.Ylp;
  oa.prec = p.precision;
  oa.d = w.d;
  oa.rinv = w.rinv;
  oa.xt = w.xt;
  oa.abort_flag = w.abort_flag;
  oa.status = status;
  return oa;
}

hipError_t launch_gram(const BatchMap& bm, int kp, int prec, bool persistent, hipStream_t s) {
  return prec == LETKF_PREC_FP64 ? launch_gram_f64(bm, kp, persistent, s)
                                 : launch_gram_lp(bm, kp, prec, persistent, s);
}

// Standalone batched eigensolve (eigenvalues and eigenvectors).
hipError_t launch_evd(const BatchMap& bm, int kp, hipStream_t s) {
  if (kp == 16) return launch_evd_kp<16>(bm, s);
  if (kp == 32) return launch_evd_kp<32>(bm, s);
  if (kp == 64) return launch_evd_kp<64>(bm, s);
  return hipErrorInvalidValue;
}

// Eigensolve + transform + update of an analysis (the eigenvectors are never
// formed).
hipError_t launch_fused(const BatchMap& bm, int kp, int prec, hipStream_t s) {
  if (kp == 16) return launch_fused_kp<16>(bm, prec, s);
  if (kp == 32) return launch_fused_kp<32>(bm, prec, s);
  if (kp == 64) return launch_fused_kp<64>(bm, prec, s);
  return hipErrorInvalidValue;
}

hipError_t launch_xf(const BatchMap& bm, int kp, hipStream_t s) {
  if (kp == 16) return launch_evd_xf_kp<16>(bm, s);
  if (kp == 32) return launch_evd_xf_kp<32>(bm, s);
  if (kp == 64) return launch_evd_xf_kp<64>(bm, s);
  return hipErrorInvalidValue;
}

// Whether a width class runs in the fused form.
bool fused_form(const letkf_plan_s* pl, int kp) {
  if (pl->flags & LETKF_FLAG_NSQRT) return false;
  return pl->form == LETKF_FORM_FUSED || (pl->form == LETKF_FORM_AUTO && kp == 64);
}

// Launch pairs per call of the Gram -> update steps over total points.
int step_launches(const letkf_plan_s* pl, int kp, int total, int slab) {
  return fused_form(pl, kp) ? 1 : ceil_div(total, slab);
}

// Timing marks of one call: [0] start, [1] after binning, [2] after the
// transposes, [3] after the forecast observations, then (Gram, eigensolve)
// per slab, then the end.
struct Marks {
  hipEvent_t* ev = nullptr;
  char* fused = nullptr;      // per launch pair of the call: one fused launch
  int next = 4;
  void at(int i, hipStream_t s) const {
    if (ev) (void)hipEventRecord(ev[i], s);
  }
  // the pair that starts at the next mark is a fused launch
  void set_fused() const {
    if (fused) fused[(next - 4) / 2] = 1;
  }
};

Marks begin_timed(letkf_plan_s* pl, int nslabs) {
  Marks m;
  if (!pl->timing) return m;
  const int slot = pl->next_slot;
  pl->next_slot = (pl->next_slot + 1) % letkf_plan_s::kSlots;
  if (pl->recorded < letkf_plan_s::kSlots) ++pl->recorded;
  m.ev = &pl->ev[(size_t)slot * pl->nev];
  m.fused = &pl->pair_fused[(size_t)slot * pl->max_pairs];
  std::fill(m.fused, m.fused + pl->max_pairs, 0);
  pl->slot_slabs[slot] = nslabs;
  return m;
}

// Gram + eigensolve over the slabs of a problem table (a class or one problem),
// or the fused launch over all of it.
int run_slabs(letkf_plan_s* pl, const GramArgs* g, const EvdArgs* e, const int* prefix, int nprob,
              int total, int kp, int prec, int slab, hipStream_t s, Marks& mk) {
  BatchMap bm{};
  bm.g = g;
  bm.e = e;
  bm.prefix = prefix;
  bm.nprob = nprob;
  bm.C = pl->slab_C;
  bm.b = pl->slab_b;
  bm.queue = pl->queue;
  if (fused_form(pl, kp)) {
    // one launch over every point; the Gram mark then closes an empty phase
    bm.g0 = 0;
    bm.n = total;
    mk.set_fused();
    mk.at(mk.next++, s);
    if (launch_fused(bm, kp, prec, s) != hipSuccess) return LETKF_EDEVICE;
    mk.at(mk.next++, s);
    return LETKF_OK;
  }
  for (int g0 = 0; g0 < total; g0 += slab) {
    bm.g0 = g0;
    bm.n = std::min(slab, total - g0);
    if (launch_gram(bm, kp, prec, pl->form == LETKF_FORM_PERSISTENT, s) != hipSuccess)
      return LETKF_EDEVICE;
    mk.at(mk.next++, s);
    const hipError_t rc = (pl->flags & LETKF_FLAG_NSQRT) ? launch_nsqrt_xf(bm, kp, s)
                                                         : launch_xf(bm, kp, s);
    if (rc != hipSuccess) return LETKF_EDEVICE;
    mk.at(mk.next++, s);
  }
  return LETKF_OK;
}

int check_io(const letkf_plan_s* pl, const letkf_io& io) {
  if (io.problem < 0 || io.problem >= (int)pl->probs.size()) return LETKF_EINVAL;
  const letkf_problem& p = pl->probs[io.problem].p;
  if (io.n_obs < 0 || io.n_obs > p.n_obs_max) return LETKF_EINVAL;
  if (!io.xb || !io.xa) return LETKF_EINVAL;
  if (io.n_obs > 0 &&
      (!io.obs_ix || !io.obs_iy || !io.obs_kind || !io.obs_val || !io.obs_var))
    return LETKF_EINVAL;
  return LETKF_OK;
}

int single_slab(const ProblemWs& w) { return slab_points(w.nb, w.kp, w.npts); }

// Estimated cost of one grid point of a problem, in FP64 flop: the Gram over
// its expected local observations (the observation density at n_obs_max
// times the window area) and the eigensolve and update (11 KP^3).
double point_cost(const ProblemWs& w) {
  const letkf_problem& p = w.p;
  const double dens = (double)p.n_obs_max / ((double)p.nx * p.ny);
  const double side = p.loc == LETKF_LOC_NONE ? 1e30 : 4.0 * p.loc_len + 1.0;
  const double area = std::min(side * side, (double)p.nx * p.ny);
  const double kp = (double)w.kp;
  return dens * area * kp * (kp + 1.0) + 11.0 * kp * kp * kp;
}

// Analyses of n_io problems; src[i] is the member-major background of io[i]
// (io[i].xb, or the cycle's ping-pong buffer).  batched: every problem of the
// plan appears exactly once.
int enqueue(letkf_plan_s* pl, const letkf_io* io, const double* const* src, int n_io, bool batched,
            hipStream_t s) {
  int* status = pl->stat + 1;
  auto prep_bin = [&](int i) -> int {
    const ProblemWs& w = pl->probs[io[i].problem];
    if (launch_fill_i32(w.abort_flag, 1, 0, s) != hipSuccess) return LETKF_EDEVICE;
    const ObsArgs oa = obs_args(w, io[i], status);
    return launch_bin(oa, s) == hipSuccess ? LETKF_OK : LETKF_EDEVICE;
  };
  // the fused form works on the caller's member-major arrays: no transposes,
  // the call's pointers go to the plan's table instead
  auto fused_io = [&](int i) { return fused_form(pl, pl->probs[io[i].problem].kp); };
  PtrBatch ptrs{};
  auto flush_ptrs = [&]() -> int {
    const hipError_t e = launch_store_ptrs(pl->xio, ptrs, s);
    ptrs.n = 0;
    return e == hipSuccess ? LETKF_OK : LETKF_EDEVICE;
  };
  auto prep_transpose = [&](int i) -> int {
    const ProblemWs& w = pl->probs[io[i].problem];
    if (fused_io(i)) {
      ptrs.slot[ptrs.n] = io[i].problem;
      ptrs.xb[ptrs.n] = src[i];
      ptrs.xa[ptrs.n] = io[i].xa;
      return ++ptrs.n == kPtrBatch ? flush_ptrs() : LETKF_OK;
    }
    return launch_transpose_in(src[i], w.xt, w.p.k, w.npts, w.abort_flag, s) == hipSuccess
               ? LETKF_OK
               : LETKF_EDEVICE;
  };
  auto prep_obs = [&](int i) -> int {
    const ProblemWs& w = pl->probs[io[i].problem];
    ObsArgs oa = obs_args(w, io[i], status);
    if (fused_io(i)) oa.xm = src[i];
    return launch_obs_operator(oa, s) == hipSuccess ? LETKF_OK : LETKF_EDEVICE;
  };
  auto untranspose = [&](int i) -> int {
    const ProblemWs& w = pl->probs[io[i].problem];
    if (fused_io(i)) return LETKF_OK;
    return launch_transpose_out(w.xt, io[i].xa, w.p.k, w.npts, w.abort_flag, s) == hipSuccess
               ? LETKF_OK
               : LETKF_EDEVICE;
  };
  int rc = LETKF_OK;
  if (batched) {
    int nslabs = 0;
    for (const ProblemClass& c : pl->classes) nslabs += step_launches(pl, c.kp, c.total, c.slab);
    Marks mk = begin_timed(pl, nslabs);
    mk.at(0, s);
    for (int i = 0; i < n_io && rc == LETKF_OK; ++i) rc = prep_bin(i);
    mk.at(1, s);
    for (int i = 0; i < n_io && rc == LETKF_OK; ++i) rc = prep_transpose(i);
    if (rc == LETKF_OK) rc = flush_ptrs();
    mk.at(2, s);
    for (int i = 0; i < n_io && rc == LETKF_OK; ++i) rc = prep_obs(i);
    mk.at(3, s);
    for (const ProblemClass& c : pl->classes) {
      if (rc != LETKF_OK) break;
      rc = run_slabs(pl, c.g, c.e, c.prefix, (int)c.members.size(), c.total, c.kp, c.prec, c.slab,
                     s, mk);
    }
    for (int i = 0; i < n_io && rc == LETKF_OK; ++i) rc = untranspose(i);
    mk.at(mk.next, s);
    return rc;
  }
  for (int i = 0; i < n_io && rc == LETKF_OK; ++i) {
    const int p = io[i].problem;
    const ProblemWs& w = pl->probs[p];
    Marks mk = i == 0 ? begin_timed(pl, step_launches(pl, w.kp, w.npts, single_slab(w))) : Marks{};
    mk.at(0, s);
    rc = prep_bin(i);
    mk.at(1, s);
    if (rc == LETKF_OK) rc = prep_transpose(i);
    if (rc == LETKF_OK) rc = flush_ptrs();
    mk.at(2, s);
    if (rc == LETKF_OK) rc = prep_obs(i);
    mk.at(3, s);
    if (rc == LETKF_OK)
      rc = run_slabs(pl, pl->g_one + p, pl->e_one + p, pl->prefix_one + 2 * p, 1, w.npts, w.kp,
                     w.p.precision, single_slab(w), s, mk);
    if (rc == LETKF_OK) rc = untranspose(i);
    mk.at(mk.next, s);
  }
  return rc;
}

bool covers_all_once(const letkf_plan_s* pl, const letkf_io* io, int n_io) {
  const int n = (int)pl->probs.size();
  if (n_io != n || n < 2) return false;
  std::vector<char> seen(n, 0);
  for (int i = 0; i < n_io; ++i) {
    if (seen[io[i].problem]) return false;
    seen[io[i].problem] = 1;
  }
  return true;
}

template <class T>
bool upload(const std::vector<T>& h, T* d) {
  return hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess;
}

// Kernel descriptors of every problem (and of each class's concatenation)
// from the plan's current settings, into the plan's device tables.
bool upload_descriptors(letkf_plan_s* pl) {
  const int n_probs = (int)pl->probs.size();
  std::vector<GramArgs> g_host(n_probs);
  std::vector<EvdArgs> e_host(n_probs);
  std::vector<int> pre_host(2 * (size_t)n_probs);
  for (int i = 0; i < n_probs; ++i) {
    g_host[i] = gram_desc(pl->probs[i]);
    e_host[i] = evd_desc(pl->probs[i], pl->stat + 1);
    e_host[i].xio = fused_form(pl, pl->probs[i].kp) ? pl->xio + 2 * i : nullptr;
    pre_host[2 * i] = 0;
    pre_host[2 * i + 1] = pl->probs[i].npts;
  }
  bool ok = upload(g_host, pl->g_one) && upload(e_host, pl->e_one) &&
            upload(pre_host, pl->prefix_one);
  for (auto& c : pl->classes) {
    const size_t n = c.members.size();
    std::vector<GramArgs> gc(n);
    std::vector<EvdArgs> ec(n);
    std::vector<int> pc(n + 1, 0);
    for (size_t j = 0; j < n; ++j) {
      gc[j] = g_host[c.members[j]];
      ec[j] = e_host[c.members[j]];
      pc[j + 1] = pc[j] + pl->probs[c.members[j]].npts;
    }
    ok = ok && upload(gc, c.g) && upload(ec, c.e) && upload(pc, c.prefix);
  }
  return ok;
}


// ---- observations in host memory (LETKF_FLAG_OBS_ON_HOST) ----

// The checks the device makes (k_obs_count), made on the host before anything
// is enqueued.
int check_host_obs(const letkf_problem& p, const letkf_io& io) {
  for (int j = 0; j < io.n_obs; ++j) {
    const int32_t x = io.obs_ix[j], y = io.obs_iy[j], kd = io.obs_kind[j];
    const double var = io.obs_var[j], val = io.obs_val[j];
    const bool var_ok = var > 0.0;                 // false for NaN and <= 0; +inf allowed
    const bool ignored = var_ok && std::isinf(var);
    if (!(x >= 0 && x < p.nx && y >= 0 && y < p.ny && kd >= LETKF_OBS_RHO && kd <= LETKF_OBS_V &&
          var_ok && (ignored || std::isfinite(val))))
      return LETKF_EINVAL;
  }
  return LETKF_OK;
}

// Copies io's host observation arrays into the problem's device buffers on s
// and returns io with its observation pointers moved there.
int stage_host_obs(const ProblemWs& w, const letkf_io& io, hipStream_t s, letkf_io& out) {
  out = io;
  if (io.n_obs == 0) return LETKF_OK;
  const size_t n = (size_t)io.n_obs;
  const hipMemcpyKind h2d = hipMemcpyHostToDevice;
  if (hipMemcpyAsync(w.h_ix, io.obs_ix, n * sizeof(int32_t), h2d, s) != hipSuccess ||
      hipMemcpyAsync(w.h_iy, io.obs_iy, n * sizeof(int32_t), h2d, s) != hipSuccess ||
      hipMemcpyAsync(w.h_kind, io.obs_kind, n * sizeof(int32_t), h2d, s) != hipSuccess ||
      hipMemcpyAsync(w.h_val, io.obs_val, n * sizeof(double), h2d, s) != hipSuccess ||
      hipMemcpyAsync(w.h_var, io.obs_var, n * sizeof(double), h2d, s) != hipSuccess)
    return LETKF_EDEVICE;
  out.obs_ix = w.h_ix;
  out.obs_iy = w.h_iy;
  out.obs_kind = w.h_kind;
  out.obs_val = w.h_val;
  out.obs_var = w.h_var;
  return LETKF_OK;
}

// Host checks of a call's observation records (OBS_ON_HOST plans only).
int check_host_obs_all(const letkf_plan_s* pl, const letkf_io* io, int n_io) {
  if (!(pl->flags & LETKF_FLAG_OBS_ON_HOST)) return LETKF_OK;
  for (int i = 0; i < n_io; ++i) {
    const int rc = check_host_obs(pl->probs[io[i].problem].p, io[i]);
    if (rc != LETKF_OK) return rc;
  }
  return LETKF_OK;
}

// io as the kernels read it: the caller's, or (OBS_ON_HOST) with the
// observations copied to the plan's buffers on s.
int device_ios(const letkf_plan_s* pl, const letkf_io* io, int n_io, hipStream_t s,
               std::vector<letkf_io>& out) {
  out.assign(io, io + n_io);
  if (!(pl->flags & LETKF_FLAG_OBS_ON_HOST)) return LETKF_OK;
  for (int i = 0; i < n_io; ++i) {
    const int rc = stage_host_obs(pl->probs[io[i].problem], io[i], s, out[i]);
    if (rc != LETKF_OK) return rc;
  }
  return LETKF_OK;
}

// ---- tuning cache (letkf_options.tune_cache_path) ----
// One line per entry: "<key> <cell> <form> <ms_per_call>", key =
// 64-bit FNV-1a of the problem list and the device's architecture and CU
// count, in hex.  The last line with a key wins.

uint64_t tune_key(const letkf_plan_s* pl) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  };
  for (const ProblemWs& w : pl->probs) mix(&w.p, sizeof(letkf_problem));
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, pl->device) == hipSuccess) {
    mix(prop.gcnArchName, std::strlen(prop.gcnArchName));
    mix(&prop.multiProcessorCount, sizeof(int));
  }
  return h;
}

bool load_tune_cache(const letkf_plan_s* pl, int* cell, int* form) {
  if (pl->cache_path.empty()) return false;
  FILE* f = std::fopen(pl->cache_path.c_str(), "r");
  if (!f) return false;
  const uint64_t key = tune_key(pl);
  bool found = false;
  char line[256];
  while (std::fgets(line, sizeof line, f)) {
    unsigned long long k = 0;
    int c = 0, pe = 0;
    double ms = 0.0;
    if (std::sscanf(line, "%llx %d %d %lf", &k, &c, &pe, &ms) == 4 && k == key &&
        (c == 4 || c == 8 || c == 16) && pe >= LETKF_FORM_GRID && pe <= LETKF_FORM_AUTO) {
      *cell = c;
      *form = pe;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

bool save_tune_cache(const letkf_plan_s* pl, int cell, int form, double ms) {
  const uint64_t key = tune_key(pl);
  std::vector<std::string> keep;
  if (FILE* f = std::fopen(pl->cache_path.c_str(), "r")) {
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
      unsigned long long k = 0;
      if (std::sscanf(line, "%llx", &k) == 1 && k == key) continue;
      keep.emplace_back(line);
    }
    std::fclose(f);
  }
  const std::string tmp = pl->cache_path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  bool ok = true;
  for (const std::string& l : keep) ok = ok && std::fputs(l.c_str(), f) >= 0;
  ok = ok && std::fprintf(f, "%016llx %d %d %.6f\n", (unsigned long long)key, cell, form, ms) > 0;
  ok = (std::fclose(f) == 0) && ok;
  return ok && std::rename(tmp.c_str(), pl->cache_path.c_str()) == 0;
}

}  // namespace

namespace {

// n_steps lattice-BGK steps of the ensemble xb in place, ping-ponging with the
// problem's BGK buffer so that the last step writes xb (an odd count starts
// from a copy in the buffer).
int advance_ensemble(ProblemWs& w, const letkf_cycle_io& c, hipStream_t s) {
  double* xb = const_cast<double*>(c.io.xb);
  double* cur = xb;
  double* nxt = w.bgk;
  if (c.n_steps % 2 == 1) {
    const size_t bytes = (size_t)w.npts * 9 * w.p.k * sizeof(double);
    if (hipMemcpyAsync(w.bgk, xb, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return LETKF_EDEVICE;
    std::swap(cur, nxt);
  }
  for (int st = 0; st < c.n_steps; ++st) {
    if (launch_bgk(cur, nxt, w.p.k, w.p.nx, w.p.ny, c.tau, c.force_amp, c.force_kx, s) !=
        hipSuccess)
      return LETKF_EDEVICE;
    std::swap(cur, nxt);
  }
  return LETKF_OK;
}

int check_cycle_io(const letkf_plan_s* plan, const letkf_cycle_io& c) {
  const int rc = check_io(plan, c.io);
  if (rc != LETKF_OK) return rc;
  if (c.io.xa != c.io.xb || c.n_steps < 0) return LETKF_EINVAL;
  if (!(c.tau > 0.5) || !std::isfinite(c.tau) || !std::isfinite(c.force_amp)) return LETKF_EINVAL;
  if (c.n_steps > 0 && !plan->probs[c.io.problem].bgk) return LETKF_EINVAL;
  return LETKF_OK;
}

}  // namespace

namespace {

// Workspace of letkf_analyze_noalloc: a file-scope device array, one copy per
// GPU (made when the code object is loaded there, held until the process
// ends).  Host code never passes the array's name to a kernel: the address of
// each device's copy comes from hipGetSymbolAddress, taken once per device
// with that device current, and only that address is used.
constexpr uint64_t kNoAllocBytes = LETKF_NOALLOC_BYTES;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kNoAllocMaxDevices = 64;
std::mutex g_noalloc_mu;
unsigned char* g_noalloc_ptr[kNoAllocMaxDevices] = {};

int noalloc_base(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kNoAllocMaxDevices) return LETKF_EDEVICE;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
      return LETKF_EDEVICE;
    g_noalloc_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_noalloc_ptr[dev];
  return LETKF_OK;
}

// Consecutive 256-byte-aligned pieces of the static workspace; null once it
// is exhausted (nothing is written while the layout is computed).
struct Carve {
  unsigned char* base;
  uint64_t off = 0;
  bool ok = true;
  template <class T>
  T* take(uint64_t count) {
    off = (off + 255) & ~255ull;
    const uint64_t bytes = count * sizeof(T) > 0 ? count * sizeof(T) : 256;
    if (!ok || off + bytes > kNoAllocBytes) {
      ok = false;
      return nullptr;
    }
    T* p = reinterpret_cast<T*>(base + off);
    off += bytes;
    return p;
  }
};

}  // namespace

extern "C" {

const char* letkf_strerror(int code) {
  switch (code) {
    case LETKF_OK: return "ok";
    case LETKF_EINVAL: return "invalid argument";
    case LETKF_ENOMEM:
      return "out of device memory, over the HBM budget, or larger than the no-allocation "
             "workspace";
    case LETKF_EDEVICE: return "no usable gfx950 device or HIP runtime error";
    case LETKF_EBUSY: return "plan in use by another call";
    case LETKF_ENONFINITE: return "non-finite analysis value";
    case LETKF_ENOTCONV: return "eigensolver did not converge";
    case LETKF_EIO: return "tuning cache file could not be written";
    default: return "unknown status";
  }
}

int letkf_plan(const letkf_problem* probs, int32_t n_probs, const letkf_options* opt,
               letkf_plan_t* out) {
  if (out) *out = nullptr;
  if (!out || !probs || n_probs < 1) return LETKF_EINVAL;
  const int flags = opt ? opt->flags : 0;
  if ((flags & ~kKnownFlags) != 0 || (opt && opt->reserved != 0)) return LETKF_EINVAL;
  if ((flags & LETKF_FLAG_GRAPH_CAPTURE) && (flags & LETKF_FLAG_PHASE_TIMING)) return LETKF_EINVAL;
  const bool cycle = flags & LETKF_FLAG_CYCLE;
  const bool host_obs = flags & LETKF_FLAG_OBS_ON_HOST;
  for (int i = 0; i < n_probs; ++i) {
    const int rc = check_problem(probs[i]);
    if (rc != LETKF_OK) return rc;
  }
  std::vector<ProblemWs> ws(n_probs);
  for (int i = 0; i < n_probs; ++i) {
    std::memset(&ws[i], 0, sizeof(ProblemWs));
    ws[i].p = probs[i];
    plan_sizes(ws[i]);
  }
  // classes by (width, precision), in order of first appearance
  std::vector<ProblemClass> classes;
  for (int i = 0; i < n_probs; ++i) {
    int c = 0;
    while (c < (int)classes.size() &&
           !(classes[c].kp == ws[i].kp && classes[c].prec == ws[i].p.precision))
      ++c;
    if (c == (int)classes.size()) {
      ProblemClass pc;
      pc.kp = ws[i].kp;
      pc.prec = ws[i].p.precision;
      pc.nb = ws[i].nb;
      classes.push_back(pc);
    }
    classes[c].members.push_back(i);
    classes[c].total += ws[i].npts;
  }
  // members dearest per point first: the fused form's queues then hand out
  // the expensive points early and the cheap ones fill the tail (the order
  // changes no result; every point is independent)
  for (auto& c : classes)
    std::stable_sort(c.members.begin(), c.members.end(), [&](int a, int b) {
      return point_cost(ws[a]) > point_cost(ws[b]);
    });
  // slab buffers: the largest slab of any class or single problem
  uint64_t c_doubles = 0, b_doubles = 0;
  for (auto& c : classes) {
    c.slab = slab_points(c.nb, c.kp, c.total);
    c_doubles = std::max(c_doubles, (uint64_t)c.slab * c.nb * 256);
    b_doubles = std::max(b_doubles, (uint64_t)c.slab * c.kp);
  }
  for (auto& w : ws) {
    const uint64_t sl = (uint64_t)single_slab(w);
    c_doubles = std::max(c_doubles, sl * w.nb * 256);
    b_doubles = std::max(b_doubles, sl * w.kp);
    // the fused form's slots: one per block of its device-filling launch
    c_doubles = std::max(c_doubles, (uint64_t)kFusedBlocks * fused_slot_c(w.kp));
    b_doubles = std::max(b_doubles, (uint64_t)kFusedBlocks * fused_slot_b(w.kp));
  }
  uint64_t total = 4096 + (c_doubles + b_doubles) * sizeof(double);
  for (auto& w : ws) total += ws_bytes(w, cycle, host_obs);
  if (opt && opt->hbm_budget_bytes && total > opt->hbm_budget_bytes) return LETKF_ENOMEM;
  int dev = 0;
  const int drc = check_device(&dev);
  if (drc != LETKF_OK) return drc;

  letkf_plan_s* pl = new (std::nothrow) letkf_plan_s();
  if (!pl) return LETKF_ENOMEM;
  pl->device = dev;
  pl->flags = flags;
  if (opt && opt->tune_cache_path) pl->cache_path = opt->tune_cache_path;
  pl->probs = ws;
  pl->classes = classes;
  bool ok = pl->alloc(&pl->stat, 2 + (size_t)n_probs);
  ok = ok && hipStreamCreateWithFlags(&pl->aux, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&pl->host_stat, sizeof(int), hipHostMallocDefault) == hipSuccess;
  for (int i = 0; ok && i < n_probs; ++i) {
    ProblemWs& w = pl->probs[i];
    const int k = w.p.k;
    const size_t no = (size_t)w.nobs_alloc;
    w.abort_flag = pl->stat + 2 + i;
    ok = ok && pl->alloc(&w.xt, (size_t)w.npts * 9 * k);
    ok = ok && pl->alloc(&w.obs_cell, no) && pl->alloc(&w.perm, no) && pl->alloc(&w.ox, no) &&
         pl->alloc(&w.oy, no);
    if (w.p.precision == LETKF_PREC_FP64) {
      ok = ok && pl->alloc(&w.Yb, no * w.kp);
    } else {
      unsigned char* q = nullptr;
      ok = ok && pl->alloc(&q, no * w.kp * (w.p.precision == LETKF_PREC_FP32 ? 4 : 2));
      w.Ylp = q;
    }
    ok = ok && pl->alloc(&w.d, no) && pl->alloc(&w.rinv, no);
    const int mc = max_cells(w);
    ok = ok && pl->alloc(&w.cell_count, mc) && pl->alloc(&w.cell_start, mc + 1) &&
         pl->alloc(&w.cell_fill, mc);
    if (cycle) ok = ok && pl->alloc(&w.bgk, (size_t)w.npts * 9 * k);
    if (host_obs)
      ok = ok && pl->alloc(&w.h_ix, no) && pl->alloc(&w.h_iy, no) && pl->alloc(&w.h_kind, no) &&
           pl->alloc(&w.h_val, no) && pl->alloc(&w.h_var, no);
  }
  // a setting recorded by an earlier letkf_tune for the same problems and device
  if (ok) {
    int cell = kCell, form = LETKF_FORM_AUTO;
    if (load_tune_cache(pl, &cell, &form)) {
      if (flags & LETKF_FLAG_DETERMINISTIC) cell = kCell;
      for (auto& w : pl->probs) set_cell(w, cell);
      pl->form = form;
    }
  }
  ok = ok && pl->alloc(&pl->slab_C, (size_t)c_doubles) && pl->alloc(&pl->slab_b, (size_t)b_doubles);
  // descriptors: one per problem, and one table per class
  ok = ok && pl->alloc(&pl->g_one, n_probs) && pl->alloc(&pl->e_one, n_probs) &&
       pl->alloc(&pl->prefix_one, 2 * (size_t)n_probs) && pl->alloc(&pl->queue, kQueueSlots) &&
       pl->alloc(&pl->xio, 2 * (size_t)n_probs);
  for (auto& c : pl->classes) {
    const size_t n = c.members.size();
    ok = ok && pl->alloc(&c.g, n) && pl->alloc(&c.e, n) && pl->alloc(&c.prefix, n + 1);
  }
  ok = ok && upload_descriptors(pl);
  if (ok && opt && (opt->flags & LETKF_FLAG_PHASE_TIMING)) {
    int max_slabs = 0;
    for (auto& c : pl->classes) max_slabs += ceil_div(c.total, c.slab);   // >= the fused form's
    for (auto& w : pl->probs) max_slabs = std::max(max_slabs, ceil_div(w.npts, single_slab(w)));
    pl->timing = true;
    pl->nev = 5 + 2 * max_slabs;
    pl->ev.resize((size_t)letkf_plan_s::kSlots * pl->nev);
    pl->slot_slabs.assign(letkf_plan_s::kSlots, 0);
    pl->max_pairs = max_slabs;
    pl->pair_fused.assign((size_t)letkf_plan_s::kSlots * max_slabs, 0);
    for (auto& e : pl->ev) ok = ok && hipEventCreate(&e) == hipSuccess;
  }
  if (!ok || hipMemset(pl->stat, 0, (2 + (size_t)n_probs) * sizeof(int)) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    pl->release();
    delete pl;
    return LETKF_ENOMEM;
  }
  *out = pl;
  return LETKF_OK;
}

int letkf_analyze(letkf_plan_t plan, const letkf_io* io, int32_t n_io, void* hip_stream) {
  if (!plan || (!io && n_io > 0) || n_io < 0) return LETKF_EINVAL;
  for (int i = 0; i < n_io; ++i) {
    const int rc = check_io(plan, io[i]);
    if (rc != LETKF_OK) return rc;
  }
  if (check_host_obs_all(plan, io, n_io) != LETKF_OK) return LETKF_EINVAL;
  int expect = 0;
  if (!plan->busy.compare_exchange_strong(expect, 1)) return LETKF_EBUSY;
  DeviceGuard guard(plan->device);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  std::vector<letkf_io> dio;
  int rc = device_ios(plan, io, n_io, s, dio);
  std::vector<const double*> src(n_io);
  for (int i = 0; i < n_io; ++i) src[i] = io[i].xb;
  if (rc == LETKF_OK)
    rc = enqueue(plan, dio.data(), src.data(), n_io, covers_all_once(plan, io, n_io), s);
  plan->last_stream = s;
  plan->busy.store(0);
  return rc;
}

int letkf_cycle(letkf_plan_t plan, const letkf_cycle_io* io, int32_t n_io, void* hip_stream) {
  if (!plan || (!io && n_io > 0) || n_io < 0) return LETKF_EINVAL;
  for (int i = 0; i < n_io; ++i) {
    const int rc = check_cycle_io(plan, io[i]);
    if (rc != LETKF_OK) return rc;
  }
  std::vector<letkf_io> ios(n_io);
  for (int i = 0; i < n_io; ++i) ios[i] = io[i].io;
  if (check_host_obs_all(plan, ios.data(), n_io) != LETKF_OK) return LETKF_EINVAL;
  int expect = 0;
  if (!plan->busy.compare_exchange_strong(expect, 1)) return LETKF_EBUSY;
  DeviceGuard guard(plan->device);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  std::vector<letkf_io> dio;
  int rc = device_ios(plan, ios.data(), n_io, s, dio);
  // the advanced state is in io.xb whether or not the analysis runs
  std::vector<const double*> src(n_io);
  for (int i = 0; i < n_io && rc == LETKF_OK; ++i) {
    rc = advance_ensemble(plan->probs[io[i].io.problem], io[i], s);
    src[i] = io[i].io.xb;
  }
  if (rc == LETKF_OK)
    rc = enqueue(plan, dio.data(), src.data(), n_io, covers_all_once(plan, ios.data(), n_io), s);
  plan->last_stream = s;
  plan->busy.store(0);
  return rc;
}

int letkf_advance(letkf_plan_t plan, const letkf_cycle_io* io, int32_t n_io, void* hip_stream) {
  if (!plan || (!io && n_io > 0) || n_io < 0) return LETKF_EINVAL;
  for (int i = 0; i < n_io; ++i) {
    if (io[i].io.problem < 0 || io[i].io.problem >= (int)plan->probs.size()) return LETKF_EINVAL;
    if (!io[i].io.xb || io[i].io.xa != io[i].io.xb || io[i].n_steps < 0) return LETKF_EINVAL;
    if (!(io[i].tau > 0.5) || !std::isfinite(io[i].tau) || !std::isfinite(io[i].force_amp))
      return LETKF_EINVAL;
    if (io[i].n_steps > 0 && !plan->probs[io[i].io.problem].bgk) return LETKF_EINVAL;
  }
  int expect = 0;
  if (!plan->busy.compare_exchange_strong(expect, 1)) return LETKF_EBUSY;
  DeviceGuard guard(plan->device);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int rc = LETKF_OK;
  for (int i = 0; i < n_io && rc == LETKF_OK; ++i)
    rc = advance_ensemble(plan->probs[io[i].io.problem], io[i], s);
  plan->last_stream = s;
  plan->busy.store(0);
  return rc;
}

int letkf_tune(letkf_plan_t plan, const letkf_io* io_in, int32_t n_io, void* hip_stream,
               letkf_tuning* out) {
  if (!plan || !io_in || n_io < 1) return LETKF_EINVAL;
  for (int i = 0; i < n_io; ++i) {
    const int rc = check_io(plan, io_in[i]);
    if (rc != LETKF_OK) return rc;
  }
  if (check_host_obs_all(plan, io_in, n_io) != LETKF_OK) return LETKF_EINVAL;
  int expect = 0;
  if (!plan->busy.compare_exchange_strong(expect, 1)) return LETKF_EBUSY;
  DeviceGuard guard(plan->device);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // the kernel descriptors are rewritten below: earlier calls must be done
  if (hipStreamSynchronize(plan->last_stream) != hipSuccess) {
    plan->busy.store(0);
    return LETKF_EDEVICE;
  }
  std::vector<letkf_io> dio;
  if (device_ios(plan, io_in, n_io, s, dio) != LETKF_OK) {
    plan->busy.store(0);
    return LETKF_EDEVICE;
  }
  const letkf_io* io = dio.data();
  std::vector<const double*> src(n_io);
  for (int i = 0; i < n_io; ++i) src[i] = io[i].xb;
  const bool batched = covers_all_once(plan, io, n_io);
  const bool saved_timing = plan->timing;
  plan->timing = false;                          // tuning calls stay out of the phase record
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess ? LETKF_OK
                                                                                 : LETKF_EDEVICE;
  constexpr int kCells[3] = {4, 8, 16};
  constexpr int kReps = 2;
  double best_ms = 0.0;
  int best_cell = kCell;
  int best_form = LETKF_FORM_GRID;
  bool have = false;
  // DETERMINISTIC: only the kernel form, which leaves every bit unchanged;
  // NSQRT plans have no fused form
  const bool det = plan->flags & LETKF_FLAG_DETERMINISTIC;
  const int nforms = (plan->flags & LETKF_FLAG_NSQRT) ? 2 : 3;
  for (int ci = det ? 1 : 0; ci < (det ? 2 : 3) && rc == LETKF_OK; ++ci) {
    for (int pi = 0; pi < nforms && rc == LETKF_OK; ++pi) {
      for (auto& w : plan->probs) set_cell(w, kCells[ci]);
      plan->form = pi;
      if (!upload_descriptors(plan)) {
        rc = LETKF_EDEVICE;
        break;
      }
      rc = enqueue(plan, io, src.data(), n_io, batched, s);          // warm-up
      if (rc == LETKF_OK && hipEventRecord(e0, s) != hipSuccess) rc = LETKF_EDEVICE;
      for (int r = 0; r < kReps && rc == LETKF_OK; ++r) rc = enqueue(plan, io, src.data(), n_io, batched, s);
      float ms = 0.f;
      if (rc == LETKF_OK && (hipEventRecord(e1, s) != hipSuccess ||
                             hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = LETKF_EDEVICE;
      if (rc == LETKF_OK && (!have || ms / kReps < best_ms)) {
        have = true;
        best_ms = ms / kReps;
        best_cell = kCells[ci];
        best_form = pi;
      }
    }
  }
  for (auto& w : plan->probs) set_cell(w, best_cell);
  plan->form = best_form;
  if (!upload_descriptors(plan) && rc == LETKF_OK) rc = LETKF_EDEVICE;
  if (rc == LETKF_OK) {
    // leave the outputs as one plain analysis with the chosen settings would
    rc = enqueue(plan, io, src.data(), n_io, batched, s);
    if (rc == LETKF_OK && hipStreamSynchronize(s) != hipSuccess) rc = LETKF_EDEVICE;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  plan->timing = saved_timing;
  plan->last_stream = s;
  if (rc == LETKF_OK && out) {
    out->cell = best_cell;
    out->form = best_form;
    out->ms_per_call = best_ms;
  }
  if (rc == LETKF_OK && !plan->cache_path.empty() &&
      !save_tune_cache(plan, best_cell, best_form, best_ms))
    rc = LETKF_EIO;
  plan->busy.store(0);
  return rc;
}

int letkf_set_tuning(letkf_plan_t plan, const letkf_tuning* t) {
  if (!plan || !t) return LETKF_EINVAL;
  if (t->cell != 4 && t->cell != 8 && t->cell != 16) return LETKF_EINVAL;
  if (t->form < LETKF_FORM_GRID || t->form > LETKF_FORM_AUTO) return LETKF_EINVAL;
  int expect = 0;
  if (!plan->busy.compare_exchange_strong(expect, 1)) return LETKF_EBUSY;
  DeviceGuard guard(plan->device);
  int rc = hipStreamSynchronize(plan->last_stream) == hipSuccess ? LETKF_OK : LETKF_EDEVICE;
  if (rc == LETKF_OK) {
    for (auto& w : plan->probs) set_cell(w, t->cell);
    plan->form = t->form;
    if (!upload_descriptors(plan)) rc = LETKF_EDEVICE;
  }
  plan->busy.store(0);
  return rc;
}

int letkf_status(letkf_plan_t plan, int32_t sync) {
  if (!plan) return LETKF_EINVAL;
  DeviceGuard guard(plan->device);
  if (sync && hipStreamSynchronize(plan->last_stream) != hipSuccess) return LETKF_EDEVICE;
  // read on the plan's own non-blocking stream (waits for nothing else), then
  // clear exactly the bits read with an atomic on the device
  if (hipMemcpyAsync(plan->host_stat, plan->stat + 1, sizeof(int), hipMemcpyDeviceToHost,
                     plan->aux) != hipSuccess ||
      hipStreamSynchronize(plan->aux) != hipSuccess)
    return LETKF_EDEVICE;
  const int bits = *plan->host_stat;
  if (bits && (launch_clear_bits(plan->stat + 1, bits, plan->aux) != hipSuccess ||
               hipStreamSynchronize(plan->aux) != hipSuccess))
    return LETKF_EDEVICE;
  if (bits & kStatEinval) return LETKF_EINVAL;
  if (bits & kStatNonfinite) return LETKF_ENONFINITE;
  if (bits & kStatNotconv) return LETKF_ENOTCONV;
  return LETKF_OK;
}

int letkf_plan_destroy(letkf_plan_t plan) {
  if (!plan) return LETKF_OK;
  {
    DeviceGuard guard(plan->device);
    (void)hipDeviceSynchronize();
    plan->release();
  }
  delete plan;
  return LETKF_OK;
}

uint64_t letkf_plan_workspace_bytes(letkf_plan_t plan) { return plan ? plan->bytes : 0; }

int letkf_phase_times(letkf_plan_t plan, double* ms, int32_t* launches, int32_t n) {
  if (!plan || !ms || n < 0) return -LETKF_EINVAL;
  if (!plan->timing) return -LETKF_EINVAL;
  DeviceGuard guard(plan->device);
  if (hipStreamSynchronize(plan->last_stream) != hipSuccess) return -LETKF_EDEVICE;
  double acc[LETKF_N_PHASES] = {0, 0, 0, 0, 0, 0, 0};
  int last_split = 0, last_fused = 0;
  const int calls = plan->recorded;
  for (int c = 0; c < calls; ++c) {
    const int slot = (plan->next_slot - 1 - c + 2 * letkf_plan_s::kSlots) % letkf_plan_s::kSlots;
    const hipEvent_t* ev = &plan->ev[(size_t)slot * plan->nev];
    const int nsl = plan->slot_slabs[slot];
    const char* fused = &plan->pair_fused[(size_t)slot * plan->max_pairs];
    last_split = last_fused = 0;
    float t = 0.f;
    auto el = [&](int a, int b) -> double {
      return hipEventElapsedTime(&t, ev[a], ev[b]) == hipSuccess ? (double)t : 0.0;
    };
    acc[LETKF_PHASE_BIN] += el(0, 1);
    acc[LETKF_PHASE_TRANSPOSE] += el(1, 2);
    acc[LETKF_PHASE_OBSOP] += el(2, 3);
    int prev = 3;
    for (int ci = 0; ci < nsl; ++ci) {
      if (fused[ci]) {
        acc[LETKF_PHASE_FUSED] += el(prev, 5 + 2 * ci);
        ++last_fused;
      } else {
        ++last_split;
        acc[LETKF_PHASE_GRAM] += el(prev, 4 + 2 * ci);
        acc[LETKF_PHASE_EVD] += el(4 + 2 * ci, 5 + 2 * ci);
      }
      prev = 5 + 2 * ci;
    }
    acc[LETKF_PHASE_UNTRANS] += el(prev, 4 + 2 * nsl);
  }
  const int bin_launches = 5;  // two fills, count, scan, scatter + sort
  const int per_call[LETKF_N_PHASES] = {bin_launches, 1, 1, last_split, last_split, 1,
                                        last_fused};
  for (int i = 0; i < n; ++i) {
    ms[i] = i < LETKF_N_PHASES ? acc[i] : 0.0;
    if (launches) launches[i] = i < LETKF_N_PHASES ? per_call[i] : 0;
  }
  plan->recorded = 0;
  return calls;
}

int letkf_eigh_batched(const double* a, int32_t batch, int32_t k, double* lam, double* vec,
                       int32_t* status, void* hip_stream) {
  if (batch < 0 || k < 1 || k > LETKF_MAX_K) return LETKF_EINVAL;
  if (batch == 0) return LETKF_OK;
  if (!a || !lam || !vec) return LETKF_EINVAL;
  BatchMap bm{};
  bm.nprob = 1;
  bm.g0 = 0;
  bm.n = batch;
  EvdArgs& ea = bm.e_inline;
  ea.mode = 1;
  ea.k = k;
  ea.npts = batch;
  ea.defl_eps = 0x1p-52;
  ea.A = a;
  ea.lam = lam;
  ea.vec = vec;
  ea.status = status;
  const int kp = pow2_at_least16(k);
  return launch_evd(bm, kp, static_cast<hipStream_t>(hip_stream)) == hipSuccess ? LETKF_OK
                                                                                 : LETKF_EDEVICE;
}

int letkf_invsqrt_batched(const double* a, int32_t batch, int32_t k, double* x,
                          int32_t* status, int32_t* steps, void* hip_stream) {
  if (batch < 0 || k < 1 || k > LETKF_MAX_K) return LETKF_EINVAL;
  if (batch == 0) return LETKF_OK;
  if (!a || !x) return LETKF_EINVAL;
  return launch_nsqrt(a, batch, k, x, status, steps, static_cast<hipStream_t>(hip_stream)) ==
                 hipSuccess
             ? LETKF_OK
             : LETKF_EDEVICE;
}

int letkf_analyze_noalloc(const letkf_problem* prob, const letkf_io* io, int32_t* status,
                          void* hip_stream) {
  if (!prob || !io || !status) return LETKF_EINVAL;
  int rc = check_problem(*prob);
  if (rc != LETKF_OK) return rc;
  if (io->n_obs < 0 || io->n_obs > prob->n_obs_max || !io->xb || !io->xa) return LETKF_EINVAL;
  if (io->n_obs > 0 &&
      (!io->obs_ix || !io->obs_iy || !io->obs_kind || !io->obs_val || !io->obs_var))
    return LETKF_EINVAL;
  int dev = 0;
  rc = check_device(&dev);
  if (rc != LETKF_OK) return rc;
  Carve cv;
  rc = noalloc_base(dev, &cv.base);
  if (rc != LETKF_OK) return rc;
  // layout of one problem's workspace (as letkf_plan's, without the tuner's
  // extra cells, the BGK buffer or host-observation copies)
  ProblemWs w;
  std::memset(&w, 0, sizeof(ProblemWs));
  w.p = *prob;
  plan_sizes(w);
  const uint64_t no = (uint64_t)w.nobs_alloc;
  w.abort_flag = cv.take<int>(1);
  w.xt = cv.take<double>((uint64_t)w.npts * 9 * w.p.k);
  w.obs_cell = cv.take<int>(no);
  w.perm = cv.take<int>(no);
  w.ox = cv.take<int>(no);
  w.oy = cv.take<int>(no);
  if (w.p.precision == LETKF_PREC_FP64)
    w.Yb = cv.take<double>(no * w.kp);
  else
    w.Ylp = cv.take<unsigned char>(no * w.kp * (w.p.precision == LETKF_PREC_FP32 ? 4 : 2));
  w.d = cv.take<double>(no);
  w.rinv = cv.take<double>(no);
  w.cell_count = cv.take<int>(w.ncells);
  w.cell_start = cv.take<int>((uint64_t)w.ncells + 1);
  w.cell_fill = cv.take<int>(w.ncells);
  // the Gram output slab takes what is left, at least 256 points (or all)
  const uint64_t per_pt = ((uint64_t)w.nb * 256 + w.kp) * sizeof(double);
  const uint64_t left = cv.ok && cv.off + 1024 < kNoAllocBytes ? kNoAllocBytes - cv.off - 1024 : 0;
  const int slab = (int)std::min<uint64_t>((uint64_t)w.npts, left / per_pt);
  if (!cv.ok || slab < std::min(256, w.npts)) return LETKF_ENOMEM;
  double* slab_C = cv.take<double>((uint64_t)slab * w.nb * 256);
  double* slab_b = cv.take<double>((uint64_t)slab * w.kp);
  if (!cv.ok) return LETKF_ENOMEM;

  DeviceGuard guard(dev);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // status and abort flag start at zero (fill kernels: no memset nodes under capture)
  if (launch_fill_i32(status, 1, 0, s) != hipSuccess) return LETKF_EDEVICE;
  if (launch_fill_i32(w.abort_flag, 1, 0, s) != hipSuccess) return LETKF_EDEVICE;
  const ObsArgs oa = obs_args(w, *io, status);
  if (launch_bin(oa, s) != hipSuccess) return LETKF_EDEVICE;
  if (launch_transpose_in(io->xb, w.xt, w.p.k, w.npts, w.abort_flag, s) != hipSuccess)
    return LETKF_EDEVICE;
  if (launch_obs_operator(oa, s) != hipSuccess) return LETKF_EDEVICE;
  BatchMap bm{};
  bm.nprob = 1;
  bm.C = slab_C;
  bm.b = slab_b;
  bm.g_inline = gram_desc(w);
  bm.e_inline = evd_desc(w, status);
  for (int g0 = 0; g0 < w.npts; g0 += slab) {
    bm.g0 = g0;
    bm.n = std::min(slab, w.npts - g0);
    if (launch_gram(bm, w.kp, w.p.precision, false, s) != hipSuccess) return LETKF_EDEVICE;
    if (launch_xf(bm, w.kp, s) != hipSuccess) return LETKF_EDEVICE;
  }
  if (launch_transpose_out(w.xt, io->xa, w.p.k, w.npts, w.abort_flag, s) != hipSuccess)
    return LETKF_EDEVICE;
  return LETKF_OK;
}

}  // extern "C"
