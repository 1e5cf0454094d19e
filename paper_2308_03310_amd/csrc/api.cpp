// C-ABI of the LETKF library (include/letkf.h): plans, argument checks,
// workspace ownership and the stream-ordered launch sequence of one analysis.
#include "../../include/letkf.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <vector>

#include "common.h"
#include "launch.h"

using namespace letkf;

namespace {

constexpr int kCell = 8;                       // observation-cell edge (lattice points)
constexpr int kMaxDim = 32768;                 // keeps squared distances inside int32
constexpr uint64_t kChunkBytes = 1ull << 30;   // per-chunk Gram output
constexpr double kJacobiTol2 = 1e-24;          // (1e-12)^2 relative off-diagonal norm
constexpr int kJacobiMaxSweeps = 60;

struct ProblemWs {
  letkf_problem p;
  int npts, kp, nb, ncx, ncy, ncells, chunk, nobs_alloc;
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
  double* C;
  double* b;
  double* bgk;   // lattice-BGK ping-pong buffer (plans made with LETKF_FLAG_CYCLE)
};

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int check_problem(const letkf_problem& p) {
  if (p.nx < 1 || p.ny < 1 || p.nx > kMaxDim || p.ny > kMaxDim) return LETKF_EINVAL;
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

}  // namespace

struct letkf_plan_s {
  int device = 0;
  std::vector<ProblemWs> probs;
  int* stat = nullptr;  // device: [0] abort flag of the running call, [1] sticky status bits
  std::vector<void*> allocs;
  uint64_t bytes = 0;
  std::atomic<int> busy{0};
  hipStream_t last_stream = nullptr;
  // Phase timing: a ring of event sets, one set per timed analyze call.
  static constexpr int kSlots = 256;
  bool timing = false;
  int nev = 0;                      // events per slot
  std::vector<hipEvent_t> ev;       // kSlots * nev
  std::vector<int> slot_chunks;     // chunks launched in the slot's call
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
  }
};

namespace {

void plan_sizes(ProblemWs& w) {
  const letkf_problem& p = w.p;
  w.npts = p.nx * p.ny;
  w.kp = pow2_at_least16(p.k);
  w.nb = n_upper_blocks(w.kp);
  w.ncx = ceil_div(p.nx, kCell);
  w.ncy = ceil_div(p.ny, kCell);
  w.ncells = w.ncx * w.ncy;
  const uint64_t per_pt = (uint64_t)w.nb * 256 * sizeof(double);
  uint64_t ch = kChunkBytes / per_pt;
  if (ch < 256) ch = 256;
  w.chunk = (int)(ch < (uint64_t)w.npts ? ch : (uint64_t)w.npts);
  w.nobs_alloc = p.n_obs_max > 0 ? p.n_obs_max : 1;
}

uint64_t ws_bytes(const ProblemWs& w) {
  const uint64_t no = (uint64_t)w.nobs_alloc;
  uint64_t b = (uint64_t)w.npts * 9 * w.p.k * sizeof(double);
  const uint64_t ybytes = w.p.precision == LETKF_PREC_FP64 ? 8 : (w.p.precision == LETKF_PREC_FP32 ? 4 : 2);
  b += no * 5 * sizeof(int) + no * w.kp * ybytes + no * 2 * sizeof(double);
  b += (uint64_t)(3 * w.ncells + 1) * sizeof(int);
  b += (uint64_t)w.chunk * (w.nb * 256 + w.kp) * sizeof(double);
  return b;
}

// src: member-major background to analyse (io.xb unless a cycle left it in
// the ping-pong buffer).
int enqueue_analysis(letkf_plan_s* pl, const letkf_io& io, hipStream_t s, bool timed,
                     const double* src) {
  ProblemWs& w = pl->probs[io.problem];
  const letkf_problem& p = w.p;
  const int k = p.k;
  int* abort_flag = pl->stat;
  hipEvent_t* ev = nullptr;
  if (timed) {
    const int slot = pl->next_slot;
    pl->next_slot = (pl->next_slot + 1) % letkf_plan_s::kSlots;
    if (pl->recorded < letkf_plan_s::kSlots) ++pl->recorded;
    ev = &pl->ev[(size_t)slot * pl->nev];
    pl->slot_chunks[slot] = ceil_div(w.npts, w.chunk);
  }
  auto mark = [&](int i) {
    if (ev) (void)hipEventRecord(ev[i], s);
  };
  hipError_t e;
  mark(0);
  if ((e = launch_fill_i32(abort_flag, 1, 0, s)) != hipSuccess) return LETKF_EDEVICE;

  ObsArgs oa{};
  oa.nx = p.nx;
  oa.ny = p.ny;
  oa.k = k;
  oa.kq = w.kp;
  oa.npts = w.npts;
  oa.n_obs = io.n_obs;
  oa.cb = kCell;
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
  oa.abort_flag = abort_flag;
  oa.status = pl->stat + 1;

  if (launch_bin(oa, s) != hipSuccess) return LETKF_EDEVICE;
  mark(1);
  if (launch_transpose_in(src, w.xt, k, w.npts, abort_flag, s) != hipSuccess) return LETKF_EDEVICE;
  mark(2);
  if (launch_obs_operator(oa, s) != hipSuccess) return LETKF_EDEVICE;
  mark(3);

  GramArgs ga{};
  ga.nx = p.nx;
  ga.ny = p.ny;
  ga.k = k;
  ga.cb = kCell;
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
  ga.C = w.C;
  ga.b = w.b;
  ga.abort_flag = abort_flag;

  EvdArgs ea{};
  ea.mode = 0;
  ea.prec = p.precision;
  ea.k = k;
  ea.npts = w.npts;
  ea.alpha = (double)(k - 1) / p.infl;
  ea.sqrt_km1 = std::sqrt((double)(k - 1));
  ea.tol2 = kJacobiTol2;
  ea.max_sweeps = kJacobiMaxSweeps;
  ea.C = w.C;
  ea.b = w.b;
  ea.xt = w.xt;
  ea.abort_flag = abort_flag;
  ea.status = pl->stat + 1;

  int ci = 0;
  for (int pt0 = 0; pt0 < w.npts; pt0 += w.chunk, ++ci) {
    const int n = (w.npts - pt0) < w.chunk ? (w.npts - pt0) : w.chunk;
    ga.pt0 = pt0;
    ga.npt = n;
    const hipError_t ge = p.precision == LETKF_PREC_FP64 ? launch_gram_f64(ga, w.kp, s)
                                                         : launch_gram_lp(ga, w.kp, p.precision, s);
    if (ge != hipSuccess) return LETKF_EDEVICE;
    mark(4 + 2 * ci);
    ea.pt0 = pt0;
    ea.npt = n;
    hipError_t le = hipErrorInvalidValue;
    if (w.kp == 16) le = launch_evd_kp<16>(ea, s);
    else if (w.kp == 32) le = launch_evd_kp<32>(ea, s);
    else if (w.kp == 64) le = launch_evd_kp<64>(ea, s);
    if (le != hipSuccess) return LETKF_EDEVICE;
    mark(5 + 2 * ci);
  }
  if (launch_transpose_out(w.xt, io.xa, k, w.npts, abort_flag, s) != hipSuccess)
    return LETKF_EDEVICE;
  mark(4 + 2 * ci);
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

}  // namespace

extern "C" {

const char* letkf_strerror(int code) {
  switch (code) {
    case LETKF_OK: return "ok";
    case LETKF_EINVAL: return "invalid argument";
    case LETKF_ENOMEM: return "out of device memory or over the HBM budget";
    case LETKF_EDEVICE: return "no usable gfx950 device or HIP runtime error";
    case LETKF_EBUSY: return "plan in use by another call";
    case LETKF_ENONFINITE: return "non-finite analysis value";
    case LETKF_ENOTCONV: return "eigensolver did not converge";
    default: return "unknown status";
  }
}

int letkf_plan(const letkf_problem* probs, int32_t n_probs, const letkf_options* opt,
               letkf_plan_t* out) {
  if (out) *out = nullptr;
  if (!out || !probs || n_probs < 1) return LETKF_EINVAL;
  if (opt && (opt->flags & ~(LETKF_FLAG_PHASE_TIMING | LETKF_FLAG_CYCLE)) != 0) return LETKF_EINVAL;
  const bool cycle = opt && (opt->flags & LETKF_FLAG_CYCLE);
  for (int i = 0; i < n_probs; ++i) {
    const int rc = check_problem(probs[i]);
    if (rc != LETKF_OK) return rc;
  }
  std::vector<ProblemWs> ws(n_probs);
  uint64_t total = 64;
  for (int i = 0; i < n_probs; ++i) {
    std::memset(&ws[i], 0, sizeof(ProblemWs));
    ws[i].p = probs[i];
    plan_sizes(ws[i]);
    total += ws_bytes(ws[i]);
    if (cycle) total += (uint64_t)ws[i].npts * 9 * probs[i].k * sizeof(double);
  }
  if (opt && opt->hbm_budget_bytes && total > opt->hbm_budget_bytes) return LETKF_ENOMEM;
  int dev = 0;
  const int drc = check_device(&dev);
  if (drc != LETKF_OK) return drc;

  letkf_plan_s* pl = new (std::nothrow) letkf_plan_s();
  if (!pl) return LETKF_ENOMEM;
  pl->device = dev;
  pl->probs = ws;
  bool ok = pl->alloc(&pl->stat, 4);
  for (auto& w : pl->probs) {
    const int k = w.p.k;
    const size_t no = (size_t)w.nobs_alloc;
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
    ok = ok && pl->alloc(&w.cell_count, w.ncells) && pl->alloc(&w.cell_start, w.ncells + 1) &&
         pl->alloc(&w.cell_fill, w.ncells);
    ok = ok && pl->alloc(&w.C, (size_t)w.chunk * w.nb * 256) && pl->alloc(&w.b, (size_t)w.chunk * w.kp);
    if (cycle) ok = ok && pl->alloc(&w.bgk, (size_t)w.npts * 9 * k);
    if (!ok) break;
  }
  if (ok && opt && (opt->flags & LETKF_FLAG_PHASE_TIMING)) {
    int max_chunks = 1;
    for (auto& w : pl->probs) max_chunks = std::max(max_chunks, ceil_div(w.npts, w.chunk));
    pl->timing = true;
    pl->nev = 5 + 2 * max_chunks;
    pl->ev.resize((size_t)letkf_plan_s::kSlots * pl->nev);
    pl->slot_chunks.assign(letkf_plan_s::kSlots, 0);
    for (auto& e : pl->ev) ok = ok && hipEventCreate(&e) == hipSuccess;
  }
  if (!ok || hipMemset(pl->stat, 0, 4 * sizeof(int)) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    pl->release();
    delete pl;
    return LETKF_ENOMEM;
  }
  *out = pl;
  return LETKF_OK;
}

int letkf_analyze(letkf_plan_t plan, const letkf_io* io, int32_t n_io, void* hip_stream) {
  if (!plan || !io || n_io < 0) return LETKF_EINVAL;
  for (int i = 0; i < n_io; ++i) {
    const int rc = check_io(plan, io[i]);
    if (rc != LETKF_OK) return rc;
  }
  int expect = 0;
  if (!plan->busy.compare_exchange_strong(expect, 1)) return LETKF_EBUSY;
  DeviceGuard guard(plan->device);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int rc = LETKF_OK;
  for (int i = 0; i < n_io && rc == LETKF_OK; ++i)
    rc = enqueue_analysis(plan, io[i], s, plan->timing && i == 0, io[i].xb);
  plan->last_stream = s;
  plan->busy.store(0);
  return rc;
}

int letkf_cycle(letkf_plan_t plan, const letkf_cycle_io* io, int32_t n_io, void* hip_stream) {
  if (!plan || !io || n_io < 0) return LETKF_EINVAL;
  for (int i = 0; i < n_io; ++i) {
    const int rc = check_io(plan, io[i].io);
    if (rc != LETKF_OK) return rc;
    if (io[i].io.xa != io[i].io.xb || io[i].n_steps < 0) return LETKF_EINVAL;
    if (!(io[i].tau > 0.5) || !std::isfinite(io[i].tau) || !std::isfinite(io[i].force_amp))
      return LETKF_EINVAL;
    if (io[i].n_steps > 0 && !plan->probs[io[i].io.problem].bgk) return LETKF_EINVAL;
  }
  int expect = 0;
  if (!plan->busy.compare_exchange_strong(expect, 1)) return LETKF_EBUSY;
  DeviceGuard guard(plan->device);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int rc = LETKF_OK;
  for (int i = 0; i < n_io && rc == LETKF_OK; ++i) {
    const letkf_cycle_io& c = io[i];
    ProblemWs& w = plan->probs[c.io.problem];
    // ping-pong between the caller's ensemble and the plan's buffer
    double* cur = const_cast<double*>(c.io.xb);
    double* nxt = w.bgk;
    for (int st = 0; st < c.n_steps && rc == LETKF_OK; ++st) {
      if (launch_bgk(cur, nxt, w.p.k, w.p.nx, w.p.ny, c.tau, c.force_amp, c.force_kx, s) !=
          hipSuccess)
        rc = LETKF_EDEVICE;
      double* t = cur;
      cur = nxt;
      nxt = t;
    }
    if (rc == LETKF_OK) rc = enqueue_analysis(plan, c.io, s, plan->timing && i == 0, cur);
  }
  plan->last_stream = s;
  plan->busy.store(0);
  return rc;
}

int letkf_status(letkf_plan_t plan, int32_t sync) {
  if (!plan) return LETKF_EINVAL;
  DeviceGuard guard(plan->device);
  if (sync && hipStreamSynchronize(plan->last_stream) != hipSuccess) return LETKF_EDEVICE;
  int bits = 0;
  if (hipMemcpy(&bits, plan->stat + 1, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return LETKF_EDEVICE;
  if (bits && hipMemset(plan->stat + 1, 0, sizeof(int)) != hipSuccess) return LETKF_EDEVICE;
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
  double acc[LETKF_N_PHASES] = {0, 0, 0, 0, 0, 0};
  int last_chunks = 0;
  const int calls = plan->recorded;
  for (int c = 0; c < calls; ++c) {
    const int slot = (plan->next_slot - 1 - c + 2 * letkf_plan_s::kSlots) % letkf_plan_s::kSlots;
    const hipEvent_t* ev = &plan->ev[(size_t)slot * plan->nev];
    const int nch = plan->slot_chunks[slot];
    last_chunks = nch;
    float t = 0.f;
    auto el = [&](int a, int b) -> double {
      return hipEventElapsedTime(&t, ev[a], ev[b]) == hipSuccess ? (double)t : 0.0;
    };
    acc[LETKF_PHASE_BIN] += el(0, 1);
    acc[LETKF_PHASE_TRANSPOSE] += el(1, 2);
    acc[LETKF_PHASE_OBSOP] += el(2, 3);
    int prev = 3;
    for (int ci = 0; ci < nch; ++ci) {
      acc[LETKF_PHASE_GRAM] += el(prev, 4 + 2 * ci);
      acc[LETKF_PHASE_EVD] += el(4 + 2 * ci, 5 + 2 * ci);
      prev = 5 + 2 * ci;
    }
    acc[LETKF_PHASE_UNTRANS] += el(prev, 4 + 2 * nch);
  }
  const int bin_launches = 5;  // two fills, count, scan, scatter/sort share the phase
  const int per_call[LETKF_N_PHASES] = {bin_launches, 1, 1, last_chunks, last_chunks, 1};
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
  EvdArgs ea{};
  ea.mode = 1;
  ea.k = k;
  ea.npt = batch;
  ea.tol2 = kJacobiTol2;
  ea.max_sweeps = kJacobiMaxSweeps;
  ea.A = a;
  ea.lam = lam;
  ea.vec = vec;
  ea.status = status;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int kp = pow2_at_least16(k);
  hipError_t e = hipErrorInvalidValue;
  if (kp == 16) e = launch_evd_kp<16>(ea, s);
  else if (kp == 32) e = launch_evd_kp<32>(ea, s);
  else if (kp == 64) e = launch_evd_kp<64>(ea, s);
  return e == hipSuccess ? LETKF_OK : LETKF_EDEVICE;
}

}  // extern "C"
