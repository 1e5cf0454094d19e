// Host-side launchers of the gfx950 kernels and their argument blocks.
// Internal to the library; the public surface is include/letkf.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef LETKF_BATCH_RUN
#define LETKF_BATCH_RUN 32
#endif

namespace letkf {

// Observation binning (uniform cells of cb x cb lattice points) and the
// forecast-observation operator.
struct ObsArgs {
  int nx, ny, k, kq, npts;
  int n_obs;
  int cb, ncx, ncy, ncells;
  const int32_t* ix;
  const int32_t* iy;
  const int32_t* kind;
  const double* val;
  const double* var;
  int* obs_cell;    // [n_obs]   cell of each observation, -1 if invalid; after the
                    //           scatter, scratch for the ordering of the cells
  int* cell_count;  // [ncells]
  int* cell_start;  // [ncells + 1] exclusive scan; cell_start[ncells] = valid count
  int* cell_fill;   // [ncells]
  int* perm;        // [n_obs]   sorted slot -> observation index
  int* ox;          // [n_obs]   sorted slot -> lattice x
  int* oy;
  double* Yb;       // [n_obs][kq] FP64 forecast-observation perturbations (zero padded to KP)
  void* Ylp;        // the same rounded to FP32 (prec 1) or BF16 (prec 2), or null
  int prec;
  double* d;        // [n_obs] yo - ybar
  double* rinv;     // [n_obs] 1/sigma^2 (0 for an ignored observation)
  const double* xt; // point-major ensemble [npts][9][k]
  const double* xm; // or, when not null, the member-major ensemble [k][9][npts] read
                    // directly (the fused form, which needs no point-major copy)
  int* abort_flag;
  int* status;
};

// Localized Gram matrix C = dY^T R_loc^-1 dY and b = dY^T R_loc^-1 d per point.
struct GramArgs {
  int nx, ny, k;
  int pt0, npt;       // this launch covers points [pt0, pt0 + npt)
  int cb, ncx, ncy;
  int R;              // window radius in lattice units; < 0 means every cell
  int loc;            // LETKF_LOC_*
  double cut2;        // r^2 cutoff (inclusive for the Gaussian)
  double inv2L2;      // 1 / (2 L^2)
  double invL;        // 1 / L   (Gaspari-Cohn)
  const int* cell_start;
  const int* ox;
  const int* oy;
  const double* Yb;
  const void* Ylp;    // reduced-precision perturbations (k_gram_lp)
  const double* d;
  const double* rinv;
  double* C;          // [npt][NB][256] upper 16x16 blocks of C
  double* b;          // [npt][KP]
  const int* abort_flag;
};

// Eigensolve of Q = alpha I + C, transform and in-place update of the
// point-major ensemble (mode 0), or a standalone batched eigensolve (mode 1).
struct EvdArgs {
  int mode;
  int prec;           // contractions of the transform: 0 FP64, 1 FP32, 2 BF16 (FP32 accumulation)
  int k, npts;
  int pt0, npt;       // mode 0: points [pt0, pt0 + npt); mode 1: npt matrices
  double alpha;       // (k - 1) / rho
  double sqrt_km1;    // sqrt(k - 1)
  double defl_eps;    // unit roundoff behind the deflation tolerance of the divide and conquer
  double* C;          // [npt][NB][256] upper 16x16 blocks of C (KP-padded); reused as
                      // scratch for the Householder reflectors once staged
  const double* b;    // [npt][KP]
  double* xt;         // point-major ensemble [npts][9][k], updated in place
  const double* const* xio;  // fused form: {xb, xa} of the current call, member-major
                             // [k][9][npts] (the plan's pointer table, set per call); null:
                             // the point-major xt
  const double* A;    // mode 1: [npt][k][k]
  double* lam;        // mode 1: [npt][k]
  double* vec;        // mode 1: [npt][k][k]
  const int* abort_flag;
  int* status;
};

// A launch of the Gram or eigensolve kernels over a slab of points taken from
// the concatenated point lists of several problems (one problem is a table
// of one).  Descriptors live in device memory; C and b of the slab are
// indexed by the slab-local point.
struct BatchMap {
  const GramArgs* g;   // [nprob]; null: one problem described by g_inline
  const EvdArgs* e;    // [nprob]; null: one problem described by e_inline
  const int* prefix;   // [nprob + 1] first global point of each problem; null: {0}
  int nprob;
  int g0, n;           // slab: global points [g0, g0 + n)
  double* C;           // [n][NB][256]
  double* b;           // [n][KP]
  int* queue;          // [kQueueSlots] work counters of the persistent launches
  GramArgs g_inline;
  EvdArgs e_inline;
};

// Work queues of a persistent launch: one counter per XCD (blocks are
// dispatched round-robin over the 8 XCDs), each over a contiguous eighth of
// the slab; a wavefront that drains its own moves on to the next XCD's.
constexpr int kQueueSlots = 8;
// Blocks (of 4 points) per XCD run when a Gram launch covers several problems.
constexpr int kBatchRun = LETKF_BATCH_RUN;
constexpr int kPersistentBlocksPerCu = 8;
constexpr int kDeviceCus = 256;

inline int persistent_blocks(int n, int per_block) {
  const int full = kDeviceCus * kPersistentBlocksPerCu;
  const int need = (n + per_block - 1) / per_block;
  return need < full ? need : full;
}

// Items [0, n) handed to the launch's wavefronts through the queues: f(item)
// once per item, each on one wavefront (wave-uniform).
template <class F>
__device__ __forceinline__ void for_each_queued(int* queue, int n, F&& f) {
  const int home = blockIdx.x & (kQueueSlots - 1);
  for (int qi = 0; qi < kQueueSlots; ++qi) {
    const int q = (home + qi) & (kQueueSlots - 1);
    const int lo = (int)((int64_t)n * q / kQueueSlots);
    const int hi = (int)((int64_t)n * (q + 1) / kQueueSlots);
    for (;;) {
      int off = 0;
      if (__lane_id() == 0) off = atomicAdd(queue + q, 1);
      off = __builtin_amdgcn_readfirstlane(off);
      if (lo + off >= hi) break;             // wave-uniform exit
      f(lo + off);
    }
  }
}

template <class F>
__device__ __forceinline__ void for_each_queued_point(const BatchMap& bm, F&& f) {
  for_each_queued(bm.queue, bm.n, f);
}

// Slab-local point pl's Gram outputs: its NB upper 16 x 16 blocks of C and
// its KP entries of b (KP = 16, 32 or 64).
__device__ __forceinline__ double* gram_c(const BatchMap& bm, int pl, int kp) {
  const int nq = kp / 16;
  return bm.C + (size_t)pl * (nq * (nq + 1) / 2) * 256;
}
__device__ __forceinline__ double* gram_b(const BatchMap& bm, int pl, int kp) {
  return bm.b + (size_t)pl * kp;
}

// Position of entry (i, j), i <= j, of a KP x KP symmetric matrix stored as
// its packed upper triangle, row by row.
__host__ __device__ constexpr int packed_upper(int i, int j, int kp) {
  return i * kp - i * (i - 1) / 2 + (j - i);
}

// Writes the upper 16 x 16 blocks of a Gram matrix from MFMA accumulators:
// acc(b, r) is element r of block b's accumulator (blocks (I, J), I <= J, in
// row-major order), holding entry (row(r), col) of the block.  PACKED false:
// the blocks as they are, 256 entries each (global memory); PACKED true: the
// packed upper triangle of the KP x KP matrix (the fused kernel's LDS).
template <int KP, bool PACKED, class Acc, class Row>
__device__ __forceinline__ void store_gram_blocks(double* Cp, Acc acc, Row row, int col) {
  constexpr int NQ = KP / 16;
  int b = 0;
#pragma unroll
  for (int I = 0; I < NQ; ++I) {
#pragma unroll
    for (int J = I; J < NQ; ++J, ++b) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = row(r);
        if constexpr (PACKED) {
          const int i = 16 * I + rr, j = 16 * J + col;
          auto* lds = (__attribute__((address_space(3))) double*)Cp;
          if (I < J || rr <= col) lds[packed_upper(i, j, KP)] = acc(b, r);
        } else {
          Cp[b * 256 + rr * 16 + col] = acc(b, r);
        }
      }
    }
  }
}

__device__ __forceinline__ int find_problem(const int* prefix, int nprob, int gidx) {
  int lo = 0, hi = nprob;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= gidx) lo = mid; else hi = mid;
  }
  return lo;
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

// evd_args_of for a point that a whole wavefront works on (pl uniform): the
// same descriptor, read into scalar registers, so that the eigensolve's
// vector registers are not spent on it.
__device__ __forceinline__ EvdArgs evd_args_uniform(const BatchMap& bm, int pl, bool& valid) {
  valid = pl < bm.n;
  const int gidx = bm.g0 + (valid ? pl : 0);
  const int prob =
      bm.prefix ? __builtin_amdgcn_readfirstlane(find_problem(bm.prefix, bm.nprob, gidx)) : 0;
  EvdArgs e = bm.e ? uniform_copy(bm.e + prob) : bm.e_inline;
  e.C = bm.C;
  e.b = bm.b;
  e.pt0 = gidx - (bm.prefix ? __builtin_amdgcn_readfirstlane(bm.prefix[prob]) : 0) -
          (valid ? pl : 0);
  if (e.abort_flag && __builtin_amdgcn_readfirstlane(*e.abort_flag)) valid = false;
  return e;
}

// --- launchers (return hipError_t of the launch) ---
hipError_t launch_fill_i32(int* p, int n, int v, hipStream_t s);
// Up to kPtrBatch (slot, xb, xa) entries of a plan's pointer table, written
// by a kernel (so that a captured call replays them).
constexpr int kPtrBatch = 16;
struct PtrBatch {
  const double* xb[kPtrBatch];
  double* xa[kPtrBatch];
  int slot[kPtrBatch];
  int n;
};
hipError_t launch_store_ptrs(const double** table, const PtrBatch& b, hipStream_t s);
hipError_t launch_clear_bits(int* p, int bits, hipStream_t s);
hipError_t launch_bin(const ObsArgs& a, hipStream_t s);
hipError_t launch_transpose_in(const double* xb, double* xt, int k, int npts, const int* abort_flag,
                               hipStream_t s);
hipError_t launch_transpose_out(const double* xt, double* xa, int k, int npts,
                                const int* abort_flag, hipStream_t s);
hipError_t launch_obs_operator(const ObsArgs& a, hipStream_t s);
hipError_t launch_gram_f64(const BatchMap& bm, int kp, bool persistent, hipStream_t s);
hipError_t launch_gram_lp(const BatchMap& bm, int kp, int prec, bool persistent, hipStream_t s);
template <int KP>
hipError_t launch_evd_kp(const BatchMap& bm, hipStream_t s);
template <int KP>
hipError_t launch_evd_xf_kp(const BatchMap& bm, hipStream_t s);
hipError_t launch_nsqrt(const double* a, int batch, int k, double* x, int* status, int* steps,
                        hipStream_t s);
hipError_t launch_nsqrt_xf(const BatchMap& bm, int kp, hipStream_t s);
// The fused form: Gram, eigensolve, transform and update of every point of
// bm (g0 = 0, n = all points of its problems) in one persistent launch whose
// blocks keep each point's C and b in their own slot of bm.C / bm.b
// (fused_slot_c / fused_slot_b doubles per block).
constexpr int kFusedBlocks = kDeviceCus * 8;
template <int KP>
hipError_t launch_fused_kp(const BatchMap& bm, int prec, hipStream_t s);
// C and b doubles of one block's slot in the fused form (64 / kp points).
__host__ __device__ constexpr uint64_t fused_slot_c(int kp) {
  return (uint64_t)(64 / kp) * ((kp / 16) * (kp / 16 + 1) / 2) * 256;
}
__host__ __device__ constexpr uint64_t fused_slot_b(int kp) { return (uint64_t)(64 / kp) * kp; }
hipError_t launch_bgk(const double* fin, double* fout, int k, int nx, int ny, double tau, double amp,
                      int force_kx, hipStream_t s);

inline int pow2_at_least16(int k) {
  int p = 16;
  while (p < k) p <<= 1;
  return p;
}
inline int n_upper_blocks(int kp) {
  const int q = kp / 16;
  return q * (q + 1) / 2;
}

}  // namespace letkf
