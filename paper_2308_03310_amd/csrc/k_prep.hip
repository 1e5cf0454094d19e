// Preparation kernels of one LETKF analysis on gfx950:
//  * observation validation and binning into uniform lattice cells (the
//    index that replaces the padded local-observation array Y_loc of
//    Sec. II-B step 2 / Algorithm 1 step 2);
//  * member-major <-> point-major transposes of the ensemble through LDS
//    (the data transposes of Sec. IV-A, done on one device);
//  * forecast observations Y^f = H(X^f), their mean and perturbations
//    (Sec. II-B step 1, eqs. enkf_ybar / enkf_deltay; moments of Sec. II-A).
#include "common.h"
#include "launch.h"

namespace letkf {

__global__ void k_fill_i32(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Clears the given bits of a status word (bits raised meanwhile survive).
__global__ void k_clear_bits(int* p, int bits) {
  if (threadIdx.x == 0) atomicAnd(p, ~bits);
}

// Validate each observation record and count it into its cell.
__global__ void k_obs_count(ObsArgs a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n_obs) return;
  const int x = a.ix[j], y = a.iy[j], kd = a.kind[j];
  const double var = a.var[j], val = a.val[j];
  const bool var_ok = var > 0.0;                 // false for NaN and <= 0; +inf allowed
  const bool ignored = var_ok && __builtin_isinf(var);
  const bool ok = x >= 0 && x < a.nx && y >= 0 && y < a.ny && kd >= 0 && kd <= 2 && var_ok &&
                  (ignored || __builtin_isfinite(val));
  if (!ok) {
    a.obs_cell[j] = -1;
    atomicOr(a.abort_flag, 1);
    atomicOr(a.status, kStatEinval);
    return;
  }
  const int c = (y / a.cb) * a.ncx + x / a.cb;
  a.obs_cell[j] = c;
  atomicAdd(&a.cell_count[c], 1);
}

// Exclusive scan of the cell counts by a single workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan(const int* count, int* start, int n) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int lo = t * per, hi = min(n, lo + per);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += count[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = t > 0 ? part[t - 1] : 0;
  for (int i = lo; i < hi; ++i) {
    start[i] = run;
    run += count[i];
  }
  if (t == 1023) start[n] = part[1023];
}

__global__ void k_obs_scatter(ObsArgs a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n_obs) return;
  const int c = a.obs_cell[j];
  if (c < 0) return;
  const int slot = a.cell_start[c] + atomicAdd(&a.cell_fill[c], 1);
  a.perm[slot] = j;
}

// Order each cell's observations by their index so that every later sum runs
// in an order fixed by the input alone (bitwise reproducible results): one
// thread per slot counts the smaller indices in its cell (its rank) and
// writes its observation there, into obs_cell (whose per-observation cells
// are no longer needed: the cell is recomputed from the coordinates).
__global__ void k_cell_rank(ObsArgs a) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.cell_start[a.ncells]) return;
  const int j = a.perm[s];
  const int c = (a.iy[j] / a.cb) * a.ncx + a.ix[j] / a.cb;
  const int lo = a.cell_start[c], hi = a.cell_start[c + 1];
  int rank = 0;
  for (int t = lo; t < hi; ++t) rank += a.perm[t] < j ? 1 : 0;
  a.obs_cell[lo + rank] = j;
}

__global__ void k_cell_copy(ObsArgs a) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < a.cell_start[a.ncells]) a.perm[s] = a.obs_cell[s];
}

// xb[k][9][npts] -> xt[npts][9][k]: one 64-point x (all members) tile of one
// direction per block, staged in LDS so both sides are coalesced.
__global__ __launch_bounds__(256) void k_transpose_in(const double* __restrict__ xb,
                                                      double* __restrict__ xt, int k, int npts,
                                                      const int* abort_flag) {
  if (*abort_flag) return;
  __shared__ double tile[64][65];
  const int p0 = blockIdx.x * 64, i = blockIdx.y;
  for (int e = threadIdx.x; e < k * 64; e += 256) {
    const int m = e >> 6, p = e & 63;
    if (p0 + p < npts) tile[p][m] = xb[((size_t)m * 9 + i) * npts + p0 + p];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < k * 64; e += 256) {
    const int p = e / k, m = e - p * k;
    if (p0 + p < npts) xt[((size_t)(p0 + p) * 9 + i) * k + m] = tile[p][m];
  }
}

// xt[npts][9][k] -> xa[k][9][npts]
__global__ __launch_bounds__(256) void k_transpose_out(const double* __restrict__ xt,
                                                       double* __restrict__ xa, int k, int npts,
                                                       const int* abort_flag) {
  if (*abort_flag) return;
  __shared__ double tile[64][65];
  const int p0 = blockIdx.x * 64, i = blockIdx.y;
  for (int e = threadIdx.x; e < k * 64; e += 256) {
    const int p = e / k, m = e - p * k;
    if (p0 + p < npts) tile[p][m] = xt[((size_t)(p0 + p) * 9 + i) * k + m];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < k * 64; e += 256) {
    const int m = e >> 6, p = e & 63;
    if (p0 + p < npts) xa[((size_t)m * 9 + i) * npts + p0 + p] = tile[p][m];
  }
}

// One wavefront per sorted observation slot, one lane per member: the
// member's moment at the observation point, the ensemble mean of the moments
// and the perturbations.
__global__ __launch_bounds__(256) void k_obs_operator(ObsArgs a) {
  if (*a.abort_flag) return;
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int m = lane_id();
  const int n_valid = a.cell_start[a.ncells];
  if (s >= n_valid) return;
  const int j = a.perm[s];
  const int x = a.ix[j], y = a.iy[j], kd = a.kind[j];
  const int pt = y * a.nx + x;
  double val = 0.0;
  if (m < a.k) {
    // point-major [pt][9][k], or member-major [k][9][npts] when xm is set
    const double* f = a.xm ? a.xm + (size_t)m * 9 * a.npts + pt : a.xt + (size_t)pt * 9 * a.k + m;
    const size_t si = a.xm ? (size_t)a.npts : (size_t)a.k;
    double fi[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) fi[i] = f[i * si];
    double rho = 0.0, ju = 0.0, jv = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      rho += fi[i];
      if (cx_of(i) != 0) ju += cx_of(i) > 0 ? fi[i] : -fi[i];
      if (cy_of(i) != 0) jv += cy_of(i) > 0 ? fi[i] : -fi[i];
    }
    val = kd == 0 ? rho : (kd == 1 ? ju / rho : jv / rho);
  }
  const double ybar = group_sum<64>(val) / (double)a.k;
  if (m < a.kq) {
    const double dy = m < a.k ? val - ybar : 0.0;   // rounded only after the FP64 subtraction
    if (a.Yb) a.Yb[(size_t)s * a.kq + m] = dy;
    if (a.prec == 1) reinterpret_cast<float*>(a.Ylp)[(size_t)s * a.kq + m] = (float)dy;
    if (a.prec == 2)
      reinterpret_cast<unsigned short*>(a.Ylp)[(size_t)s * a.kq + m] = to_bf16((float)dy);
  }
  if (m == 0) {
    const double var = a.var[j];
    a.d[s] = a.val[j] - ybar;
    a.rinv[s] = __builtin_isinf(var) ? 0.0 : 1.0 / var;
    a.ox[s] = x;
    a.oy[s] = y;
  }
}

__global__ void k_store_ptrs(const double** table, PtrBatch b) {
  const int i = threadIdx.x;
  if (i < b.n) {
    table[2 * b.slot[i]] = b.xb[i];
    table[2 * b.slot[i] + 1] = b.xa[i];
  }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_store_ptrs(const double** table, const PtrBatch& b, hipStream_t s) {
  if (b.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_store_ptrs, dim3(1), dim3(kPtrBatch), 0, s, table, b);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, int n, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(ceil_div(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_clear_bits(int* p, int bits, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_bits, dim3(1), dim3(64), 0, s, p, bits);
  return hipGetLastError();
}

hipError_t launch_bin(const ObsArgs& a, hipStream_t s) {
  hipError_t e;
  if ((e = launch_fill_i32(a.cell_count, a.ncells, 0, s)) != hipSuccess) return e;
  if ((e = launch_fill_i32(a.cell_fill, a.ncells, 0, s)) != hipSuccess) return e;
  if (a.n_obs > 0) {
    hipLaunchKernelGGL(k_obs_count, dim3(ceil_div(a.n_obs, 256)), dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, (const int*)a.cell_count, a.cell_start,
                     a.ncells);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (a.n_obs > 0) {
    hipLaunchKernelGGL(k_obs_scatter, dim3(ceil_div(a.n_obs, 256)), dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cell_rank, dim3(ceil_div(a.n_obs, 256)), dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cell_copy, dim3(ceil_div(a.n_obs, 256)), dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_transpose_in(const double* xb, double* xt, int k, int npts, const int* abort_flag,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_transpose_in, dim3(ceil_div(npts, 64), 9), dim3(256), 0, s, xb, xt, k, npts,
                     abort_flag);
  return hipGetLastError();
}

hipError_t launch_transpose_out(const double* xt, double* xa, int k, int npts,
                                const int* abort_flag, hipStream_t s) {
  hipLaunchKernelGGL(k_transpose_out, dim3(ceil_div(npts, 64), 9), dim3(256), 0, s, xt, xa, k, npts,
                     abort_flag);
  return hipGetLastError();
}

hipError_t launch_obs_operator(const ObsArgs& a, hipStream_t s) {
  if (a.n_obs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_obs_operator, dim3(ceil_div(a.n_obs, 4)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace letkf
