// One D2Q9 lattice-BGK step of every ensemble member (the lattice Boltzmann
// equation of Sec. II-A in collide-then-stream order), member-major in and
// out, periodic box, with a Kolmogorov body force F_x(y) = A sin(kappa y)
// added as the source 3 w_i (c_i . F) after relaxation.
//
// One thread per (member, lattice point): nine coalesced plane reads, the
// collision in registers, nine coalesced plane writes shifted by c_i (push).
// HBM-bound: 2 x 9 x 8 bytes per point and member.
#include "common.h"
#include "launch.h"

namespace letkf {

__global__ __launch_bounds__(256) void k_bgk(const double* __restrict__ fin, double* __restrict__ fout,
                                             int nx, int ny, double omega, double amp, double kappa) {
  const int npts = nx * ny;
  const int p = blockIdx.x * 256 + threadIdx.x;
  const int m = blockIdx.y;
  if (p >= npts) return;
  const int x = p % nx, y = p / nx;
  const double* src = fin + (size_t)m * 9 * npts + p;
  double f[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = src[(size_t)i * npts];
  double rho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    rho += f[i];
    if (cx_of(i) != 0) jx += cx_of(i) > 0 ? f[i] : -f[i];
    if (cy_of(i) != 0) jy += cy_of(i) > 0 ? f[i] : -f[i];
  }
  const double ux = jx / rho, uy = jy / rho;
  const double uu = ux * ux + uy * uy;
  const double fx = amp * sin(kappa * (double)y);
  double* dst = fout + (size_t)m * 9 * npts;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double w = i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    const double cu = cx_of(i) * ux + cy_of(i) * uy;
    const double feq = w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    const double post = f[i] - (f[i] - feq) * omega + 3.0 * w * cx_of(i) * fx;
    int xd = x + cx_of(i), yd = y + cy_of(i);
    xd = xd < 0 ? xd + nx : (xd >= nx ? xd - nx : xd);
    yd = yd < 0 ? yd + ny : (yd >= ny ? yd - ny : yd);
    dst[(size_t)i * npts + yd * nx + xd] = post;
  }
}

hipError_t launch_bgk(const double* fin, double* fout, int k, int nx, int ny, double tau, double amp,
                      int force_kx, hipStream_t s) {
  const int npts = nx * ny;
  const double kappa = 2.0 * 3.14159265358979323846 * (double)force_kx / (double)ny;
  hipLaunchKernelGGL(k_bgk, dim3(ceil_div(npts, 256), k), dim3(256), 0, s, fin, fout, nx, ny,
                     1.0 / tau, amp, kappa);
  return hipGetLastError();
}

}  // namespace letkf
