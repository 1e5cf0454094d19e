// Device-side helpers shared by the gfx950 kernels of the LETKF library.
// Wavefront size is 64 throughout; every kernel is written for CDNA4.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace letkf {

constexpr int kWave = 64;

// D2Q9 directions in the library's order (see include/letkf.h):
// (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1)
__host__ __device__ constexpr int cx_of(int i) {
  return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0);
}
__host__ __device__ constexpr int cy_of(int i) {
  return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0);
}

// Status bits kept in the plan's device status word (bit n <-> error code n).
constexpr int kStatEinval = 1 << 1;
constexpr int kStatNonfinite = 1 << 5;
constexpr int kStatNotconv = 1 << 6;

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// The lane's index in its wavefront.  A translation unit that defines
// LETKF_OPAQUE_LANE before its includes gets it as a fresh value at every
// call (an empty asm), so that nothing computed from it can be hoisted out
// of a loop (the fused persistent kernel's item loop: hoisted per-lane
// addresses of the loop body would stay live through all of it).
__device__ __forceinline__ int lane_id() {
  int l = (int)__lane_id();
#ifdef LETKF_OPAQUE_LANE
  asm volatile("" : "+v"(l));
#endif
  return l;
}

// *p copied into scalar registers (the fields are read per lane, then taken
// from the first lane): for a descriptor whose address is uniform but whose
// memory the compiler cannot prove unwritten (a kernel that also does
// atomics), so that it would otherwise keep every field in vector registers.
template <typename T>
__device__ __forceinline__ T uniform_copy(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "uniform_copy: size must be a multiple of 4");
  T out;
  const int* src = reinterpret_cast<const int*>(p);
  int* dst = reinterpret_cast<int*>(&out);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
  return out;
}

// p[i] read as global memory.  Pointers that arrive inside a descriptor are
// generic to the compiler, and a generic (flat) load counts against the LDS
// wait counter too, so a wait for an LDS read would also wait for it; a
// global load keeps the two streams apart.
template <typename T>
__device__ __forceinline__ T ldg(const T* p, size_t i) {
  return ((const __attribute__((address_space(1))) T*)p)[i];
}

// p[i] = v as a global store (counted by the vector-memory counter only; a
// flat store to a generic pointer also counts against the LDS one).
template <typename T>
__device__ __forceinline__ void stg(T* p, size_t i, T v) {
  ((__attribute__((address_space(1))) T*)p)[i] = v;
}

// Make LDS writes of this wavefront visible to its other lanes (and keep the
// compiler from moving LDS accesses across this point).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane exchange lane <-> lane ^ M for a 32-bit value.  Masks below 32 use the
// swizzle network (bitmask mode, within 32-lane halves); larger masks use
// ds_bpermute.
template <int M>
__device__ __forceinline__ int xor_lane_i32(int x) {
  static_assert(M > 0 && M < 64, "xor mask");
  if constexpr (M < 32) {
    return __builtin_amdgcn_ds_swizzle(x, (M << 10) | 0x1F);
  } else {
    return __builtin_amdgcn_ds_bpermute((lane_id() ^ M) << 2, x);
  }
}

template <int M>
__device__ __forceinline__ double xor_lane(double x) {
  const int lo = xor_lane_i32<M>(__double2loint(x));
  const int hi = xor_lane_i32<M>(__double2hiint(x));
  return __hiloint2double(hi, lo);
}

// Value of x from the lane that a DPP pattern selects within each row of 16
// lanes (CDNA data-parallel primitives: a VALU move, no LDS round trip).
// Every pattern below writes every lane, so the move needs no prior value
// in its destination (mov_dpp rather than update_dpp, which would cost an
// extra move to initialize it).
//   0xB1 quad_perm [1,0,3,2]  (lane ^ 1)       0x4E quad_perm [2,3,0,1]  (lane ^ 2)
//   0x141 row_half_mirror     (i <-> 7 - i)    0x140 row_mirror         (i <-> 15 - i)
template <int CTRL>
__device__ __forceinline__ double dpp_lane(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// The values of lanes l and l ^ W (W = 16 or 32) as a pair (a, b), in an
// order that is the same on both lanes: v_permlane16_swap / v_permlane32_swap
// (CDNA4) on two copies of x exchange the odd 16-lane rows (upper 32-lane
// half) of one with the even rows (lower half) of the other, so one result
// holds the lower row's value and the other the upper row's on every lane of
// the pair.  A VALU exchange, with no LDS round trip.
template <int W>
__device__ __forceinline__ void row_pair(double x, double& a, double& b) {
  static_assert(W == 16 || W == 32, "row_pair: W is 16 or 32");
  const int lo = __double2loint(x), hi = __double2hiint(x);
  if constexpr (W == 16) {
    const auto rl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    a = __hiloint2double(rh[0], rl[0]);
    b = __hiloint2double(rh[1], rl[1]);
  } else {
    const auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    a = __hiloint2double(rh[0], rl[0]);
    b = __hiloint2double(rh[1], rl[1]);
  }
}

// Sum over aligned groups of G lanes (G a power of two <= 64).  Stages within
// 16 lanes use DPP, the wider ones the row swaps above.  Every stage combines
// the same two values on both lanes of a pair, and after each stage all
// lanes of a sub-group hold the same bits, so every lane of a group receives
// the bitwise-identical total.
template <int G>
__device__ __forceinline__ double group_sum(double x) {
  if constexpr (G >= 2) x += dpp_lane<0xB1>(x);
  if constexpr (G >= 4) x += dpp_lane<0x4E>(x);
  if constexpr (G >= 8) x += dpp_lane<0x141>(x);
  if constexpr (G >= 16) x += dpp_lane<0x140>(x);
  if constexpr (G >= 32) {
    double a, b;
    row_pair<16>(x, a, b);
    x = a + b;
  }
  if constexpr (G >= 64) {
    double a, b;
    row_pair<32>(x, a, b);
    x = a + b;
  }
  return x;
}

// Maximum over aligned groups of G lanes (every lane of a group gets it).
template <int G>
__device__ __forceinline__ double group_max(double x) {
  if constexpr (G >= 2) x = fmax(x, dpp_lane<0xB1>(x));
  if constexpr (G >= 4) x = fmax(x, dpp_lane<0x4E>(x));
  if constexpr (G >= 8) x = fmax(x, dpp_lane<0x141>(x));
  if constexpr (G >= 16) x = fmax(x, dpp_lane<0x140>(x));
  if constexpr (G >= 32) {
    double a, b;
    row_pair<16>(x, a, b);
    x = fmax(a, b);
  }
  if constexpr (G >= 64) {
    double a, b;
    row_pair<32>(x, a, b);
    x = fmax(a, b);
  }
  return x;
}

// Block index remap so that consecutive logical blocks land on the same XCD
// (blocks are dispatched round-robin over the 8 XCDs, each with its own L2).
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
  const int nb8 = nblocks >> 3, rem = nblocks & 7;
  const int xcd = b & 7, idx = b >> 3;
  return xcd < rem ? xcd * (nb8 + 1) + idx : rem * (nb8 + 1) + (xcd - rem) * nb8 + idx;
}

// Block index remap for a launch over several problems whose cost per point
// differs (observation density, localization length): runs of RUN
// consecutive logical blocks go to one XCD and successive runs to successive
// XCDs, so that every XCD gets a share of each problem (with xcd_remap a
// contiguous eighth of the launch, possibly a whole heavy problem, sits on
// one XCD and the launch waits for it), while the blocks of a run still
// share their XCD's L2.  Blocks past the last whole round of 8 runs keep
// their index.
template <int RUN>
__device__ __forceinline__ int xcd_remap_runs(int b, int nblocks) {
  const int full = nblocks / (8 * RUN) * (8 * RUN);
  if (b >= full) return b;
  const int xcd = b & 7, idx = b >> 3;
  return ((idx / RUN) * 8 + xcd) * RUN + idx % RUN;
}

__host__ __device__ constexpr int ceil_div(int a, int b) { return (a + b - 1) / b; }

// bfloat16 <-> float, round to nearest even (finite values).
__device__ __forceinline__ unsigned short to_bf16(float x) {
  const unsigned u = __float_as_uint(x);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h) {
  return __uint_as_float(((unsigned)h) << 16);
}
// Operand rounding of the reduced-precision forms: prec 1 = FP32, 2 = BF16.
__device__ __forceinline__ float round_operand(double x, int prec) {
  const float f = (float)x;
  return prec == 2 ? from_bf16(to_bf16(f)) : f;
}

}  // namespace letkf
