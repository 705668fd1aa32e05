// Wavefront-level helpers shared by the per-walker kernels (wave64, DPP).
#pragma once

#include <hip/hip_runtime.h>

namespace mvmc {
namespace wave {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes: butterflies inside each row of 16 (quad_perm,
// half-row and row mirrors), then the row sums are carried up by the row
// broadcasts; lane 63 ends with the total, which is read back as a scalar.
__device__ __forceinline__ double wave_total(double v) {
  v += dpp_d<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v += dpp_d<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  v += dpp_d<0x141, 0xF>(v);   // row_half_mirror
  v += dpp_d<0x140, 0xF>(v);   // row_mirror
  v += dpp_d<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_d<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_keep(double v) {
  // lanes outside the row mask keep their own value
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), CTRL, ROWMASK,
                                             0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), CTRL, ROWMASK,
                                             0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_keep<0xB1, 0xF>(v));
  v = fmax(v, dpp_keep<0x4E, 0xF>(v));
  v = fmax(v, dpp_keep<0x141, 0xF>(v));
  v = fmax(v, dpp_keep<0x140, 0xF>(v));
  v = fmax(v, dpp_keep<0x142, 0xA>(v));
  v = fmax(v, dpp_keep<0x143, 0xC>(v));
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_keep_i(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, ROWMASK, 0xF, false);
}


template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint64_t dpp_keep_u64(uint64_t v) {
  const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
  const int nlo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWMASK, 0xF, false);
  const int nhi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWMASK, 0xF, false);
  return ((uint64_t)(uint32_t)nhi << 32) | (uint64_t)(uint32_t)nlo;
}
__device__ __forceinline__ uint64_t max_u64(uint64_t a, uint64_t b) { return a > b ? a : b; }
// Unsigned 64-bit maximum over the 64 lanes (same DPP pattern as wave_max).
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  v = max_u64(v, dpp_keep_u64<0xB1, 0xF>(v));
  v = max_u64(v, dpp_keep_u64<0x4E, 0xF>(v));
  v = max_u64(v, dpp_keep_u64<0x141, 0xF>(v));
  v = max_u64(v, dpp_keep_u64<0x140, 0xF>(v));
  v = max_u64(v, dpp_keep_u64<0x142, 0xA>(v));
  v = max_u64(v, dpp_keep_u64<0x143, 0xC>(v));
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}

// Partial-pivot search key of a candidate: the IEEE bits of |x| (ordered like
// the values for x >= 0) with the low six mantissa bits replaced by 63 - lane,
// so one maximum gives the largest magnitude (to 2^-46 relative) and, among
// those, the lowest lane.  Rows that may not be chosen take key 0.
__device__ __forceinline__ uint64_t pivot_key(double x, int lane, bool free_row) {
  const uint64_t b = (uint64_t)__double_as_longlong(fabs(x));
  return free_row ? ((b & ~(uint64_t)63) | (uint64_t)(63 - lane)) : 0;
}
__device__ __forceinline__ int pivot_lane(uint64_t key) { return 63 - (int)(key & 63); }
__device__ __forceinline__ double pivot_mag(uint64_t key) {
  return __longlong_as_double((long long)(key & ~(uint64_t)63));
}

// The same key from the high word of |x| alone (sign, exponent and 14
// mantissa bits, then 63 - lane): the pivot is within 2^-14 relative of the
// largest magnitude (threshold partial pivoting), and the maximum is six
// single-instruction DPP steps.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  v = max(v, (uint32_t)dpp_keep_i<0xB1, 0xF>((int)v));
  v = max(v, (uint32_t)dpp_keep_i<0x4E, 0xF>((int)v));
  v = max(v, (uint32_t)dpp_keep_i<0x141, 0xF>((int)v));
  v = max(v, (uint32_t)dpp_keep_i<0x140, 0xF>((int)v));
  v = max(v, (uint32_t)dpp_keep_i<0x142, 0xA>((int)v));
  v = max(v, (uint32_t)dpp_keep_i<0x143, 0xC>((int)v));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ uint32_t pivot_key32(double x, int lane, bool free_row) {
  const uint32_t hi = (uint32_t)__double2hiint(fabs(x));
  return free_row ? ((hi & ~63u) | (uint32_t)(63 - lane)) : 0u;
}
__device__ __forceinline__ int pivot_lane32(uint32_t key) { return 63 - (int)(key & 63u); }
__device__ __forceinline__ double pivot_mag32(uint32_t key) {
  return __hiloint2double((int)(key & ~63u), 0);
}

__device__ __forceinline__ int sgpr(int v) { return __builtin_amdgcn_readfirstlane(v); }

}  // namespace wave
}  // namespace mvmc
