// Shared definitions of the HIP implementation (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/mak.h"

namespace mak {

constexpr int WAVE = 64;

// Error raised inside the host driver; converted to a status at the ABI.
struct Error {
  mak_status status;
  std::string msg;
};

#define MAK_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      throw ::mak::Error{MAK_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define MAK_FAIL(code, text) throw ::mak::Error{code, text}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- device side
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of set bits of `mask` below the calling lane.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ uint32_t readlane_u(uint32_t v, int l) {
  return uint32_t(__builtin_amdgcn_readlane(int(v), l));
}
__device__ __forceinline__ float readlane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double readlane_d(double v, int l) {
  const int64_t b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(int(uint32_t(b)), l);
  const int hi = __builtin_amdgcn_readlane(int(uint32_t(uint64_t(b) >> 32)), l);
  return __longlong_as_double(int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo)));
}
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
  const uint32_t lo = readlane_u(uint32_t(v), l);
  const uint32_t hi = readlane_u(uint32_t(v >> 32), l);
  return (uint64_t(hi) << 32) | lo;
}

// A value known to be equal on every lane, moved to a scalar register.
__device__ __forceinline__ float uniform_f(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Wave reductions (fixed order: deterministic).  Within each 16-lane row,
// DPP steps combine lane i with lane i^1 and i^2 (quad permutes), then with
// the mirrored lane of its half-row and of its row: every lane of a row then
// holds the row's result (bitwise equal across the row, the combining
// operations being commutative).  The four row results are read into
// scalars and combined in a fixed order, so the result is wave-uniform.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

template <int C>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, C, 0xF, 0xF, false);
}
template <int C>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(dpp_i<C>(__float_as_int(v)));
}
template <int C>
__device__ __forceinline__ double dpp_d(double v) {
  const uint64_t b = uint64_t(__double_as_longlong(v));
  const uint32_t lo = uint32_t(dpp_i<C>(int(uint32_t(b))));
  const uint32_t hi = uint32_t(dpp_i<C>(int(uint32_t(b >> 32))));
  return __longlong_as_double((long long)((uint64_t(hi) << 32) | lo));
}

__device__ __forceinline__ float wave_sum_f(float v) {
  v += dpp_f<kDppXor1>(v);
  v += dpp_f<kDppXor2>(v);
  v += dpp_f<kDppHalfMirror>(v);
  v += dpp_f<kDppMirror>(v);
  return (readlane_f(v, 0) + readlane_f(v, 16)) + (readlane_f(v, 32) + readlane_f(v, 48));
}
__device__ __forceinline__ float wave_max_f(float v) {
  v = fmaxf(v, dpp_f<kDppXor1>(v));
  v = fmaxf(v, dpp_f<kDppXor2>(v));
  v = fmaxf(v, dpp_f<kDppHalfMirror>(v));
  v = fmaxf(v, dpp_f<kDppMirror>(v));
  return fmaxf(fmaxf(readlane_f(v, 0), readlane_f(v, 16)), fmaxf(readlane_f(v, 32), readlane_f(v, 48)));
}
__device__ __forceinline__ double wave_sum_d(double v) {
  v += dpp_d<kDppXor1>(v);
  v += dpp_d<kDppXor2>(v);
  v += dpp_d<kDppHalfMirror>(v);
  v += dpp_d<kDppMirror>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}
__device__ __forceinline__ double wave_max_d(double v) {
  v = fmax(v, dpp_d<kDppXor1>(v));
  v = fmax(v, dpp_d<kDppXor2>(v));
  v = fmax(v, dpp_d<kDppHalfMirror>(v));
  v = fmax(v, dpp_d<kDppMirror>(v));
  return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}
__device__ __forceinline__ int wave_sum_i(int v) {
  v += dpp_i<kDppXor1>(v);
  v += dpp_i<kDppXor2>(v);
  v += dpp_i<kDppHalfMirror>(v);
  v += dpp_i<kDppMirror>(v);
  return (readlane_i(v, 0) + readlane_i(v, 16)) + (readlane_i(v, 32) + readlane_i(v, 48));
}
// Inclusive prefix sum over lanes.
__device__ __forceinline__ int wave_incl_scan_i(int v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int t = __shfl_up(v, o);
    if (l >= o) v += t;
  }
  return v;
}

// 1 / x in float64 for normal, finite x: the hardware reciprocal estimate
// refined by two Newton-Raphson steps r <- r + r (1 - x r), each of which
// roughly doubles the correct bits; the result is within a few ulps of the
// correctly rounded quotient (a vertex position needs no more).
__device__ __forceinline__ double recip_d(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// Order-preserving map of a float to uint32 (for sort keys).
__device__ __forceinline__ uint32_t float_key(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ int floor_div(int a, int b) {
  const int q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// Packed periodic image shift: three signed 10-bit fields.
__host__ __device__ __forceinline__ int32_t pack_shift(int sx, int sy, int sz) {
  return int32_t((uint32_t(sx & 1023) << 20) | (uint32_t(sy & 1023) << 10) | uint32_t(sz & 1023));
}
__host__ __device__ __forceinline__ int unpack_shift(int32_t p, int axis) {
  const int v = int((uint32_t(p) >> (20 - 10 * axis)) & 1023u);
  return v >= 512 ? v - 1024 : v;
}

}  // namespace mak
