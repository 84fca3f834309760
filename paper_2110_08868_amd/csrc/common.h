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
// operations being commutative).  Two row broadcasts then fold row 0 into
// row 1 and row 2 into row 3 (lane 15 / lane 47 to the next row), and row 1
// into row 3 (lane 31 to rows 2 and 3): lane 63 holds
// (r3 op r2) op (r1 op r0), which by commutativity is bitwise
// (r0 op r1) op (r2 op r3), and is read into a scalar register.
// Every DPP move of the in-row steps has a valid source lane, so it is
// issued with bound_ctrl and no "old" operand, which lets the compiler fold
// it into the instruction that consumes it (one VALU instruction per step
// instead of three).  The lanes of the rows a broadcast does not write hold
// unspecified values afterwards; only lane 63 is read.
// Floats are maximised as order-preserving integers (no NaN operands
// occur): the integer max folds its DPP move, while fmaxf would first
// quiet each moved operand.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;
constexpr int kDppBcast15 = 0x142, kDppBcast31 = 0x143;

template <int C>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, C, 0xF, 0xF, true);
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
// Row broadcast into the rows of mask RM (other rows: unspecified).
template <int C, int RM>
__device__ __forceinline__ int bcast_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, C, RM, 0xF, false);
}
template <int C, int RM>
__device__ __forceinline__ float bcast_f(float v) {
  return __int_as_float(bcast_i<C, RM>(__float_as_int(v)));
}
template <int C, int RM>
__device__ __forceinline__ double bcast_d(double v) {
  const uint64_t b = uint64_t(__double_as_longlong(v));
  const uint32_t lo = uint32_t(bcast_i<C, RM>(int(uint32_t(b))));
  const uint32_t hi = uint32_t(bcast_i<C, RM>(int(uint32_t(b >> 32))));
  return __longlong_as_double((long long)((uint64_t(hi) << 32) | lo));
}
// float <-> int with the same order (an involution; -0 below +0)
__device__ __forceinline__ int float_ord(float f) {
  const int b = __float_as_int(f);
  return b ^ ((b >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float ord_float(int k) { return __int_as_float(k ^ ((k >> 31) & 0x7fffffff)); }

__device__ __forceinline__ float wave_sum_f(float v) {
  v += dpp_f<kDppXor1>(v);
  v += dpp_f<kDppXor2>(v);
  v += dpp_f<kDppHalfMirror>(v);
  v += dpp_f<kDppMirror>(v);
  v += bcast_f<kDppBcast15, 0xA>(v);
  v += bcast_f<kDppBcast31, 0xC>(v);
  return readlane_f(v, 63);
}
__device__ __forceinline__ int wave_max_i(int v) {
  v = max(v, dpp_i<kDppXor1>(v));
  v = max(v, dpp_i<kDppXor2>(v));
  v = max(v, dpp_i<kDppHalfMirror>(v));
  v = max(v, dpp_i<kDppMirror>(v));
  v = max(v, bcast_i<kDppBcast15, 0xA>(v));
  v = max(v, bcast_i<kDppBcast31, 0xC>(v));
  return readlane_i(v, 63);
}
__device__ __forceinline__ float wave_max_f(float v) { return ord_float(wave_max_i(float_ord(v))); }
__device__ __forceinline__ double wave_sum_d(double v) {
  v += dpp_d<kDppXor1>(v);
  v += dpp_d<kDppXor2>(v);
  v += dpp_d<kDppHalfMirror>(v);
  v += dpp_d<kDppMirror>(v);
  v += bcast_d<kDppBcast15, 0xA>(v);
  v += bcast_d<kDppBcast31, 0xC>(v);
  return readlane_d(v, 63);
}
__device__ __forceinline__ double wave_max_d(double v) {
  v = fmax(v, dpp_d<kDppXor1>(v));
  v = fmax(v, dpp_d<kDppXor2>(v));
  v = fmax(v, dpp_d<kDppHalfMirror>(v));
  v = fmax(v, dpp_d<kDppMirror>(v));
  v = fmax(v, bcast_d<kDppBcast15, 0xA>(v));
  v = fmax(v, bcast_d<kDppBcast31, 0xC>(v));
  return readlane_d(v, 63);
}
__device__ __forceinline__ int wave_sum_i(int v) {
  v += dpp_i<kDppXor1>(v);
  v += dpp_i<kDppXor2>(v);
  v += dpp_i<kDppHalfMirror>(v);
  v += dpp_i<kDppMirror>(v);
  v += bcast_i<kDppBcast15, 0xA>(v);
  v += bcast_i<kDppBcast31, 0xC>(v);
  return readlane_i(v, 63);
}
// Inclusive prefix sum over lanes: within each row, shifts by 1, 2, 4 and 8
// lanes (a lane whose source lies before its row reads 0: bound_ctrl), then
// row 0's total into row 1 and row 2's into row 3, then the total of rows 0
// and 1 into rows 2 and 3 (the rows a broadcast skips add 0).
constexpr int kDppShr1 = 0x111, kDppShr2 = 0x112, kDppShr4 = 0x114, kDppShr8 = 0x118;
__device__ __forceinline__ int wave_incl_scan_i(int v) {
  v += dpp_i<kDppShr1>(v);
  v += dpp_i<kDppShr2>(v);
  v += dpp_i<kDppShr4>(v);
  v += dpp_i<kDppShr8>(v);
  v += __builtin_amdgcn_update_dpp(0, v, kDppBcast15, 0xA, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0, v, kDppBcast31, 0xC, 0xF, false);
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
