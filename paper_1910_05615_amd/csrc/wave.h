// Wave-wide scans and reductions on DPP (data movement inside the VALU, no
// LDS round trip), for 64-lane waves of CDNA (gfx9 DPP controls).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtd {

// A DPP move: lane i reads the lane CTRL names (row_shr, row_ror, row_bcast,
// wave_shr, ...) in the rows RM enables; lanes whose source is out of range
// or disabled read `ident`.  Scans below are Hillis-Steele within each row
// of 16 lanes (row_shr 1, 2, 4, 8), then the row totals carried across rows
// (row_bcast 15 and 31); every operation order is fixed, so the results are
// deterministic.
template <int CTRL, int RM>
__device__ inline int dpp_i(int v, int ident) {
  return __builtin_amdgcn_update_dpp(ident, v, CTRL, RM, 0xf, false);
}
template <int CTRL, int RM>
__device__ inline double dpp_d(double v, double ident) {
  const long long b = __double_as_longlong(v), o = __double_as_longlong(ident);
  const int lo = dpp_i<CTRL, RM>((int)b, (int)o);
  const int hi = dpp_i<CTRL, RM>((int)(b >> 32), (int)(o >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL, int RM>
__device__ inline int64_t dpp_l(int64_t v, int64_t ident) {
  const int lo = dpp_i<CTRL, RM>((int)v, (int)ident);
  const int hi = dpp_i<CTRL, RM>((int)(v >> 32), (int)(ident >> 32));
  return ((int64_t)hi << 32) | (int64_t)(unsigned)lo;
}

// inclusive prefix sum over the wave's 64 lanes
__device__ inline int wave_incl_sum(int x) {
  x += dpp_i<0x111, 0xf>(x, 0);
  x += dpp_i<0x112, 0xf>(x, 0);
  x += dpp_i<0x114, 0xf>(x, 0);
  x += dpp_i<0x118, 0xf>(x, 0);
  x += dpp_i<0x142, 0xa>(x, 0);
  x += dpp_i<0x143, 0xc>(x, 0);
  return x;
}
__device__ inline double wave_incl_sum(double x) {
  x += dpp_d<0x111, 0xf>(x, 0.0);
  x += dpp_d<0x112, 0xf>(x, 0.0);
  x += dpp_d<0x114, 0xf>(x, 0.0);
  x += dpp_d<0x118, 0xf>(x, 0.0);
  x += dpp_d<0x142, 0xa>(x, 0.0);
  x += dpp_d<0x143, 0xc>(x, 0.0);
  return x;
}
// sum over the wave, in every lane
__device__ inline double wave_sum(double x) {
  const double t = wave_incl_sum(x);
  const long long b = __double_as_longlong(t);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// a value that is the same in every lane, as a wave-uniform (scalar) value
__device__ inline double uniform_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)b);
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// lane l's value in every lane (l uniform over the wave)
__device__ inline double lane_bcast_d(double v, int l) {
  const int sl = __builtin_amdgcn_readfirstlane(l);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, sl);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), sl);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ inline int64_t lane_bcast_l(int64_t v, int l) {
  const int sl = __builtin_amdgcn_readfirstlane(l);
  const int lo = __builtin_amdgcn_readlane((int)v, sl);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), sl);
  return ((int64_t)hi << 32) | (int64_t)(unsigned)lo;
}

// (value, index) with the smallest value, ties to the smallest index; index
// -1 marks "none".  The result is valid in every lane.
__device__ inline bool argmin_takes(double b2, int64_t j2, double b, int64_t j) {
  return j2 >= 0 && (j < 0 || b2 < b || (b2 == b && j2 < j));
}
template <int CTRL, int RM>
__device__ inline void argmin_step(double& b, int64_t& j) {
  const double b2 = dpp_d<CTRL, RM>(b, INFINITY);
  const int64_t j2 = dpp_l<CTRL, RM>(j, -1);
  if (argmin_takes(b2, j2, b, j)) {
    b = b2;
    j = j2;
  }
}
__device__ inline void wave_argmin(double& b, int64_t& j) {
  argmin_step<0x111, 0xf>(b, j);
  argmin_step<0x112, 0xf>(b, j);
  argmin_step<0x114, 0xf>(b, j);
  argmin_step<0x118, 0xf>(b, j);
  argmin_step<0x142, 0xa>(b, j);
  argmin_step<0x143, 0xc>(b, j);
  const long long bb = __double_as_longlong(b);
  const int blo = __builtin_amdgcn_readlane((int)bb, 63);
  const int bhi = __builtin_amdgcn_readlane((int)(bb >> 32), 63);
  b = __longlong_as_double(((long long)bhi << 32) | (long long)(unsigned)blo);
  const int jlo = __builtin_amdgcn_readlane((int)j, 63);
  const int jhi = __builtin_amdgcn_readlane((int)(j >> 32), 63);
  j = ((int64_t)jhi << 32) | (int64_t)(unsigned)jlo;
}

// unsigned minimum / maximum over the wave, in every lane
__device__ inline uint32_t wave_min_u32(uint32_t x) {
  x = min(x, (uint32_t)dpp_i<0x111, 0xf>((int)x, -1));
  x = min(x, (uint32_t)dpp_i<0x112, 0xf>((int)x, -1));
  x = min(x, (uint32_t)dpp_i<0x114, 0xf>((int)x, -1));
  x = min(x, (uint32_t)dpp_i<0x118, 0xf>((int)x, -1));
  x = min(x, (uint32_t)dpp_i<0x142, 0xa>((int)x, -1));
  x = min(x, (uint32_t)dpp_i<0x143, 0xc>((int)x, -1));
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}
__device__ inline uint32_t wave_max_u32(uint32_t x) {
  x = max(x, (uint32_t)dpp_i<0x111, 0xf>((int)x, 0));
  x = max(x, (uint32_t)dpp_i<0x112, 0xf>((int)x, 0));
  x = max(x, (uint32_t)dpp_i<0x114, 0xf>((int)x, 0));
  x = max(x, (uint32_t)dpp_i<0x118, 0xf>((int)x, 0));
  x = max(x, (uint32_t)dpp_i<0x142, 0xa>((int)x, 0));
  x = max(x, (uint32_t)dpp_i<0x143, 0xc>((int)x, 0));
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// maximum over the wave, in every lane
__device__ inline double wave_max(double x) {
  x = fmax(x, dpp_d<0x111, 0xf>(x, -INFINITY));
  x = fmax(x, dpp_d<0x112, 0xf>(x, -INFINITY));
  x = fmax(x, dpp_d<0x114, 0xf>(x, -INFINITY));
  x = fmax(x, dpp_d<0x118, 0xf>(x, -INFINITY));
  x = fmax(x, dpp_d<0x142, 0xa>(x, -INFINITY));
  x = fmax(x, dpp_d<0x143, 0xc>(x, -INFINITY));
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// sum over each row of 16 lanes, in every lane of the row (rotations by 8,
// 4, 2, 1 within the row)
__device__ inline double row16_sum(double x) {
  x += dpp_d<0x128, 0xf>(x, 0.0);
  x += dpp_d<0x124, 0xf>(x, 0.0);
  x += dpp_d<0x122, 0xf>(x, 0.0);
  x += dpp_d<0x121, 0xf>(x, 0.0);
  return x;
}

}  // namespace rtd
