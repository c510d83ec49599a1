// Device helpers shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

namespace fkf {

typedef double v2d __attribute__((ext_vector_type(2)));

// Sum over the 64 lanes of a wavefront (butterfly; every lane gets the sum).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

// Lane-to-lane move of a double by a DPP pattern; lanes of rows outside
// ROWS receive 0.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Largest of v over the 64 lanes (same DPP pattern as wave_sum_all).
__device__ __forceinline__ double wave_max_all(double v) {
  v = fmax(v, dpp_d<0xb1>(v));
  v = fmax(v, dpp_d<0x4e>(v));
  v = fmax(v, dpp_d<0x141>(v));
  v = fmax(v, dpp_d<0x140>(v));
  v = fmax(v, dpp_d<0x142, 0xa>(v));
  v = fmax(v, dpp_d<0x143, 0xc>(v));
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wavefront with DPP moves (pairs, quads, rows of
// 16 by mirrors, then row broadcasts; fixed order), returned to every lane
// from lane 63.  All 64 lanes must be active.
__device__ __forceinline__ double wave_sum_all(double v) {
  v += dpp_d<0xb1>(v);         // quad_perm [1,0,3,2]
  v += dpp_d<0x4e>(v);         // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);        // row_half_mirror
  v += dpp_d<0x140>(v);        // row_mirror
  v += dpp_d<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_d<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// exp(x) for x <= 0 (finite), used for Matern kernel entries.  Method: Cody &
// Waite argument reduction x = k ln2 + r with |r| <= ln2/2 (ln2 split into a
// 32-bit-exact high part and a low correction), a degree-12 Taylor polynomial
// for e^r (truncation error below 2e-16 relative on that interval), and an
// exact scaling by 2^k.  No NaN/overflow handling: callers pass x <= 0.
__device__ __forceinline__ double exp_nonpos(double x) {
  const double kLog2e = 1.4426950408889634074;
  const double kLn2Hi = 0.6931471803691238164902;       // ln 2 truncated to 32 significant bits
  const double kLn2Lo = 1.9082149292705877000e-10;      // ln 2 - kLn2Hi
  double k = rint(x * kLog2e);
  double r = fma(-k, kLn2Hi, x);
  r = fma(-k, kLn2Lo, r);
  double p = 1.0 / 479001600.0;                          // 1/12!
  p = fma(p, r, 1.0 / 39916800.0);
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return __builtin_amdgcn_ldexp(p, (int)k);
}

// sqrt(x) for x > 0 (finite, normal): hardware reciprocal square root refined
// by two Newton steps y <- y (3 - x y^2) / 2, then x * y.
__device__ __forceinline__ double sqrt_pos(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return x * y;
}

// 1/x for finite normal x != 0: hardware reciprocal refined by two Newton steps.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * fma(-x, r, 2.0);
  r = r * fma(-x, r, 2.0);
  return r;
}

// 1/sqrt(x) for finite x > 0: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

}  // namespace fkf
