// Elementary functions for the pair kernels, written for gfx950.
//
// FP64:
//   exp_neg(x), x <= 0: Cody-Waite reduction x = k ln2 + r (|r| <= ln2/2,
//     ln2 split into a 32-bit head and a tail so k*head is exact), e^r by its
//     Taylor polynomial to degree 13 (truncation < 4e-18), times 2^k built
//     directly in the exponent field.  About 1 ulp.
//   erfcx(y) = exp(y^2) erfc(y): piecewise polynomials (32 pieces on [0, 8],
//     degree 11, max relative error 2.2e-16; erfcx_table.inc), read from an
//     LDS copy of the table.  erfc(y) = exp_neg(-y^2) * erfcx(y), so the
//     Ewald kernels share one exponential between erfc and the B_n recursion.
//   rsqrt: hardware estimate refined by two Newton steps.
// FP32 (mixed precision): hardware exp2 and rsqrt, degree-6 erfcx pieces
//   (max relative error 1.0e-7).
#pragma once

#include <hip/hip_runtime.h>

#include "erfcx_table.inc"

namespace tk {

constexpr int kErfcxPieces = 32;

// LDS copies of the erfcx tables, one per workgroup (filled by erfcx_stage).
__device__ __forceinline__ double* erfcx_lds64() {
  __shared__ double t[kErfcxPieces * (kErfcxTab64Deg + 1)];
  return t;
}
__device__ __forceinline__ float* erfcx_lds32() {
  __shared__ float t[kErfcxPieces * (kErfcxTab32Deg + 1)];
  return t;
}

// The LDS copy is coefficient-major (t[k * 32 + piece]): lanes on different
// pieces read different banks.
// The FP32 kernels also stage the FP64 table: their same-molecule pairs take
// the FP64 path.
template <class R>
__device__ __forceinline__ void erfcx_stage(int lane, int nthreads) {
  {
    double* t = erfcx_lds64();
    for (int e = lane; e < kErfcxPieces * (kErfcxTab64Deg + 1); e += nthreads) {
      const int j = e / (kErfcxTab64Deg + 1), k = e - j * (kErfcxTab64Deg + 1);
      t[k * kErfcxPieces + j] = kErfcxTab64[e];
    }
  }
  if (sizeof(R) == 4) {
    float* t = erfcx_lds32();
    for (int e = lane; e < kErfcxPieces * (kErfcxTab32Deg + 1); e += nthreads) {
      const int j = e / (kErfcxTab32Deg + 1), k = e - j * (kErfcxTab32Deg + 1);
      t[k * kErfcxPieces + j] = kErfcxTab32[e];
    }
  }
}

__device__ __forceinline__ double exp_neg(double x) {
  x = fmax(x, -708.0);
  const double k = rint(x * 1.4426950408889634074);
  double r = fma(-k, 0x1.62e42fee00000p-1, x);
  r = fma(-k, 1.9082149292705877e-10, r);
  double p = 1.6059043836821613e-10;
  p = fma(p, r, 2.08767569878681e-09);
  p = fma(p, r, 2.505210838544172e-08);
  p = fma(p, r, 2.755731922398589e-07);
  p = fma(p, r, 2.7557319223985893e-06);
  p = fma(p, r, 2.48015873015873e-05);
  p = fma(p, r, 0.0001984126984126984);
  p = fma(p, r, 0.001388888888888889);
  p = fma(p, r, 0.008333333333333333);
  p = fma(p, r, 0.041666666666666664);
  p = fma(p, r, 0.16666666666666666);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  const int ki = (int)k;   // in [-1022, 0]
  return p * __hiloint2double((ki + 1023) << 20, 0);
}

__device__ __forceinline__ float exp_neg(float x) { return __expf(x); }

// FP32 exp of an FP64 argument x <= 0: the reduction x = k ln2 + r runs in
// FP64 (so the rounding of a large argument is not amplified), 2^r in FP32.
__device__ __forceinline__ float exp_neg_f32_of(double x) {
  x = fmax(x, -87.0);
  const double k = rint(x * 1.4426950408889634074);
  double r = fma(-k, 0x1.62e42fee00000p-1, x);
  r = fma(-k, 1.9082149292705877e-10, r);
  return __expf((float)r) * __int_as_float(((int)k + 127) << 23);
}

__device__ __forceinline__ double erfcx(double y) {
  const double* t = erfcx_lds64();
  const double s = fmin(fmax(y, 0.0) * 4.0, 31.999999);
  const int j = (int)s;
  const double x = 2.0 * (s - (double)j) - 1.0;   // = 8 (y - y_mid)
  const double* c = t + j;
  double p = c[kErfcxTab64Deg * kErfcxPieces];
#pragma unroll
  for (int k = kErfcxTab64Deg - 1; k >= 0; --k) p = fma(p, x, c[k * kErfcxPieces]);
  return p;
}

__device__ __forceinline__ float erfcx(float y) {
  const float* t = erfcx_lds32();
  const float s = fminf(fmaxf(y, 0.0f) * 4.0f, 31.99998f);
  const int j = (int)s;
  const float x = 2.0f * (s - (float)j) - 1.0f;
  const float* c = t + j;
  float p = c[kErfcxTab32Deg * kErfcxPieces];
#pragma unroll
  for (int k = kErfcxTab32Deg - 1; k >= 0; --k) p = fmaf(p, x, c[k * kErfcxPieces]);
  return p;
}

__device__ __forceinline__ double rsqrt_r(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  y = y * fma(-0.5 * x * y, y, 1.5);
  return y;
}

__device__ __forceinline__ float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }

__device__ __forceinline__ double sqrt_r(double x) { return x * rsqrt_r(x); }
__device__ __forceinline__ float sqrt_r(float x) { return x * rsqrt_r(x); }

}  // namespace tk
