// Device-side constants, the kernel parameter block and small float64 /
// fixed-point helpers shared by the log-polar kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "fft.hpp"
#include "plan.hpp"

namespace hrt {

constexpr int kNtBand = 512;        // threads of the band kernels
constexpr int kNtCol = 256;         // threads of the column kernel
constexpr int kAbsMaxBlocks = 256;  // partial maxima of the input
constexpr int kXcds = 8;            // MI355X: workgroups go round-robin to 8 XCDs

// Everything the kernels need about one plan (passed by value).
struct DevGeo {
  int nt, nx, ntau, nq;
  double dt, x0, dx, tau0, dtau, T, X;
  double a, O1, O2, ca, sa;
  double inv_dtheta, inv_drho, drho, ctheta, crho;
  double wconst;  // 2 a^2 (dt/T)(dx/X): smear weight without t^, trapezoid, 1/|p|
  int Mt, Mr, K1, K2, u0, u1, R, nbands;
  int bands_per_xcd;  // ceil(nbands / kXcds)
  int grp1, grp3;     // FFT scratch sequences of the band kernels
  int xw0, W;         // angle columns [xw0, xw0 + W) that points can touch
  // LDS layout of the band kernels (byte offsets into the dynamic LDS)
  int k1_scratch, k1_anchor, k3_scratch, k3_anchor;
  float knorm;                  // 1/(Mt Mr): both inverse FFTs are unnormalised
  float wmax_data, wmax_radon;  // bounds on the smear weights of the two point sets
  const int* jmin;
  const double* qA;
  const double* qB;
  const int* q_i0;
  const float4* q_w;
  const float* q_scale;
};

// Band handled by this workgroup.  Workgroup i runs on XCD i % 8; giving
// consecutive bands to one XCD lets neighbouring bands, which read and write
// neighbouring samples, share that XCD's L2.  Returns -1 for the few padding
// workgroups of the last XCDs.
__device__ __forceinline__ int xcd_band(const DevGeo& G) {
  const int i = static_cast<int>(blockIdx.x);
  const int band = (i % kXcds) * G.bands_per_xcd + i / kXcds;
  return band < G.nbands ? band : -1;
}

// Cubic B-spline weights of taps i0-1 .. i0+2 for fractional offset f.
__device__ __forceinline__ void bspline4(float f, float w[4]) {
  const float g = 1.0f - f;
  w[0] = g * g * g * (1.0f / 6.0f);
  w[1] = 2.0f / 3.0f - f * f + 0.5f * f * f * f;
  w[2] = 2.0f / 3.0f - g * g + 0.5f * g * g * g;
  w[3] = f * f * f * (1.0f / 6.0f);
}

// The point anchors move to nearby samples by small increments; the two
// series below are exact to float64 rounding for increments up to kSeries.
constexpr double kSeries = 0.25;

// atan(z), |z| <= 0.25: Taylor series to z^31 (truncation < 1e-21 |z|).
__device__ __forceinline__ double atan_series(double z) {
  const double z2 = z * z;
  double p = -1.0 / 31.0;
#pragma unroll
  for (int n = 14; n >= 0; --n) {
    const double c = ((n & 1) ? -1.0 : 1.0) / (2 * n + 1);
    p = fma(p, z2, c);
  }
  return z * p;
}

// 1/d for d within 15 % of 1: hardware reciprocal and two Newton steps.
__device__ __forceinline__ double rcp_near1(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return r;
}

// log(1 + x), |x| <= 0.25, as 2 atanh(y), y = x / (2 + x) (|y| < 0.12),
// series to y^17 (truncation < 1e-19 |y|).
__device__ __forceinline__ double log1p_series(double x) {
  const double y = x * (0.5 * rcp_near1(1.0 + 0.5 * x));
  const double y2 = y * y;
  double p = 1.0 / 17.0;
#pragma unroll
  for (int n = 7; n >= 0; --n) p = fma(p, y2, 1.0 / (2 * n + 1));
  return 2.0 * y * p;
}

// atan(z) for any z: halve the angle, atan(z) = 2 atan(z / (1 + sqrt(1 + z^2))),
// until the series applies (no halving for the increments the walk meets).
__device__ __forceinline__ double atan_any(double z) {
  double m = 1.0;
  while (fabs(z) > kSeries) {
    z = z / (1.0 + sqrt(fma(z, z, 1.0)));
    m *= 2.0;
  }
  return m * atan_series(z);
}

// log(1 + x) for any x > -1: halve the logarithm,
// log1p(x) = 2 log1p(x / (1 + sqrt(1 + x))), until the series applies.
__device__ __forceinline__ double log1p_any(double x) {
  double m = 1.0;
  while (fabs(x) > kSeries) {
    x = x / (1.0 + sqrt(1.0 + x));
    m *= 2.0;
  }
  return m * log1p_series(x);
}

// round(v * scale) as a 64-bit integer for |v * scale| < 2^51: adding
// 1.5 * 2^52 leaves the rounded integer in the low mantissa bits.
__device__ __forceinline__ unsigned long long to_fixed(float v, double scale) {
  const double d = fma(static_cast<double>(v), scale, 6755399441055744.0);
  return static_cast<unsigned long long>(__double_as_longlong(d) - 0x4338000000000000ll);
}

// 64-bit two's complement fixed point back to float.
__device__ __forceinline__ float from_fixed(unsigned long long q, float inv_scale) {
  return static_cast<float>(static_cast<double>(static_cast<long long>(q))) * inv_scale;
}

}  // namespace hrt
