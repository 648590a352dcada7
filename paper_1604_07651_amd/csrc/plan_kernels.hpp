// Plan-time kernels: the kernel spectrum of eq. finiteconv by composite
// Gauss-Legendre quadrature in float64, as a product of two exponential
// tables.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hrt {

// ---------------------------------------------------- kernel spectrum (plan)

// E1[k1][n] = 2 w_n sec(theta_n) cos(2 pi k1 theta_n / P_theta),
// E2[n][k2] = exp(-2 pi i k2 ln cos(theta_n) / P_rho), nodes on [0, beta_k]
// (the integrand of eq. finiteconv's kernel spectrum is even in theta).
__global__ void k_zeta_tables(int N, int K1, int K2, const double* __restrict__ nodes,
                              const double* __restrict__ weights, double inv_pt,
                              double inv_pr, double* __restrict__ E1,
                              double2* __restrict__ E2) {
  const int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t n1 = static_cast<int64_t>(K1) * N;
  const int64_t n2 = static_cast<int64_t>(K2) * N;
  if (tid < n1) {
    const int k1 = static_cast<int>(tid / N);
    const int n = static_cast<int>(tid - static_cast<int64_t>(k1) * N);
    const double th = nodes[n];
    double x = static_cast<double>(k1) * th * inv_pt;
    x -= floor(x);
    E1[tid] = 2.0 * weights[n] / cos(th) * cospi(2.0 * x);
  } else if (tid < n1 + n2) {
    const int64_t t = tid - n1;
    const int n = static_cast<int>(t / K2);
    const int k2 = static_cast<int>(t - static_cast<int64_t>(n) * K2);
    double x = static_cast<double>(k2) * log(cos(nodes[n])) * inv_pr;
    x -= floor(x);
    double s, c;
    sincospi(2.0 * x, &s, &c);
    E2[t] = make_double2(c, -s);
  }
}

// K[k1][k2] = s1[k1] s2[k2] c * sum_n E1[k1][n] E2[n][k2] (float64, tiled)
__global__ __launch_bounds__(256) void k_zeta_gemm(int N, int K1, int K2,
                                                   const double* __restrict__ E1,
                                                   const double2* __restrict__ E2,
                                                   const double* __restrict__ s1,
                                                   const double* __restrict__ s2,
                                                   double c, float2* __restrict__ K) {
  constexpr int TB = 16, TN = 32;
  __shared__ double a[TB][TN + 1];
  __shared__ double2 b[TN][TB];
  const int tx = threadIdx.x % TB, ty = threadIdx.x / TB;
  const int k1 = blockIdx.y * TB + ty;
  const int k2 = blockIdx.x * TB + tx;
  double re = 0.0, im = 0.0;
  for (int n0 = 0; n0 < N; n0 += TN) {
    for (int i = threadIdx.x; i < TB * TN; i += 256) {
      const int r = i / TN, cc = i % TN;
      const int kk = blockIdx.y * TB + r;
      a[r][cc] = (kk < K1 && n0 + cc < N) ? E1[static_cast<int64_t>(kk) * N + n0 + cc] : 0.0;
      const int rr = i / TB, c2 = i % TB;
      const int kq = blockIdx.x * TB + c2;
      b[rr][c2] = (kq < K2 && n0 + rr < N) ? E2[static_cast<int64_t>(n0 + rr) * K2 + kq]
                                           : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 8
    for (int t = 0; t < TN; ++t) {
      re = fma(a[ty][t], b[t][tx].x, re);
      im = fma(a[ty][t], b[t][tx].y, im);
    }
    __syncthreads();
  }
  if (k1 < K1 && k2 < K2) {
    const double sc = s1[k1] * s2[k2] * c;
    K[static_cast<int64_t>(k1) * K2 + k2] =
        make_float2(static_cast<float>(re * sc), static_cast<float>(im * sc));
  }
}

}  // namespace hrt
