// Element-wise kernels of the soft-thresholding iteration (Section 3, eqs.
// iters and itersmd), the float64 reductions of the power iteration that
// bounds its step size, and the Radon-domain mute of multiple attenuation
// (Section 6).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hrt {

constexpr int kVecThreads = 256;
constexpr int kDotBlocks = 1024;

// Data-domain residual of eq. itersmd, in place: r = f - chi_S r, where r
// holds R* g on entry and chi_S is `mask` (1 where a trace was recorded,
// 0 where it is missing; null means every sample was recorded).
__global__ __launch_bounds__(kVecThreads) void k_residual(const float* __restrict__ f,
                                                          const float* __restrict__ mask,
                                                          float* __restrict__ r, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride) {
    const float m = mask ? mask[i] : 1.0f;
    r[i] = f[i] - m * r[i];
  }
}

// Radon-domain update of eq. itersmd: g = S_{c^2 mu}(g + c^2 d), with the
// soft threshold S_mu(v) = v - mu/2 (v >= mu/2), 0 (|v| < mu/2),
// v + mu/2 (v <= -mu/2); `half_thr` = c^2 mu / 2.
__global__ __launch_bounds__(kVecThreads) void k_soft_update(float* __restrict__ g,
                                                             const float* __restrict__ d,
                                                             float c2, float half_thr,
                                                             int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride) {
    const float v = fmaf(c2, d[i], g[i]);
    g[i] = v >= half_thr ? v - half_thr : (v <= -half_thr ? v + half_thr : 0.0f);
  }
}

// The same update over the packed Radon panels of a batch: element i
// belongs to gather b with off[b] <= i < off[b+1] (found by bisection over
// the n + 1 offsets) and takes that gather's (c^2, c^2 mu / 2) = par[b].
__global__ __launch_bounds__(kVecThreads) void k_soft_update_batch(
    float* __restrict__ g, const float* __restrict__ d, const float2* __restrict__ par,
    const int64_t* __restrict__ off, int n) {
  const int64_t total = off[n];
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += stride) {
    int lo = 0, hi = n;  // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (off[mid] <= i) lo = mid;
      else hi = mid;
    }
    const float2 p = par[lo];
    const float v = fmaf(p.x, d[i], g[i]);
    g[i] = v >= p.y ? v - p.y : (v <= -p.y ? v + p.y : 0.0f);
  }
}

// kDotBlocks partial sums of a[i] * b[i] accumulated in float64.
__global__ __launch_bounds__(kVecThreads) void k_dot64(const float* __restrict__ a,
                                                       const float* __restrict__ b, int64_t n,
                                                       double* __restrict__ partial) {
  __shared__ double s[kVecThreads / 64];
  double acc = 0.0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride)
    acc = fma(static_cast<double>(a[i]), static_cast<double>(b[i]), acc);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kVecThreads / 64; ++w) t += s[w];
    partial[blockIdx.x] = t;
  }
}

// x = s * y (float32 vectors, float64 factor rounded once).
__global__ __launch_bounds__(kVecThreads) void k_scale(float* __restrict__ x,
                                                       const float* __restrict__ y, double s,
                                                       int64_t n) {
  const float sf = static_cast<float>(s);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride)
    x[i] = sf * y[i];
}

// Multiple attenuation (Section 6): keep the part of a Radon panel on the
// multiples' side of a border line in the (tau, q) plane, out[l][i] = g[l][i]
// where q_l > qb0 + qb_slope * tau_i, else 0.  The border decision is taken
// in float64 without contraction: q_l = q0 + l dq, tau_i = tau0 + i dtau.
__global__ __launch_bounds__(kVecThreads) void k_mute_multiples(
    const float* __restrict__ g, float* __restrict__ out, int ntau, int nq, double tau0,
    double dtau, double q0, double dq, double qb0, double qb_slope) {
  const int64_t n = static_cast<int64_t>(ntau) * nq;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < n;
       idx += stride) {
    const int l = static_cast<int>(idx / ntau);
    const int i = static_cast<int>(idx - static_cast<int64_t>(l) * ntau);
    const double q = __dadd_rn(q0, __dmul_rn(static_cast<double>(l), dq));
    const double tau = __dadd_rn(tau0, __dmul_rn(static_cast<double>(i), dtau));
    const double qb = __dadd_rn(qb0, __dmul_rn(qb_slope, tau));
    out[idx] = q > qb ? g[idx] : 0.0f;
  }
}

}  // namespace hrt
