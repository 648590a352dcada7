// The reference method of Section 5 on the GPU: direct summation over
// hyperbolas (eq. Rhdef) with Keys cubic interpolation in time and the
// trapezoid rule in offset, float32, and its exact transpose.
#pragma once

#include <hip/hip_runtime.h>

namespace hrt {

// ------------------------------------------------------ direct summation --

struct DirectGeo {
  int nt, nx, ntau, nq;
  float dt, inv_dt, x0, dx, tau0, dtau, q0, dq;
};

__device__ __forceinline__ float keys_near(float s) {  // |s| <= 1, a = -1/2
  return (1.5f * s - 2.5f) * s * s + 1.0f;
}
__device__ __forceinline__ float keys_far(float s) {   // 1 < |s| < 2
  return ((-0.5f * s + 2.5f) * s - 4.0f) * s + 2.0f;
}

// Hyperbola time in samples and the Keys weights of taps j0-1 .. j0+2; both
// directions call this so the adjoint is the exact transpose.
__device__ __forceinline__ float hyper_c(const DirectGeo& D, int i, int l, int k) {
  const float tau = D.tau0 + static_cast<float>(i) * D.dtau;
  const float qx = (D.q0 + static_cast<float>(l) * D.dq) *
                   (D.x0 + static_cast<float>(k) * D.dx);
  return sqrtf(tau * tau + qx * qx) * D.inv_dt;
}
__device__ __forceinline__ void keys4(float u, float w[4]) {
  w[0] = keys_far(1.0f + u);
  w[1] = keys_near(u);
  w[2] = keys_near(1.0f - u);
  w[3] = keys_far(2.0f - u);
}

__global__ __launch_bounds__(256) void k_direct_fwd(DirectGeo D,
                                                    const float* __restrict__ f,
                                                    float* __restrict__ g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (i >= D.ntau) return;
  float acc = 0.0f;
  for (int k = 0; k < D.nx; ++k) {
    const float c = hyper_c(D, i, l, k);
    const float fl = floorf(c);
    const int j0 = static_cast<int>(fl);
    float w[4];
    keys4(c - fl, w);
    const float* fk = f + static_cast<size_t>(k) * D.nt;
    float s = 0.0f;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int m = j0 - 1 + d;
      if (m >= 0 && m < D.nt) s += fk[m] * w[d];
    }
    const float wk = (k == 0 || k == D.nx - 1) ? 0.5f * D.dx : D.dx;
    acc += wk * s;
  }
  g[static_cast<size_t>(l) * D.ntau + i] = acc;
}

__global__ __launch_bounds__(256) void k_direct_adj(DirectGeo D,
                                                    const float* __restrict__ g,
                                                    float* __restrict__ f) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (m >= D.nt) return;
  const float x = D.x0 + static_cast<float>(k) * D.dx;
  float acc = 0.0f;
  for (int l = 0; l < D.nq; ++l) {
    const float qx = (D.q0 + static_cast<float>(l) * D.dq) * x;
    // tau range whose hyperbola time c satisfies floor(c) in [m-2, m+1]
    const float tlo = fmaxf(0.0f, (m - 2) * D.dt);
    const float thi = (m + 2) * D.dt;
    const float a2 = tlo * tlo - qx * qx;
    const float b2 = thi * thi - qx * qx;
    if (b2 < 0.0f) continue;
    const float tau_lo = a2 > 0.0f ? sqrtf(a2) : 0.0f;
    const float tau_hi = sqrtf(b2);
    int ilo = static_cast<int>(floorf((tau_lo - D.tau0) / D.dtau)) - 1;
    int ihi = static_cast<int>(ceilf((tau_hi - D.tau0) / D.dtau)) + 2;
    ilo = max(ilo, 0);
    ihi = min(ihi, D.ntau);
    const float* gl = g + static_cast<size_t>(l) * D.ntau;
    for (int i = ilo; i < ihi; ++i) {
      const float c = hyper_c(D, i, l, k);
      const float fl = floorf(c);
      const int d = m - static_cast<int>(fl) + 1;
      if (d < 0 || d > 3) continue;
      float w[4];
      keys4(c - fl, w);
      acc += gl[i] * w[d];
    }
  }
  const float wk = (k == 0 || k == D.nx - 1) ? 0.5f * D.dx : D.dx;
  f[static_cast<size_t>(k) * D.nt + m] = wk * acc;
}

}  // namespace hrt
