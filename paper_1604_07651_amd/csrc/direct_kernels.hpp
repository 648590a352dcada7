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
// directions call these so the adjoint is the exact transpose.  The time is
// computed without fused multiply-adds (contraction off here): otherwise the
// compiler fuses it with the caller's code in ways that depend on which
// index is loop-invariant there (tau^2 + (qx)^2 fused on either product,
// the division by dt fused with the caller's subtraction of the floor), and
// the forward and adjoint kernels would place the same tap an ulp apart.
__device__ __forceinline__ float hyper_c(const DirectGeo& D, int i, int l, int k) {
#pragma clang fp contract(off)
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

// Bytes of dynamic LDS k_direct_adj_rows takes: a slowness's four weighted
// panel rows and its taus' tap bases (ntau each), the first-tau table
// (nt + 4) and the trace's sums (nt).
inline size_t direct_adj_rows_bytes(int nt, int ntau) {
  return sizeof(float) * (5 * static_cast<size_t>(ntau) + 2 * static_cast<size_t>(nt) + 4);
}

// The same transpose, one workgroup per trace k (kDirectThreads threads).
// For every slowness l in turn, each tau's hyperbola time c_i = hyper_c(i,
// l, k), its tap base j_i = floor(c_i) and its four Keys weights (keys4, as
// the forward computes them) are formed once; LDS holds v_d[i] = g[l][i] *
// w_d(c_i - j_i) for d = 0 .. 3 and j_i.  Since tau >= 0, c_i never
// decreases with i (every float operation in hyper_c is monotone), so with
// I(j) the first i with j_i >= j (tabulated from the steps of j_i), the
// taus whose tap d lands on sample m, j_i = m + 1 - d, are the run I(m + 1
// - d) <= i < I(m + 2 - d).  The thread owning sample m adds v_3, v_2, v_1,
// v_0 over those four runs, in increasing i, and that slowness's sum to the
// sample's total: every output sample is summed by one thread in a fixed
// order (deterministic, no atomics), and only taus whose taps reach the
// sample are visited.  The next slowness's panel row is loaded into
// registers while the current one is summed.
constexpr int kDirectThreads = 1024;
constexpr int kDirectRowRegs = 4;  // panel-row values a thread prefetches
__global__ __launch_bounds__(kDirectThreads) void k_direct_adj_rows(DirectGeo D,
                                                                    const float* __restrict__ g,
                                                                    float* __restrict__ f) {
  extern __shared__ float sm_direct[];
  const int nt = D.nt, ntau = D.ntau, k = blockIdx.x;
  float* v = sm_direct;                                 // [4][ntau]: v_d at d * ntau
  int* jb = reinterpret_cast<int*>(v + 4 * ntau);       // [ntau]: tap bases
  int* first = jb + ntau;                               // [nt + 4]: I(j) at j + 2
  float* acc = reinterpret_cast<float*>(first + nt + 4);  // [nt]
  for (int m = threadIdx.x; m < nt; m += kDirectThreads) acc[m] = 0.0f;
  // a thread's share of a panel row, prefetched a slowness ahead (rows
  // longer than kDirectRowRegs * kDirectThreads read the rest directly)
  float pre[kDirectRowRegs];
  auto load_row = [&](int l) {
    const float* row = g + static_cast<size_t>(l) * ntau;
#pragma unroll
    for (int r = 0; r < kDirectRowRegs; ++r) {
      const int i = threadIdx.x + r * kDirectThreads;
      pre[r] = i < ntau ? row[i] : 0.0f;
    }
  };
  auto stage = [&](int i, int l, float gv) {
    const float c = hyper_c(D, i, l, k);
    const float fl = floorf(c);
    float w[4];
    keys4(c - fl, w);
#pragma unroll
    for (int d = 0; d < 4; ++d) v[d * ntau + i] = gv * w[d];
    jb[i] = static_cast<int>(fl);
  };
  load_row(0);
  for (int l = 0; l < D.nq; ++l) {
    __syncthreads();  // the previous slowness is done with v, jb and first
#pragma unroll
    for (int r = 0; r < kDirectRowRegs; ++r) {
      const int i = threadIdx.x + r * kDirectThreads;
      if (i < ntau) stage(i, l, pre[r]);
    }
    for (int i = threadIdx.x + kDirectRowRegs * kDirectThreads; i < ntau; i += kDirectThreads)
      stage(i, l, g[static_cast<size_t>(l) * ntau + i]);
    __syncthreads();
    const int jf = jb[0], jl = jb[ntau - 1];
    // I(j) for jf < j <= jl, only where a sample reads it (j in [-2, nt + 1])
    for (int i = threadIdx.x + 1; i < ntau; i += kDirectThreads) {
      const int lo = max(jb[i - 1] + 1, -2), hi = min(jb[i], nt + 1);
      for (int j = lo; j <= hi; ++j) first[j + 2] = i;
    }
    if (l + 1 < D.nq) load_row(l + 1);
    __syncthreads();
    for (int m = threadIdx.x; m < nt; m += kDirectThreads) {
      // b[q] = I(m - 2 + q), q = 0 .. 4
      int b[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const int j = m - 2 + q;
        b[q] = j <= jf ? 0 : (j > jl ? ntau : first[j + 2]);
      }
      float s = 0.0f;
#pragma unroll
      for (int d = 3; d >= 0; --d) {  // tap d: taus with j_i = m + 1 - d
        const float* vd = v + d * ntau;
        for (int i = b[3 - d]; i < b[4 - d]; ++i) s += vd[i];
      }
      acc[m] += s;
    }
  }
  __syncthreads();
  const float wk = (k == 0 || k == D.nx - 1) ? 0.5f * D.dx : D.dx;
  for (int m = threadIdx.x; m < nt; m += kDirectThreads)
    f[static_cast<size_t>(k) * nt + m] = wk * acc[m];
}

}  // namespace hrt
