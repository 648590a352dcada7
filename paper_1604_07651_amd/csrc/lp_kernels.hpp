// The kernels of one direction of the log-polar transform (Section 2.2,
// eqs. B3tx2, lok, B3tauq; Section 3 for the adjoint):
//
//   k_absmax          largest |input| (fixes the spread's fixed-point scale)
//   k_spread_rowfft   one workgroup per band of R lattice rows: smear every
//                     sample whose B-spline stencil reaches the band (data
//                     samples for the forward, Radon samples for the
//                     adjoint), then the FFT along the angle, two real rows
//                     per complex sequence; store k1 < K1 of the half
//                     spectrum, column-major S[k1][row].
//   k_colfft          one workgroup per kept k1: FFT along the log radius,
//                     multiply by the kernel multiplier (its conjugate for
//                     the adjoint), inverse FFT.
//   k_rowifft_gather  one workgroup per band: Hermitian completion and
//                     inverse FFT along the angle of the band plus a 3-row
//                     halo, then the 4x4 B-spline interpolation at every
//                     sample whose base row lies in the band (Radon samples
//                     for the forward, data samples times their smear weight
//                     for the adjoint).
#pragma once

#include "points.hpp"

namespace hrt {

// Largest |x| over n floats as kAbsMaxBlocks partial maxima (no atomics and
// nothing to clear, so replays are safe); a non-finite input makes its block
// report +inf.
__global__ __launch_bounds__(256) void k_absmax(const float* __restrict__ x, int64_t n,
                                                float* __restrict__ partial) {
  __shared__ float s_m[4];
  float m = 0.0f;
  bool bad = false;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride) {
    const float v = fabsf(x[i]);
    bad |= !(v <= 3.0e38f);
    m = fmaxf(m, v);
  }
  if (bad) m = INFINITY;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    partial[blockIdx.x] = fmaxf(fmaxf(s_m[0], s_m[1]), fmaxf(s_m[2], s_m[3]));
}

// MODE 0: data samples f[nx][nt] (forward); MODE 1: Radon samples g[nq][ntau]
// (adjoint).  Dynamic LDS: the band's complex pairs at 0, the FFT scratch /
// fixed-point accumulator at k1_scratch, the walk's anchors at k1_anchor.
template <int MODE>
__global__ __launch_bounds__(kNtBand, 4) void k_spread_rowfft(
    DevGeo G, FftDev F, const float2* __restrict__ tw, const float* __restrict__ in,
    const float* __restrict__ absmax, float2* __restrict__ S) {
  extern __shared__ float2 lds[];
  __shared__ WalkLds walk;
  __shared__ float2 s_tw[kTwLds];
  const int band = xcd_band(G);
  if (band < 0) return;
  load_twiddles<kNtBand>(s_tw, tw, G.Mt);
  char* base = reinterpret_cast<char*>(lds);
  unsigned long long* acc64 = reinterpret_cast<unsigned long long*>(base + G.k1_scratch);
  const int n0 = G.u0 + band * G.R;
  const int nr = min(G.R, G.u1 - n0);
  const int npair = nr >> 1;
  const int Mt = G.Mt;
  const double Ylo = n0 - 2, Yhi = n0 + nr + 1;

  // largest |input| (from k_absmax) fixes the fixed-point scale
  float vmax = 0.0f;
  for (int i = threadIdx.x; i < kAbsMaxBlocks; i += kNtBand) vmax = fmaxf(vmax, absmax[i]);
  vmax = block_max(vmax, walk.wave);
  const float wmax = MODE == 0 ? G.wmax_data : G.wmax_radon;
  const bool finite = vmax <= 3.0e38f;  // false for inf and NaN
  const double scale =
      (vmax > 0.0f && finite) ? 1099511627776.0 / (static_cast<double>(wmax) * vmax) : 0.0;
  for (int i = threadIdx.x; i < nr * G.W; i += kNtBand) acc64[i] = 0ull;
  __syncthreads();

  // smear every point of the band (skipped when all inputs are 0)
  auto done = [&](TapAcc& acc) { acc.flush(acc64, G, n0, nr, scale); };
  if (scale > 0.0) {
    if (MODE == 0) {
      DataAnchors& an = *reinterpret_cast<DataAnchors*>(base + G.k1_anchor);
      balanced_walk<TapAcc>(
          G.nx, walk,
          [&](int slot, int k, int& lo, int& hi) {
            data_range(G, k, Ylo, Yhi, lo, hi);
            if (hi > lo) an.set(slot, G, lo, k);
          },
          [&](TapAcc& acc, int slot, int k, int j0, int len) {
            for_run_values(in, static_cast<size_t>(k) * G.nt + j0, len, [&](int t, float val) {
              if (val == 0.0f) return;
              double xg, yg;
              float w;
              an.eval(slot, G, j0 + t, xg, yg, w);
              const double fx0 = floor(xg);
              float wx[4];
              bspline4(static_cast<float>(xg - fx0), wx);
              acc.add(acc64, G, n0, nr, scale, static_cast<int>(fx0) - 1, wx, yg, w * val);
            });
          },
          done);
    } else {
      RadonAnchors& an = *reinterpret_cast<RadonAnchors*>(base + G.k1_anchor);
      balanced_walk<TapAcc>(
          G.nq, walk,
          [&](int slot, int l, int& lo, int& hi) {
            radon_range(G, G.qA[l], G.qB[l], Ylo, Yhi, lo, hi);
            if (hi > lo) an.set(slot, G, lo, l);
          },
          [&](TapAcc& acc, int slot, int l, int i0, int len) {
            const float4 q = an.qw[slot];
            const float wx[4] = {q.x, q.y, q.z, q.w};
            const int ix = an.i0[slot];
            const float sc = an.sc[slot];
            for_run_values(in, static_cast<size_t>(l) * G.ntau + i0, len, [&](int t, float val) {
              if (val == 0.0f) return;
              acc.add(acc64, G, n0, nr, scale, ix, wx, an.eval_y(slot, G, i0 + t), sc * val);
            });
          },
          done);
    }
  }
  __syncthreads();

  // fixed point -> float, rows (2p, 2p+1) into complex pair p (zero outside
  // the columns points can reach)
  const float inv = scale > 0.0 ? static_cast<float>(1.0 / scale) : 0.0f;
  const float bad = finite ? 0.0f : __int_as_float(0x7fc00000);
  for (int idx = threadIdx.x; idx < npair * Mt; idx += kNtBand) {
    const int p = idx / Mt;
    const int m = idx - p * Mt;
    const int c = m - G.xw0;
    float lo = 0.0f, hi = 0.0f;
    if (c >= 0 && c < G.W) {
      lo = from_fixed(acc64[(2 * p) * G.W + c], inv);
      hi = from_fixed(acc64[(2 * p + 1) * G.W + c], inv);
    }
    lds[idx] = make_float2(lo + bad, hi + bad);
  }
  __syncthreads();
  fft_batch<kNtBand, false>(lds, Mt, npair, reinterpret_cast<float2*>(base + G.k1_scratch),
                            G.grp1, F, s_tw);
  // two real rows per complex sequence: X1 = (Z[k] + conj Z[-k])/2,
  // X2 = (Z[k] - conj Z[-k])/(2i); keep k1 < K1
  for (int idx = threadIdx.x; idx < G.K1 * npair; idx += kNtBand) {
    const int k = idx / npair;
    const int p = idx - k * npair;
    const float2 Z = lds[p * Mt + k];
    const float2 Zm = lds[p * Mt + (k == 0 ? 0 : Mt - k)];
    const float4 o = make_float4(0.5f * (Z.x + Zm.x), 0.5f * (Z.y - Zm.y),
                                 0.5f * (Z.y + Zm.y), -0.5f * (Z.x - Zm.x));
    *reinterpret_cast<float4*>(S + static_cast<size_t>(k) * G.Mr + n0 + 2 * p) = o;
  }
}

template <bool ADJ>
__global__ __launch_bounds__(kNtCol) void k_colfft(DevGeo G, FftDev F,
                                                   const float2* __restrict__ tw,
                                                   float2* __restrict__ S,
                                                   const float2* __restrict__ K) {
  extern __shared__ float2 lds[];
  __shared__ float2 s_tw[kTwLds];
  load_twiddles<kNtCol>(s_tw, tw, G.Mr);
  const int k1 = blockIdx.x;
  const int Mr = G.Mr;
  float2* col = S + static_cast<size_t>(k1) * Mr;
  for (int n = threadIdx.x; n < Mr; n += kNtCol)
    lds[n] = (n >= G.u0 && n < G.u1) ? col[n] : make_float2(0.f, 0.f);
  __syncthreads();
  fft_batch<kNtCol, false>(lds, Mr, 1, lds + Mr, 1, F, s_tw);
  const float2* Kr = K + static_cast<size_t>(k1) * G.K2;
  for (int n = threadIdx.x; n < Mr; n += kNtCol) {
    const int k = (n < Mr / 2) ? n : n - Mr;
    const int ak = k < 0 ? -k : k;
    float2 v = make_float2(0.f, 0.f);
    if (ak < G.K2) {
      float2 kv = Kr[ak];
      // K(k1, -k2) = conj K(k1, k2); the adjoint uses conj K
      if ((k < 0) != ADJ) kv.y = -kv.y;
      v = cscale(cmul(lds[n], kv), G.knorm);
    }
    lds[n] = v;
  }
  __syncthreads();
  fft_batch<kNtCol, true>(lds, Mr, 1, lds + Mr, 1, F, s_tw);
  for (int n = G.u0 + threadIdx.x; n < G.u1; n += kNtCol) col[n] = lds[n];
}

// MODE 0: gather at Radon samples into g[nq][ntau] (forward); MODE 1: gather
// at data samples into f[nx][nt] (adjoint), zero outside the trapezoid.
// Dynamic LDS: the band's rows plus halo as complex pairs at 0, the FFT
// scratch at k3_scratch, the walk's anchors at k3_anchor.
template <int MODE>
__global__ __launch_bounds__(kNtBand, 4) void k_rowifft_gather(
    DevGeo G, FftDev F, const float2* __restrict__ tw, const float2* __restrict__ S,
    float* __restrict__ out) {
  extern __shared__ float2 lds[];
  __shared__ WalkLds walk;
  __shared__ float2 s_tw[kTwLds];
  const int band = xcd_band(G);
  if (band < 0) return;
  load_twiddles<kNtBand>(s_tw, tw, G.Mt);
  char* base = reinterpret_cast<char*>(lds);
  const float* ldsf = reinterpret_cast<const float*>(lds);
  const int n0 = G.u0 + band * G.R;
  const int nr = min(G.R, G.u1 - n0);
  const int L0 = max(G.u0, n0 - 1);
  const int L1 = min(G.u1, n0 + nr + 2);
  const int npair = (L1 - L0 + 1) >> 1;
  const int Mt = G.Mt;
  for (int i = threadIdx.x; i < npair * Mt; i += kNtBand) lds[i] = make_float2(0.f, 0.f);
  __syncthreads();
  // Z = X1 + i X2 for two real rows, Hermitian completion Z[-k]
  for (int idx = threadIdx.x; idx < G.K1 * npair; idx += kNtBand) {
    const int k = idx / npair;
    const int p = idx - k * npair;
    const int ra = L0 + 2 * p;
    const float2* src = S + static_cast<size_t>(k) * G.Mr;
    const float2 X1 = src[ra];
    const float2 X2 = (ra + 1 < L1) ? src[ra + 1] : make_float2(0.f, 0.f);
    lds[p * Mt + k] = make_float2(X1.x - X2.y, X1.y + X2.x);
    if (k > 0) lds[p * Mt + Mt - k] = make_float2(X1.x + X2.y, X2.x - X1.y);
  }
  __syncthreads();
  fft_batch<kNtBand, true>(lds, Mt, npair, reinterpret_cast<float2*>(base + G.k3_scratch),
                           G.grp3, F, s_tw);
  const double Ylo = n0, Yhi = n0 + nr;
  if (MODE == 0) {
    RadonAnchors& an = *reinterpret_cast<RadonAnchors*>(base + G.k3_anchor);
    balanced_walk<NoAcc>(
        G.nq, walk,
        [&](int slot, int l, int& lo, int& hi) {
          radon_range(G, G.qA[l], G.qB[l], Ylo, Yhi, lo, hi);
          if (hi > lo) an.set(slot, G, lo, l);
        },
        [&](NoAcc&, int slot, int l, int i0, int len) {
          const float4 q = an.qw[slot];
          const float wx[4] = {q.x, q.y, q.z, q.w};
          const int ix = an.i0[slot];
          const float sc = an.sc[slot];
          float* orow = out + static_cast<size_t>(l) * G.ntau;
          for (int i = i0; i < i0 + len; ++i) {
            double yg = an.eval_y(slot, G, i);
            if (near_row(yg)) yg = RadonAnchors::exact_y(G, i, l);
            const double fy0 = floor(yg);
            const int iy = static_cast<int>(fy0);
            if (iy < n0 || iy >= n0 + nr) continue;
            float wy[4];
            bspline4(static_cast<float>(yg - fy0), wy);
            orow[i] = sc * gather_taps(ldsf, Mt, L0, L1, ix, wx, iy, wy);
          }
        },
        [](NoAcc&) {});
  } else {
    DataAnchors& an = *reinterpret_cast<DataAnchors*>(base + G.k3_anchor);
    balanced_walk<NoAcc>(
        G.nx, walk,
        [&](int slot, int k, int& lo, int& hi) {
          data_range(G, k, Ylo, Yhi, lo, hi);
          if (hi > lo) an.set(slot, G, lo, k);
        },
        [&](NoAcc&, int slot, int k, int j0, int len) {
          float* orow = out + static_cast<size_t>(k) * G.nt;
          for (int j = j0; j < j0 + len; ++j) {
            double xg, yg;
            float w;
            an.eval(slot, G, j, xg, yg, w);
            if (near_row(yg)) DataAnchors::exact(G, j, k, xg, yg, w);
            const double fy0 = floor(yg);
            const int iy = static_cast<int>(fy0);
            if (iy < n0 || iy >= n0 + nr) continue;
            const double fx0 = floor(xg);
            float wx[4], wy[4];
            bspline4(static_cast<float>(xg - fx0), wx);
            bspline4(static_cast<float>(yg - fy0), wy);
            orow[j] = w * gather_taps(ldsf, Mt, L0, L1, static_cast<int>(fx0) - 1, wx, iy, wy);
          }
        },
        [](NoAcc&) {});
    // samples outside the trapezoid: each trace zeroed by one band
    for (int k = band; k < G.nx; k += G.nbands) {
      float* fk = out + static_cast<size_t>(k) * G.nt;
      for (int j = threadIdx.x; j < G.jmin[k]; j += kNtBand) fk[j] = 0.0f;
    }
  }
}

}  // namespace hrt
