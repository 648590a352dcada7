// The kernels of one direction of the log-polar transform (Section 2.2,
// eqs. B3tx2, lok, B3tauq; Section 3 for the adjoint):
//
//   k_absmax          largest |input| (fixes the spread's fixed-point scale)
//   k_spread_rowfft   one workgroup per band of R lattice rows: smear every
//                     sample whose B-spline stencil reaches the band (data
//                     samples for the forward, Radon samples for the
//                     adjoint; the band's list of placed points comes from
//                     the plan), then the FFT along the angle, two real
//                     rows per complex sequence; store k1 < K1 of the half
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

// Spread of one point set (MODE 0: data samples of f[nx][nt], forward;
// MODE 1: Radon samples of g[nq][ntau], adjoint) from the band's list
// ent[off[band] .. off[band+1]); workgroup i takes band order[i] (heaviest
// lists first).  Dynamic LDS: the band's complex pairs at 0 (they first
// stage the point list), the 32-bit fixed-point rows at k1_acc, the FFT
// scratch (if any) at k1_scratch over the fixed-point rows.
template <int MODE>
__global__ __launch_bounds__(kNtBand, 4) void k_spread_rowfft(
    DevGeo G, FftDev F, const float2* __restrict__ tw, const float* __restrict__ in,
    const float* __restrict__ absmax, const uint4* __restrict__ ent,
    const int64_t* __restrict__ off, const int* __restrict__ order, float2* __restrict__ S) {
  extern __shared__ float2 lds[];
  __shared__ float s_wave[kNtBand / 64];
  __shared__ float2 s_tw[kTwLds];
  const int band = order[blockIdx.x];
  load_twiddles<kNtBand>(s_tw, tw, G.Mt);
  char* base = reinterpret_cast<char*>(lds);
  int* acc = reinterpret_cast<int*>(base + G.k1_acc);
  const int n0 = G.u0 + band * G.R;
  const int nr = min(G.R, G.u1 - n0);
  const int npair = nr >> 1;
  const int Mt = G.Mt, W = G.W, SP = padded_len(G.Mt);

  // largest |input| (from k_absmax) fixes the fixed-point scale: every
  // cell stays within 2^30 (cmax bounds a cell per unit input)
  float vmax = 0.0f;
  for (int i = threadIdx.x; i < kAbsMaxBlocks; i += kNtBand) vmax = fmaxf(vmax, absmax[i]);
  vmax = block_max(vmax, s_wave);
  const float cmax = MODE == 0 ? G.cmax_data : G.cmax_radon;
  const bool finite = vmax <= 3.0e38f;  // false for inf and NaN
  const float scale = (vmax > 0.0f && finite) ? 1073741824.0f / (cmax * vmax) : 0.0f;
  for (int i = threadIdx.x; i < nr * W; i += kNtBand) acc[i] = 0;
  __syncthreads();

  // smear the band's points (skipped when all inputs are 0).  The list is
  // read in chunks, coalesced, into the pair rows (idle until the FFT); in a
  // chunk thread s takes a contiguous segment, segments dealt lane-major so
  // that the lanes of a wave work far apart on the lattice.
  if (scale > 0.0f) {
    uint4* stage = reinterpret_cast<uint4*>(base);
    const int cap = G.k1_acc / static_cast<int>(sizeof(uint4));
    const int64_t e0 = off[band], e1 = off[band + 1];
    const int seg = (threadIdx.x & 63) * (kNtBand / 64) + (threadIdx.x >> 6);
    for (int64_t c0 = e0; c0 < e1; c0 += cap) {
      const int n = static_cast<int>(min(static_cast<int64_t>(cap), e1 - c0));
      for (int i = threadIdx.x; i < n; i += kNtBand) stage[i] = ent[c0 + i];
      __syncthreads();
      const int per = (n + kNtBand - 1) / kNtBand;
      int p = seg * per;
      const int pend = min(p + per, n);
      for (; p < pend; p += 4) {
        uint4 E[4];
        float v[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) E[t] = (p + t < pend) ? stage[p + t] : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int t = 0; t < 4; ++t) v[t] = (p + t < pend) ? in[E[t].x] : 0.0f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if (v[t] != 0.0f) {
            const EntryTaps tp = decode_entry(E[t].y, E[t].z, G.x_frac_bits);
            spread_taps(acc, W, nr, tp, v[t] * __uint_as_float(E[t].w) * scale);
          }
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();

  // fixed point -> float, rows (2p, 2p+1) into complex pair p (zero outside
  // the columns points can reach)
  const float inv = scale > 0.0f ? 1.0f / scale : 0.0f;
  const float bad = finite ? 0.0f : __int_as_float(0x7fc00000);
  for (int idx = threadIdx.x; idx < npair * Mt; idx += kNtBand) {
    const int p = idx / Mt;
    const int m = idx - p * Mt;
    const int c = m - G.xw0;
    float lo = 0.0f, hi = 0.0f;
    if (c >= 0 && c < W) {
      lo = static_cast<float>(acc[(2 * p) * W + c]) * inv;
      hi = static_cast<float>(acc[(2 * p + 1) * W + c]) * inv;
    }
    lds[p * SP + lpad(m)] = make_float2(lo + bad, hi + bad);
  }
  __syncthreads();
  fft_rows<kNtBand, false>(lds, SP, npair, fft_scratch(base, G.k1_scratch), G.grp1, F, s_tw);
  // two real rows per complex sequence: X1 = (Z[k] + conj Z[-k])/2,
  // X2 = (Z[k] - conj Z[-k])/(2i); keep k1 < K1
  for (int idx = threadIdx.x; idx < G.K1 * npair; idx += kNtBand) {
    const int k = idx / npair;
    const int p = idx - k * npair;
    const float2 Z = lds[p * SP + lpad(k)];
    const float2 Zm = lds[p * SP + lpad(k == 0 ? 0 : Mt - k)];
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
  const int Mr = G.Mr, SP = padded_len(G.Mr);
  float2* col = S + static_cast<size_t>(k1) * Mr;
  for (int n = threadIdx.x; n < Mr; n += kNtCol)
    lds[lpad(n)] = (n >= G.u0 && n < G.u1) ? col[n] : make_float2(0.f, 0.f);
  __syncthreads();
  float2* cscr = G.col_inplace ? nullptr : lds + SP;
  fft_rows<kNtCol, false>(lds, SP, 1, cscr, 1, F, s_tw);
  const float2* Kr = K + static_cast<size_t>(k1) * G.K2;
  for (int n = threadIdx.x; n < Mr; n += kNtCol) {
    const int k = (n < Mr / 2) ? n : n - Mr;
    const int ak = k < 0 ? -k : k;
    float2 v = make_float2(0.f, 0.f);
    if (ak < G.K2) {
      float2 kv = Kr[ak];
      // K(k1, -k2) = conj K(k1, k2); the adjoint uses conj K
      if ((k < 0) != ADJ) kv.y = -kv.y;
      v = cscale(cmul(lds[lpad(n)], kv), G.knorm);
    }
    lds[lpad(n)] = v;
  }
  __syncthreads();
  fft_rows<kNtCol, true>(lds, SP, 1, cscr, 1, F, s_tw);
  for (int n = G.u0 + threadIdx.x; n < G.u1; n += kNtCol) col[n] = lds[lpad(n)];
}

// Gather at the points the band owns (MODE 0: Radon samples into
// g[nq][ntau], forward; MODE 1: data samples times their smear weight into
// f[nx][nt], adjoint, zero outside the trapezoid), from the band's list
// ent[off[band] .. off[band+1]), workgroup i taking band order[i].  Dynamic
// LDS: the band's rows plus halo as
// complex pairs at 0, the FFT scratch (if any) at k3_scratch.
template <int MODE>
__global__ __launch_bounds__(kNtBand, 4) void k_rowifft_gather(
    DevGeo G, FftDev F, const float2* __restrict__ tw, const float2* __restrict__ S,
    const uint4* __restrict__ ent, const int64_t* __restrict__ off, const int* __restrict__ order,
    float* __restrict__ out) {
  extern __shared__ float2 lds[];
  __shared__ float2 s_tw[kTwLds];
  const int band = order[blockIdx.x];
  load_twiddles<kNtBand>(s_tw, tw, G.Mt);
  char* base = reinterpret_cast<char*>(lds);
  const float* ldsf = reinterpret_cast<const float*>(lds);
  const int n0 = G.u0 + band * G.R;
  const int nr = min(G.R, G.u1 - n0);
  const int L0 = max(G.u0, n0 - 1);
  const int L1 = min(G.u1, n0 + nr + 2);
  const int npair = (L1 - L0 + 1) >> 1;
  const int Mt = G.Mt, SP = padded_len(G.Mt);
  for (int i = threadIdx.x; i < npair * SP; i += kNtBand) lds[i] = make_float2(0.f, 0.f);
  __syncthreads();
  // Z = X1 + i X2 for two real rows, Hermitian completion Z[-k]
  for (int idx = threadIdx.x; idx < G.K1 * npair; idx += kNtBand) {
    const int k = idx / npair;
    const int p = idx - k * npair;
    const int ra = L0 + 2 * p;
    const float2* src = S + static_cast<size_t>(k) * G.Mr;
    const float2 X1 = src[ra];
    const float2 X2 = (ra + 1 < L1) ? src[ra + 1] : make_float2(0.f, 0.f);
    lds[p * SP + lpad(k)] = make_float2(X1.x - X2.y, X1.y + X2.x);
    if (k > 0) lds[p * SP + lpad(Mt - k)] = make_float2(X1.x + X2.y, X2.x - X1.y);
  }
  __syncthreads();
  fft_rows<kNtBand, true>(lds, SP, npair, fft_scratch(base, G.k3_scratch), G.grp3, F, s_tw);
  // one point per thread, consecutive threads on consecutive entries
  const int64_t e0 = off[band], e1 = off[band + 1];
  const int nheld = L1 - L0, shift = n0 - L0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kNtBand) {
    const uint4 E = ent[e];
    const EntryTaps tp = decode_entry(E.y, E.z, G.x_frac_bits);
    out[E.x] = __uint_as_float(E.w) *
               gather_taps(ldsf, SP, nheld, tp.cy + shift, G.xw0 + tp.cx, tp.wx, tp.wy);
  }
  if (MODE == 1) {
    // samples outside the trapezoid: each trace zeroed by one band
    for (int k = band; k < G.nx; k += G.nbands) {
      float* fk = out + static_cast<size_t>(k) * G.nt;
      for (int j = threadIdx.x; j < G.jmin[k]; j += kNtBand) fk[j] = 0.0f;
    }
  }
}

}  // namespace hrt
