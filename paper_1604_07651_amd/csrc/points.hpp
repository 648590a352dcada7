// Point work of the band kernels: the fixed-point tap accumulator of the
// spread and the 4x4 interpolation of the gather.
#pragma once

#include "device_common.hpp"

namespace hrt {

// Per-thread accumulator of the 4x4 B-spline taps of consecutive points that
// fall on the same lattice cell (a thread runs through consecutive entries
// of its band list, which are consecutive samples of one trace or slowness
// column, and where the lattice is coarse many of them share a cell): their
// taps are summed in registers and reach LDS as one set of 16 atomic adds.
//
// The band accumulates in 64-bit fixed point: a tap value v enters as
// round(v * scale), scale = 2^40 / (bound on |v|), added with the integer
// LDS atomic (float LDS atomics are far slower on gfx950).  Integer sums are
// exact and order-independent, so the band is deterministic; the quantum is
// 2^-40 of the largest possible tap.  Band row r, window column c is
// acc64[r * W + c]; rows outside [0, nr) are other bands' and dropped.
struct TapAcc {
  int cx = -1, cy = 0;  // pending cell (first tap column and row), cx < 0: none
  float a[4][4];

  __device__ __forceinline__ void flush(unsigned long long* acc64, int W, int nr,
                                        double scale) {
    if (cx < 0) return;
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      const int rl = cy + bb;
      if (rl < 0 || rl >= nr) continue;
      unsigned long long* row = acc64 + rl * W + cx;
#pragma unroll
      for (int aa = 0; aa < 4; ++aa) atomicAdd(row + aa, to_fixed(a[bb][aa], scale));
    }
    cx = -1;
  }

  // add v * B3(x - x_m) B3(y - y_n) over the taps of entry t
  __device__ __forceinline__ void add(unsigned long long* acc64, int W, int nr, double scale,
                                      const EntryTaps& t, float v) {
    if (t.cx != cx || t.cy != cy) {
      flush(acc64, W, nr, scale);
      cx = t.cx;
      cy = t.cy;
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
#pragma unroll
        for (int aa = 0; aa < 4; ++aa) a[bb][aa] = 0.0f;
    }
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      const float wr = v * t.wy[bb];
#pragma unroll
      for (int aa = 0; aa < 4; ++aa) a[bb][aa] += wr * t.wx[aa];
    }
  }
};

// Sum of C[m, n] B3(x - m) B3(y - n) over the 4x4 taps of a point, C being
// lattice rows held in LDS as complex pairs in the FFT's padded layout (held
// row r at component r & 1 of pair r >> 1, pairs SP complex values apart,
// rows [0, nheld)); `row0` is the held row of the first tap, `col0` the
// lattice column of the first tap.  Taps outside the held rows are skipped
// (no point a band owns reaches them with a non-zero weight).
__device__ __forceinline__ float gather_taps(const float* ldsf, int SP, int nheld, int row0,
                                             int col0, const float wx[4], const float wy[4]) {
  int pc[4];
#pragma unroll
  for (int aa = 0; aa < 4; ++aa) pc[aa] = 2 * lpad(col0 + aa);
  float acc = 0.0f;
#pragma unroll
  for (int bb = 0; bb < 4; ++bb) {
    const int rl = row0 + bb;
    if (rl < 0 || rl >= nheld) continue;
    const float* base = ldsf + (rl >> 1) * SP * 2 + (rl & 1);
    float row = 0.0f;
#pragma unroll
    for (int aa = 0; aa < 4; ++aa) row += base[pc[aa]] * wx[aa];
    acc += row * wy[bb];
  }
  return acc;
}

// Maximum over the workgroup (kNtBand threads; s_wave holds kNtBand/64 floats).
__device__ __forceinline__ float block_max(float v, float* s_wave) {
  constexpr int kWaves = kNtBand / 64;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_wave[threadIdx.x >> 6] = v;
  __syncthreads();
  float m = s_wave[0];
#pragma unroll
  for (int i = 1; i < kWaves; ++i) m = fmaxf(m, s_wave[i]);
  __syncthreads();
  return m;
}

}  // namespace hrt
