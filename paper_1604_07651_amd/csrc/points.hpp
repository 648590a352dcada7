// Point work of the spread: the fixed-point taps of one point, and a
// workgroup maximum.
#pragma once

#include "device_common.hpp"

namespace hrt {

// Adds v * B3(x - x_m) B3(y - y_n) over the taps of entry t to the band's
// accumulator, in 32-bit fixed point: a tap value enters as round(tap *
// scale) through the integer LDS atomic (float LDS atomics are far slower on
// gfx950).  `v` arrives already multiplied by the scale, chosen so that
// |every cell| <= 2^30 (the plan bounds the cells per unit input); integer
// sums are exact and independent of order, so the band is deterministic.
// Band row r, window column c is acc[r * W + c]; rows outside [0, nr) belong
// to other bands and are dropped.
__device__ __forceinline__ void spread_taps(int* acc, int W, int nr, const EntryTaps& t,
                                            float v) {
#pragma unroll
  for (int bb = 0; bb < 4; ++bb) {
    const int rl = t.cy + bb;
    if (rl < 0 || rl >= nr) continue;
    int* row = acc + rl * W + t.cx;
    const float wr = v * t.wy[bb];
#pragma unroll
    for (int aa = 0; aa < 4; ++aa) atomicAdd(row + aa, __float2int_rn(wr * t.wx[aa]));
  }
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
