// Point work of the spread: the fixed-point taps of one point, and a
// workgroup maximum.
#pragma once

#include "device_common.hpp"

namespace hrt {

// Adds v * B3(x - x_m) B3(y - y_n) over the taps of entry t to the chunk's
// accumulator in 64-bit fixed point: each tap is formed in float32 (so it
// carries float32's relative precision whatever its size) and enters as
// round(tap * scale) through the 64-bit integer LDS atomic.  `v` arrives
// already multiplied by the scale, chosen so that |every cell| <= 2^61 (the
// plan bounds the cells per unit input); the integer sums are exact and
// independent of order, so a chunk's sums are deterministic and each cell is
// rounded to float32 once, when the chunk stores it.  (Float LDS atomics
// would give float32 sums, but they run about ten times slower than integer
// ones on gfx950 and their order, hence their rounding, varies from run to
// run.)  Band row r, window column c0 + c is acc[r * wc + c]; rows outside
// [0, nr) belong to other bands and are dropped.
__device__ __forceinline__ void spread_taps(unsigned long long* acc, int wc, int c0, int nr,
                                            const EntryTaps& t, float v) {
#pragma unroll
  for (int bb = 0; bb < 4; ++bb) {
    const int rl = t.cy + bb;
    if (rl < 0 || rl >= nr) continue;
    unsigned long long* row = acc + rl * wc + (t.cx - c0);
    const float wr = v * t.wy[bb];
#pragma unroll
    for (int aa = 0; aa < 4; ++aa)
      atomicAdd(row + aa, static_cast<unsigned long long>(__float2ll_rn(wr * t.wx[aa])));
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
