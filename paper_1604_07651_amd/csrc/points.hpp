// Point work of the spread: the fixed-point taps of one point, and a
// workgroup maximum.
#pragma once

#include "device_common.hpp"

namespace hrt {

// Adds v * B3(x - x_m) B3(y - y_n) over the taps of entry t to the chunk's
// accumulator in 64-bit fixed point.  `v` arrives already multiplied by the
// scale, chosen so that |every cell| and |every tap| <= 2^50 (the plan
// bounds the cells per unit input).  Each tap is the float64 product of v
// and the two float32 B-spline weights, rounded once to the nearest integer
// and added through the 64-bit integer LDS atomic; the integer sums are
// exact and independent of order, so a chunk's sums are deterministic and
// each cell is rounded to float32 once, when the chunk stores it.  (Float
// LDS atomics would give float32 sums, but they run about ten times slower
// than integer ones on gfx950 and their order, hence their rounding, varies
// from run to run.)  The rounding to an integer is one fused multiply-add
// with 1.5 * 2^52: for |x| < 2^51, x + 1.5 * 2^52 lies in [2^52, 2^53),
// where the float64 spacing is 1, so the sum is x rounded to the nearest
// integer and its low 52 bits hold that integer in two's complement; the
// constant's low word is zero, so subtracting its high word from the sum's
// high word leaves the integer as a 64-bit value.  Band row r, window column
// c0 + c is acc[r * wc + c]; rows outside [0, nr) belong to other bands and
// are dropped.
__device__ __forceinline__ void spread_taps(unsigned long long* acc, int wc, int c0, int nr,
                                            const EntryTaps& t, double v) {
  constexpr double kRound = 6755399441055744.0;  // 1.5 * 2^52
  constexpr int kRoundHi = 0x43380000;             // its high word
  double wx[4];
#pragma unroll
  for (int aa = 0; aa < 4; ++aa) wx[aa] = t.wx[aa];
#pragma unroll
  for (int bb = 0; bb < 4; ++bb) {
    const int rl = t.cy + bb;
    if (rl < 0 || rl >= nr) continue;
    unsigned long long* row = acc + rl * wc + (t.cx - c0);
    const double wr = v * static_cast<double>(t.wy[bb]);
#pragma unroll
    for (int aa = 0; aa < 4; ++aa) {
      const double s = fma(wr, wx[aa], kRound);
      const unsigned lo = static_cast<unsigned>(__double2loint(s));
      const unsigned hi = static_cast<unsigned>(__double2hiint(s) - kRoundHi);
      atomicAdd(row + aa, (static_cast<unsigned long long>(hi) << 32) | lo);
    }
  }
}

// Maximum over the workgroup (kNtBand threads; s_wave holds kNtBand/64
// floats and is used once per kernel, so one barrier suffices; it also
// orders every thread's earlier LDS writes before the return).
__device__ __forceinline__ float block_max(float v, float* s_wave) {
  constexpr int kWaves = kNtBand / 64;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) s_wave[threadIdx.x >> 6] = v;
  __syncthreads();
  float m = s_wave[0];
#pragma unroll
  for (int i = 1; i < kWaves; ++i) m = fmaxf(m, s_wave[i]);
  return m;
}

}  // namespace hrt
