// Device-side constants, the kernel parameter block and the small helpers
// shared by the log-polar kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft.hpp"
#include "plan.hpp"

namespace hrt {

constexpr int kNtBand = kBandThreads;  // threads of the band kernels
constexpr int kNtCol = kColThreads;    // threads of the column kernel
constexpr int kAbsMaxBlocks = 1024;    // partial maxima of the input, one gather
constexpr int kAbsMaxBlocksBatch = 64; // ... per gather of a batch

// The four point lists of a plan, cut into chunks (see BandLists).
enum { kDataSpread = 0, kDataOwn = 1, kRadonSpread = 2, kRadonOwn = 3 };
struct DevList {
  const uint4* ent;   // 16-byte entries (data lists)
  const uint2* ent2;  // Radon lists: {sample index, log-radius coordinate}; the
                      // angle coordinate and weight are the slowness's (q_tab)
  const int64_t* chunk_off;
  const int* chunk_band;
  const int* band_chunk;
  // spread lists: the window columns {c_lo, wc} of each chunk and where its
  // partial rows (R x wc floats) start in Hp; null for the owned lists
  const int2* chunk_col;
  const int64_t* chunk_hp;
  int nchunks;
};

// Everything the kernels need about one gather's plan.  The kernels read it
// from a device table, one entry per gather of a batch (one for a single
// plan), and get their work as (gather, item) pairs.
struct DevGeo {
  int nt, nx, ntau, nq;
  int Mt, Mr, K1, K2, u0, u1, R, nbands;
  int row_rows, row_sub_shift;  // rows of a row-FFT item, log2 items per band
  int xw0, W;         // angle columns [xw0, xw0 + W) that points can touch
  int x_frac_bits;    // fraction bits of the angle coordinate of a point entry
  int spread_cols;    // most columns of a spread chunk (its LDS accumulator)
  // row FFTs: sequences per group, byte offset of the LDS scratch (-1: in
  // place); the column FFT in place or not
  int row_group, row_scratch;
  int col_inplace, col_batch;
  float knorm;                  // 1/(Mt Mr): both inverse FFTs are unnormalised
  float cmax_data, cmax_radon;  // bounds of the accumulated cells per unit input
  int absmax_blocks;            // partial maxima of this gather's input
  int64_t data_off, radon_off;  // this gather's offsets in packed batch arrays
  // placement of a part of a split gather (whole grids: data_ld = nt,
  // radon_ld = ntau, j_lo = 0, j_hi = nt, radon_row0 = 0, nx_fill = nx):
  // row strides of the arrays, the data band [j_lo, j_hi) the part takes
  // in, its first slowness row, the traces the adjoint's zero fill covers
  int data_ld, radon_ld, j_lo, j_hi, radon_row0, nx_fill;
  int accumulate;               // the gathers add into the output
  FftDev ft, fr;                // angle and log-radius FFTs
  const float2* tw_t;
  const float2* tw_r;
  const float2* K;              // kernel multiplier [K1][K2]
  float2* S;                    // half spectrum [K1][Mr]
  float* Hp;                    // spread partial rows, chunk c's R x wc at chunk_hp[c]
  float* Cr;                    // real rows after the inverse row FFT [u1-u0][W]
  float* absmax;                // absmax_blocks partial maxima
  // when set, the forward gather stores the largest |output| of each of its
  // chunks here (+inf for a non-finite output): the partial maxima of an
  // adjoint that takes the forward's output as its input
  float* gmax;
  // per slowness of the plan: {angle coordinate, weight bits} of its Radon
  // points; a Radon sample index idx lies in array row
  // (idx * rdiv_m) >> rdiv_s = idx / radon_ld (exact for idx < 2^31, which
  // plans enforce; the plan also checks it for every entry)
  const uint2* q_tab;
  uint64_t rdiv_m;
  int rdiv_s;
  const int* jmin;              // [nx_fill] first kept time sample of each trace
  DevList lists[4];
};

// Cubic B-spline weights of taps i0-1 .. i0+2 for fractional offset f.
__device__ __forceinline__ void bspline4(float f, float w[4]) {
  const float g = 1.0f - f;
  w[0] = g * g * g * (1.0f / 6.0f);
  w[1] = 2.0f / 3.0f - f * f + 0.5f * f * f * f;
  w[2] = 2.0f / 3.0f - g * g + 0.5f * g * g * g;
  w[3] = f * f * f * (1.0f / 6.0f);
}

// A point entry's coordinates: first angle tap column relative to xw0,
// first tap row relative to the band's row n0 (rows n0 - 3 + yi .. n0 + yi),
// and the B-spline weights of the four taps along each axis.
struct EntryTaps {
  int cx, cy;
  float wx[4], wy[4];
};

__device__ __forceinline__ EntryTaps decode_entry(uint32_t xq, uint32_t yq, int xbits) {
  EntryTaps t;
  const uint32_t xmask = (1u << xbits) - 1u;
  t.cx = static_cast<int>(xq >> xbits) - 1;
  t.cy = static_cast<int>(yq >> kYFracBits) - 3;
  const float fx = static_cast<float>(xq & xmask) * __builtin_ldexpf(1.0f, -xbits);
  const float fy = static_cast<float>(yq & ((1u << kYFracBits) - 1u)) *
                   (1.0f / static_cast<float>(1u << kYFracBits));
  bspline4(fx, t.wx);
  bspline4(fy, t.wy);
  return t;
}

// for (i = threadIdx.x; i < n; i += NT) use(i, load(i)), with the loads of
// G consecutive iterations issued before the first of their uses: their
// memory latencies overlap instead of adding up one iteration at a time.
template <int NT, int G, typename Load, typename Use>
__device__ __forceinline__ void grouped_for(int n, Load load, Use use) {
  using T = decltype(load(0));
  for (int i0 = static_cast<int>(threadIdx.x); i0 < n; i0 += NT * G) {
    T v[G];
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (i0 + g * NT < n) v[g] = load(i0 + g * NT);
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (i0 + g * NT < n) use(i0 + g * NT, v[g]);
  }
}

// The full entry {idx, angle, log radius, weight} of a compact Radon entry
// {idx, log radius}: the slowness row from the index, its angle coordinate
// and weight from the plan's table (the row clamped into the table).
__device__ __forceinline__ uint4 radon_entry(const DevGeo& G, uint2 e) {
  const uint64_t row = (static_cast<uint64_t>(e.x) * G.rdiv_m) >> G.rdiv_s;
  const int l = min(max(static_cast<int>(row) - G.radon_row0, 0), G.nq - 1);
  const uint2 t = G.q_tab[l];
  return make_uint4(e.x, t.x, e.y, t.y);
}

// LDS scratch of an FFT: null when it runs in place.
__device__ __forceinline__ float2* fft_scratch(char* lds_base, int offset) {
  return offset < 0 ? nullptr : reinterpret_cast<float2*>(lds_base + offset);
}

}  // namespace hrt
