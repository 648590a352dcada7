// The kernels of one direction of the log-polar transform (Section 2.2,
// eqs. B3tx2, lok, B3tauq; Section 3 for the adjoint).  The lattice rows
// [u0, u1) are cut into bands of R rows; the point lists of the plan are cut
// into chunks of at most a fixed number of entries, so that the point
// kernels get equal work whatever the density of points along the lattice.
// A single plan passes its gather descriptor by value and workgroup w does
// item w; a batch (BATCH = true) passes a device table of descriptors and a
// list of work items (gather, index), workgroup w doing item w, so that one
// launch covers every gather of the batch.
//
//   k_absmax   largest |input| (fixes the spread's fixed-point scale)
//   k_spread   one workgroup per chunk of a band's spread list: smear the
//              chunk's samples (data samples for the forward, Radon samples
//              for the adjoint) onto the band's rows over the columns the
//              chunk spans, in LDS (exact 64-bit fixed-point sums); store
//              them rounded to float32 as the chunk's partial rows
//   k_rowfft   one workgroup per band: sum the band's partials (float32, in
//              chunk order), FFT along
//              the angle, two real rows per complex sequence; store k1 < K1
//              of the half spectrum, column-major S[k1][row]
//   k_colfft   one workgroup per kept k1: FFT along the log radius, multiply
//              by the kernel multiplier (its conjugate for the adjoint),
//              inverse FFT
//   k_rowifft  one workgroup per band: Hermitian completion and inverse FFT
//              along the angle; store the real rows, window columns only,
//              as Cr[row - u0][column - xw0]
//   k_gather   one workgroup per chunk of a band's owned list: stage the
//              band's rows plus a 3-row halo from Cr in LDS and interpolate
//              at each sample (Radon samples times X cos(psi)/a for the
//              forward, data samples times their smear weight for the
//              adjoint, which also zeroes the samples outside the trapezoid)
#pragma once

#include "points.hpp"

namespace hrt {

// The gather descriptor and the index of this workgroup's work item.
struct Work {
  const DevGeo& G;
  int i;
};
template <bool BATCH>
__device__ __forceinline__ Work work_item(const DevGeo& one, const DevGeo* __restrict__ geos,
                                          const int2* __restrict__ items) {
  // a single plan's launch may come with its own order of items (negative:
  // nothing to do); without one, item i is workgroup i
  if (!BATCH) return Work{one, items ? items[blockIdx.x].y : static_cast<int>(blockIdx.x)};
  const int2 it = items[blockIdx.x];
  return Work{geos[it.x], it.y};
}

// Largest |x| of one gather's input (MODE 0: the data band, MODE 1: the
// Radon rows) as absmax_blocks partial maxima (no atomics and nothing to
// clear, so replays are safe); item i is partial i.  A non-finite input
// makes its block report +inf.  A contiguous input takes 16-byte loads when
// it is 16-byte aligned; the band of a part is read row by row.
template <int MODE, bool BATCH>
__global__ __launch_bounds__(256) void k_absmax(DevGeo one, const DevGeo* __restrict__ geos,
                                                const int2* __restrict__ items,
                                                const float* __restrict__ in) {
  __shared__ float s_m[4];
  const Work w = work_item<BATCH>(one, geos, items);
  const DevGeo& G = w.G;
  const float* x = in + (MODE == 0 ? G.data_off + G.j_lo
                                    : G.radon_off + static_cast<int64_t>(G.radon_row0) * G.radon_ld);
  const int rows = MODE == 0 ? G.nx : G.nq;
  const int cols = MODE == 0 ? G.j_hi - G.j_lo : G.ntau;
  const int ld = MODE == 0 ? G.data_ld : G.radon_ld;
  const int64_t n = cols == ld ? static_cast<int64_t>(rows) * cols : 0;
  float m = 0.0f;
  bool bad = false;
  const int64_t tid = static_cast<int64_t>(w.i) * blockDim.x + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(G.absmax_blocks) * blockDim.x;
  int64_t done = 0;
  if (cols != ld) {
    for (int r = w.i; r < rows; r += G.absmax_blocks) {
      const float* xr = x + static_cast<int64_t>(r) * ld;
      for (int c = threadIdx.x; c < cols; c += blockDim.x) {
        const float v = fabsf(xr[c]);
        bad |= !(v <= 3.0e38f);
        m = fmaxf(m, v);
      }
    }
  } else if ((reinterpret_cast<uintptr_t>(x) & 15) == 0) {
    const float4* x4 = reinterpret_cast<const float4*>(x);
    const int64_t n4 = n / 4;
    for (int64_t i = tid; i < n4; i += stride) {
      const float4 v = x4[i];
      const float a = fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w)));
      bad |= !(fabsf(v.x) <= 3.0e38f && fabsf(v.y) <= 3.0e38f && fabsf(v.z) <= 3.0e38f &&
               fabsf(v.w) <= 3.0e38f);
      m = fmaxf(m, a);
    }
    done = 4 * n4;
  }
  for (int64_t i = done + tid; i < n; i += stride) {
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
    G.absmax[w.i] = fmaxf(fmaxf(s_m[0], s_m[1]), fmaxf(s_m[2], s_m[3]));
}

// The spread's fixed-point scale (float64) from each thread's maximum over
// its share of the input maximum's partials: every accumulated cell and
// every tap stays within 2^50 (cmax bounds a cell per unit of input, and a
// single tap by as much); 0 for an all-zero or non-finite input (the latter
// is reported through `finite`).  Ends with a barrier.
__device__ __forceinline__ double spread_scale(float vmax, float cmax, float* s_wave,
                                               bool& finite) {
  vmax = block_max(vmax, s_wave);
  finite = vmax <= 3.0e38f;  // false for inf and NaN
  return (vmax > 0.0f && finite)
             ? 1125899906842624.0 / (static_cast<double>(cmax) * vmax)  // 2^50 / (cmax vmax)
             : 0.0;
}

// Spread of one chunk (MODE 0: data samples of f[nx][nt]; MODE 1: Radon
// samples of g[nq][ntau]); item i is chunk i of the spread list.  Dynamic
// LDS: the band's R rows over the chunk's wc columns [c_lo, c_lo + wc) as
// 64-bit fixed-point cells (R x spread_cols reserved).  Each thread reads
// its entries straight from the list, kNtBand entries apart, dealt so that
// the lanes of a wave work far apart on the lattice.  The chunk's exact
// sums are rounded once to float32 into its partial rows, R x wc floats at
// Hp + chunk_hp[chunk].
template <int MODE, bool BATCH>
__global__ __launch_bounds__(kNtBand) void k_spread(DevGeo one, const DevGeo* __restrict__ geos,
                                                    const int2* __restrict__ items,
                                                    const float* __restrict__ in_base) {
  extern __shared__ unsigned long long lds_q[];
  __shared__ float s_wave[kNtBand / 64];
  const Work w = work_item<BATCH>(one, geos, items);
  if (w.i < 0) return;  // a gap in the XCD-ordered items
  const DevGeo& G = w.G;
  const DevList& L = G.lists[MODE == 0 ? kDataSpread : kRadonSpread];
  const float* in = in_base + (MODE == 0 ? G.data_off : G.radon_off);
  const int chunk = w.i;
  const int band = L.chunk_band[chunk];
  const int n0 = G.u0 + band * G.R;
  const int nr = min(G.R, G.u1 - n0);
  const int2 cols = L.chunk_col[chunk];  // {c_lo, wc}
  const int wc = cols.y;
  unsigned long long* acc = lds_q;
  // the input maximum's partials are loaded first and the accumulator is
  // cleared while they arrive; the scale's barriers also close the clearing
  constexpr int kPre = 4;
  float pre[kPre];
#pragma unroll
  for (int k = 0; k < kPre; ++k) {
    const int i = threadIdx.x + k * kNtBand;
    pre[k] = i < G.absmax_blocks ? G.absmax[i] : 0.0f;
  }
  for (int i = threadIdx.x; i < nr * wc; i += kNtBand) acc[i] = 0ull;
  float vpart = fmaxf(fmaxf(pre[0], pre[1]), fmaxf(pre[2], pre[3]));
  for (int i = threadIdx.x + kPre * kNtBand; i < G.absmax_blocks; i += kNtBand)
    vpart = fmaxf(vpart, G.absmax[i]);
  bool finite;
  const double scale =
      spread_scale(vpart, MODE == 0 ? G.cmax_data : G.cmax_radon, s_wave, finite);
  if (scale > 0.0) {
    const int64_t e0 = L.chunk_off[chunk], e1 = L.chunk_off[chunk + 1];
    // the chunk is taken kNtBand entries at a time, thread t doing entry
    // seg(t) of each block: data points: lane l of wave v takes (l % 8) *
    // (kNtBand / 8) + 8 v + l / 8, the eight lane groups of a wave an eighth
    // of the block apart; Radon points (runs of one slowness share their
    // columns): 101 t mod kNtBand, lanes scattered over the block (both
    // measured fastest for their point set).  Entries are read straight
    // from the list (a block is 4-8 KB, cached); each thread's entry two
    // blocks ahead and its value one block ahead are in flight while it
    // adds the current point's taps.
    const int seg = MODE == 0 ? (threadIdx.x & 7) * (kNtBand / 8) + (threadIdx.x >> 3)
                              : (threadIdx.x * 101) & (kNtBand - 1);
    static_assert((kNtBand & (kNtBand - 1)) == 0, "segment permutation needs a power of two");
    auto entry = [&](int64_t e) {
      if (e >= e1) return make_uint4(0u, 0u, 0u, 0u);
      return MODE == 1 ? radon_entry(G, L.ent2[e]) : L.ent[e];
    };
    int64_t c0 = e0 + seg;
    uint4 E0 = entry(c0), E1 = entry(c0 + kNtBand);
    float v0 = c0 < e1 ? in[E0.x] : 0.0f;
    for (; c0 < e1; c0 += kNtBand) {
      const float v1 = c0 + kNtBand < e1 ? in[E1.x] : 0.0f;
      const uint4 E2 = entry(c0 + 2 * kNtBand);
      if (v0 != 0.0f) {
        const EntryTaps tp = decode_entry(E0.y, E0.z, G.x_frac_bits);
        spread_taps(acc, wc, cols.x, nr, tp, static_cast<double>(v0) * __uint_as_float(E0.w) * scale);
      }
      E0 = E1;
      E1 = E2;
      v0 = v1;
    }
  }
  __syncthreads();
  // the chunk's partial rows, R x wc (rows past nr unused), each exact sum
  // rounded to float32; NaN throughout for a non-finite input, which the
  // row FFTs carry into every row (and the column pass into every column)
  const double inv = scale > 0.0 ? 1.0 / scale : 0.0;
  float* dst = G.Hp + L.chunk_hp[chunk];
  for (int i = threadIdx.x; i < nr * wc; i += kNtBand)
    dst[i] = finite ? static_cast<float>(static_cast<double>(static_cast<long long>(acc[i])) * inv)
                    : __int_as_float(0x7fc00000);
}

static_assert(kMaxBandRows >= 2 && (kMaxBandRows & (kMaxBandRows - 1)) == 0,
              "band heights are powers of two");

// log2 of a band's row-pair count, for pair counts 1, 2, 4, ... (the last
// band of a plan may hold fewer rows; its pair count is rounded up to a
// power of two and the missing pairs are skipped)
__device__ __forceinline__ int pair_shift(int npair) {
  return 31 - __clz(npair) + ((npair & (npair - 1)) ? 1 : 0);
}

// Row FFT of row_rows rows of a band (item i: band i >> row_sub_shift, the
// rows from (i mod 2^row_sub_shift) * row_rows on): the sum of the band's
// chunks' float32 partials of those rows, in chunk order, rows
// (2p, 2p+1) into complex pair p, FFT along the angle, and the k1 < K1 half
// spectrum of both rows to S.  Dynamic LDS: the pairs, then the FFT scratch
// (if any).
template <int MODE, bool BATCH>
__global__ __launch_bounds__(kNtBand, 6) void k_rowfft(DevGeo one,
                                                       const DevGeo* __restrict__ geos,
                                                       const int2* __restrict__ items) {
  extern __shared__ float2 lds[];
  __shared__ float2 s_tw[kTwLds];
  const Work w = work_item<BATCH>(one, geos, items);
  if (w.i < 0) return;  // a gap in the XCD-ordered items
  const DevGeo& G = w.G;
  const DevList& L = G.lists[MODE == 0 ? kDataSpread : kRadonSpread];
  const int band = w.i >> G.row_sub_shift;
  const int r0 = (w.i & ((1 << G.row_sub_shift) - 1)) * G.row_rows;  // first row in the band
  load_twiddles<kNtBand>(s_tw, G.tw_t, G.Mt);
  const int n0 = G.u0 + band * G.R + r0;
  const int nr = min(G.row_rows, G.u1 - n0);
  const int npair = nr >> 1;
  const int Mt = G.Mt, W = G.W, SP = padded_len(G.Mt);
  const int q0 = L.band_chunk[band], q1 = L.band_chunk[band + 1];
  // angle columns outside the window hold no point: zero
  for (int p = 0; p < npair; ++p)
    for (int m = threadIdx.x; m < Mt; m += kNtBand)
      if (m < G.xw0 || m >= G.xw0 + W) lds[p * SP + lpad(m)] = make_float2(0.0f, 0.0f);
  // the window: the sum over the band's chunks, in chunk order, of their
  // float32 partials; chunk q holds rows x columns [c_lo, c_lo + wc) of the
  // band (c_lo, wc multiples of 4, so a 16-byte group never crosses a row
  // or a chunk's edge).  Work unit j: row j / W4 of the item, columns
  // 4 (j mod W4) .. +3; a thread holds kGroups units and loads them from
  // kQ chunks at a time (a chunk that does not cover a unit adds zero).
  {
    constexpr int kGroups = 3, kQ = 2;
    const int W4 = W >> 2;
    const int n4 = 2 * npair * W4;
    const unsigned m_w4 = div_magic(W4);
    float* ldsf = reinterpret_cast<float*>(lds);
    for (int j0 = threadIdx.x; j0 < n4; j0 += kNtBand * kGroups) {
      float4 acc[kGroups];
      int rr[kGroups], cc[kGroups];
#pragma unroll
      for (int g = 0; g < kGroups; ++g) {
        acc[g] = make_float4(0.f, 0.f, 0.f, 0.f);
        const int j = j0 + g * kNtBand;
        rr[g] = div_small(j, m_w4);
        cc[g] = 4 * (j - rr[g] * W4);
      }
      for (int q = q0; q < q1; q += kQ) {
        float4 v[kQ][kGroups];
#pragma unroll
        for (int s = 0; s < kQ; ++s) {
          const bool has = q + s < q1;
          const int2 cq = has ? L.chunk_col[q + s] : make_int2(0, 0);
          const float* part = G.Hp + (has ? L.chunk_hp[q + s] : 0) + static_cast<size_t>(r0) * cq.y;
#pragma unroll
          for (int g = 0; g < kGroups; ++g) {
            const int c = cc[g] - cq.x;
            v[s][g] = (j0 + g * kNtBand < n4 && c >= 0 && c < cq.y)
                          ? *reinterpret_cast<const float4*>(part + rr[g] * cq.y + c)
                          : make_float4(0.f, 0.f, 0.f, 0.f);
          }
        }
#pragma unroll
        for (int s = 0; s < kQ; ++s) {
#pragma unroll
          for (int g = 0; g < kGroups; ++g) {
            acc[g].x += v[s][g].x;
            acc[g].y += v[s][g].y;
            acc[g].z += v[s][g].z;
            acc[g].w += v[s][g].w;
          }
        }
      }
#pragma unroll
      for (int g = 0; g < kGroups; ++g) {
        if (j0 + g * kNtBand < n4) {
          const int r = rr[g];
          float* dst = ldsf + 2 * ((r >> 1) * SP) + (r & 1);
          const float a[4] = {acc[g].x, acc[g].y, acc[g].z, acc[g].w};
#pragma unroll
          for (int t = 0; t < 4; ++t) dst[2 * lpad(G.xw0 + cc[g] + t)] = a[t];
        }
      }
    }
  }
  __syncthreads();
  fft_rows<kNtBand, kInplaceValues, false>(lds, SP, npair,
                                           fft_scratch(reinterpret_cast<char*>(lds), G.row_scratch),
                                           G.row_group, G.ft, s_tw);
  // two real rows per complex sequence: X1 = (Z[k] + conj Z[-k])/2,
  // X2 = (Z[k] - conj Z[-k])/(2i); keep k1 < K1
  const int psh = pair_shift(npair);
  for (int idx = threadIdx.x; idx < (G.K1 << psh); idx += kNtBand) {
    const int k = idx >> psh;
    const int p = idx & ((1 << psh) - 1);
    if (p >= npair) continue;
    const float2 Z = lds[p * SP + lpad(k)];
    const float2 Zm = lds[p * SP + lpad(k == 0 ? 0 : Mt - k)];
    const float4 o = make_float4(0.5f * (Z.x + Zm.x), 0.5f * (Z.y - Zm.y),
                                 0.5f * (Z.y + Zm.y), -0.5f * (Z.x - Zm.x));
    *reinterpret_cast<float4*>(G.S + static_cast<size_t>(k) * G.Mr + n0 + 2 * p) = o;
  }
}

// Column pass (item i = columns [i col_batch, (i+1) col_batch) of the kept
// k1): FFT along the log radius, multiply by K (conj K for the adjoint;
// K(k1, -k2) = conj K(k1, k2)), normalise, inverse FFT; only the used rows
// [u0, u1) come from and go back to S.  Dynamic LDS: the columns, then the
// FFT scratch (if any).
template <bool ADJ, bool BATCH>
__global__ __launch_bounds__(kNtCol, 2) void k_colfft(DevGeo one, const DevGeo* __restrict__ geos,
                                                      const int2* __restrict__ items) {
  extern __shared__ float2 lds[];
  __shared__ float2 s_tw[kTwLds];
  const Work w = work_item<BATCH>(one, geos, items);
  const DevGeo& G = w.G;
  load_twiddles<kNtCol>(s_tw, G.tw_r, G.Mr);
  const int c0 = w.i * G.col_batch;
  const int nc = min(G.col_batch, G.K1 - c0);
  const int Mr = G.Mr, SP = padded_len(G.Mr);
  float2* S = G.S;
  const int u0 = G.u0, U = G.u1 - G.u0, K2 = G.K2;
  // K(k1, k2) for |k2| < K2 at position n of the column (its conjugate as
  // the sign of k2 and the direction ask), zero outside
  auto kval = [&](const float2* kc, int n) {
    const int k = (n < Mr / 2) ? n : n - Mr;
    const int ak = k < 0 ? -k : k;
    float2 kv = make_float2(0.f, 0.f);
    if (ak < K2) {
      kv = kc[ak];
      if ((k < 0) != ADJ) kv.y = -kv.y;
    }
    return kv;
  };
  auto kmul = [&](float2* lc, int n, float2 kv) {
    const int ak = n < Mr / 2 ? n : Mr - n;
    lc[lpad(n)] = ak < K2 ? cscale(cmul(lc[lpad(n)], kv), G.knorm) : make_float2(0.f, 0.f);
  };
  // One column of at most kKRegs * kNtCol points: the raw K values of its
  // points are loaded into registers first (unconditionally, from an index
  // clamped into the row, so that no load waits for another), and arrive
  // while the column loads and the forward FFT run (barriers wait for LDS
  // only); sign and range are applied at the multiply.
  constexpr int kKRegs = 16;
  const bool kpre = nc == 1 && Mr <= kKRegs * kNtCol;
  float2 kr[kKRegs];
  if (kpre) {
    const float2* kc = G.K + static_cast<size_t>(c0) * K2;
#pragma unroll
    for (int g = 0; g < kKRegs; ++g) {
      const int n = min(static_cast<int>(threadIdx.x) + g * kNtCol, Mr - 1);
      const int ak = n < Mr / 2 ? n : Mr - n;
      kr[g] = kc[min(ak, K2 - 1)];
    }
  }
  float2* cscr = G.col_inplace ? nullptr : lds + SP;
  // where the forward FFT's last pass gives thread t exactly the outputs
  // t + r kNtCol (one butterfly per thread over all kNtCol threads), the
  // multiply by K is done on them before they are stored (their K values
  // are the thread's registers kr[r]); the first pass then also reads the
  // column straight from S, and the inverse's last pass stores it there
  const bool fused = kpre && cscr == nullptr && Mr == kNtCol * fft_radix(G.fr, G.fr.npass - 1);
  if (!fused) {
    for (int c = 0; c < nc; ++c) {
      const float2* col = S + static_cast<size_t>(c0 + c) * Mr;
      float2* lc = lds + c * SP;
      grouped_for<kNtCol, 8>(
          Mr,
          [&](int n) { return (n >= u0 && n < u0 + U) ? col[n] : make_float2(0.f, 0.f); },
          [&](int n, float2 v) { lc[lpad(n)] = v; });
    }
    __syncthreads();
  }
  if (fused) {
    const float2* col = S + static_cast<size_t>(c0) * Mr;
    fft_inplace_hooks<kNtCol, kInplaceValues, false>(
        lds, SP, 1, G.fr, s_tw,
        make_pre([&](int, int n) { return (n >= u0 && n < u0 + U) ? col[n] : make_float2(0.f, 0.f); }),
        make_post<false>([&](int, int n, int r, float2& x) {
          float2 kv = kr[r];  // n = threadIdx.x + r * kNtCol
          if ((n >= Mr / 2) != ADJ) kv.y = -kv.y;  // as in kval: k2 < 0 takes conj K
          const int ak = n < Mr / 2 ? n : Mr - n;
          x = ak < K2 ? cscale(cmul(x, kv), G.knorm) : make_float2(0.f, 0.f);
        }));
  } else {
    fft_rows<kNtCol, kInplaceValues, false>(lds, SP, nc, cscr, nc, G.fr, s_tw);
    if (kpre) {
#pragma unroll
      for (int g = 0; g < kKRegs; ++g) {
        const int n = static_cast<int>(threadIdx.x) + g * kNtCol;
        float2 kv = kr[g];
        if ((n >= Mr / 2) != ADJ) kv.y = -kv.y;  // as in kval: k2 < 0 takes conj K
        if (n < Mr) kmul(lds, n, kv);
      }
    } else {
      for (int c = 0; c < nc; ++c) {
        const float2* kc = G.K + static_cast<size_t>(c0 + c) * K2;
        float2* lc = lds + c * SP;
        grouped_for<kNtCol, 8>(
            Mr, [&](int n) { return kval(kc, n); }, [&](int n, float2 kv) { kmul(lc, n, kv); });
      }
    }
    __syncthreads();
  }
  if (fused) {
    // the inverse's last pass stores the used rows straight to S
    float2* col = S + static_cast<size_t>(c0) * Mr;
    fft_inplace_hooks<kNtCol, kInplaceValues, true>(
        lds, SP, 1, G.fr, s_tw, NoPre(), make_post<true>([&](int, int n, int, float2& x) {
          if (n >= u0 && n < u0 + U) col[n] = x;
        }));
    return;
  }
  fft_rows<kNtCol, kInplaceValues, true>(lds, SP, nc, cscr, nc, G.fr, s_tw);
  for (int c = 0; c < nc; ++c) {
    float2* col = S + static_cast<size_t>(c0 + c) * Mr + u0;
    const float2* lc = lds + c * SP;
    grouped_for<kNtCol, 8>(
        U, [&](int n) { return lc[lpad(u0 + n)]; }, [&](int n, float2 v) { col[n] = v; });
  }
}

// Inverse row FFT of row_rows rows of a band (item i as in k_rowfft):
// Z = X1 + i X2 for rows
// (2p, 2p+1) with the Hermitian completion Z[-k], inverse FFT along the
// angle, real rows to Cr (window columns only).  Dynamic LDS: the pairs,
// then the FFT scratch.
template <bool BATCH>
__global__ __launch_bounds__(kNtBand, 6) void k_rowifft(DevGeo one,
                                                        const DevGeo* __restrict__ geos,
                                                        const int2* __restrict__ items) {
  extern __shared__ float2 lds[];
  __shared__ float2 s_tw[kTwLds];
  const Work w = work_item<BATCH>(one, geos, items);
  if (w.i < 0) return;  // a gap in the XCD-ordered items
  const DevGeo& G = w.G;
  const int band = w.i >> G.row_sub_shift;
  const int r0 = (w.i & ((1 << G.row_sub_shift) - 1)) * G.row_rows;  // first row in the band
  load_twiddles<kNtBand>(s_tw, G.tw_t, G.Mt);
  const int n0 = G.u0 + band * G.R + r0;
  const int nr = min(G.row_rows, G.u1 - n0);
  const int npair = nr >> 1;
  const int Mt = G.Mt, SP = padded_len(G.Mt), W = G.W;
  // the half spectra k < K1 of both rows of each pair (and through them
  // the pair's spectrum at Mt - k) come from S; the frequencies K1 .. Mt - K1
  // in between are zero.  The loads of the first group are issued before the
  // zero fill, which touches other slots, so one barrier closes both.
  const int psh = pair_shift(npair);
  const int nk = G.K1 << psh;
  constexpr int kG = 4;
  for (int i0 = threadIdx.x; i0 < nk || i0 == static_cast<int>(threadIdx.x); i0 += kNtBand * kG) {
    float4 x[kG];
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      const int idx = i0 + g * kNtBand;
      const int k = idx >> psh;
      const int p = idx & ((1 << psh) - 1);
      x[g] = (idx < nk && p < npair)
                 ? *reinterpret_cast<const float4*>(G.S + static_cast<size_t>(k) * G.Mr + n0 + 2 * p)
                 : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (i0 == static_cast<int>(threadIdx.x)) {
      const int gap = Mt - 2 * G.K1 + 1;  // frequencies K1 .. Mt - K1
      const unsigned m_gap = div_magic(gap);
      for (int i = threadIdx.x; i < npair * gap; i += kNtBand) {
        const int p = div_small(i, m_gap);
        lds[p * SP + lpad(G.K1 + i - p * gap)] = make_float2(0.f, 0.f);
      }
    }
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      const int idx = i0 + g * kNtBand;
      const int k = idx >> psh;
      const int p = idx & ((1 << psh) - 1);
      if (idx < nk && p < npair) {
        // X1 = (x.x, x.y), X2 = (x.z, x.w)
        lds[p * SP + lpad(k)] = make_float2(x[g].x - x[g].w, x[g].y + x[g].z);
        if (k > 0) lds[p * SP + lpad(Mt - k)] = make_float2(x[g].x + x[g].w, x[g].z - x[g].y);
      }
    }
  }
  __syncthreads();
  float* dst = G.Cr + static_cast<size_t>(n0 - G.u0) * W;
  if (G.row_scratch < 0 && G.row_group >= npair) {
    // all pairs in place at once: the last pass stores the window columns of
    // both rows of each pair straight to Cr
    fft_inplace_hooks<kNtBand, kInplaceValues, true>(
        lds, SP, npair, G.ft, s_tw, NoPre(), make_post<true>([&](int p, int m, int, float2& z) {
          const int c = m - G.xw0;
          if (c >= 0 && c < W) {
            float* d = dst + (2 * p) * W;
            d[c] = z.x;
            d[W + c] = z.y;
          }
        }));
    return;
  }
  fft_rows<kNtBand, kInplaceValues, true>(lds, SP, npair,
                                          fft_scratch(reinterpret_cast<char*>(lds), G.row_scratch),
                                          G.row_group, G.ft, s_tw);
  for (int p = 0; p < npair; ++p) {
    const float2* lp = lds + p * SP;
    float* d = dst + (2 * p) * W;
    grouped_for<kNtBand, 4>(
        W, [&](int c) { return lp[lpad(G.xw0 + c)]; },
        [&](int c, float2 z) {
          d[c] = z.x;
          d[W + c] = z.y;
        });
  }
}

// Gather for one chunk of a band's owned list (item i = chunk i; MODE 0:
// into g[nq][ntau]; MODE 1: into f[nx][nt], plus zeros outside the
// trapezoid, traces dealt over the chunks; a part of a split stores into
// its place in the whole arrays, zero-fills only its data band, and with
// `accumulate` adds to the output and fills nothing).  Dynamic LDS: rows [L0, L1) of
// Cr, the band's rows and the halo its points' stencils reach.  One point per
// thread, consecutive threads on consecutive entries.
template <int MODE, bool BATCH>
__global__ __launch_bounds__(kNtBand) void k_gather(DevGeo one, const DevGeo* __restrict__ geos,
                                                    const int2* __restrict__ items,
                                                    float* __restrict__ out_base) {
  extern __shared__ float rows[];
  __shared__ float s_wave[kNtBand / 64];
  const Work w = work_item<BATCH>(one, geos, items);
  if (w.i < 0) return;  // a gap in the XCD-ordered items
  const DevGeo& G = w.G;
  const DevList& L = G.lists[MODE == 0 ? kRadonOwn : kDataOwn];
  float* out = out_base + (MODE == 0 ? G.radon_off : G.data_off);
  const int chunk = w.i;
  const int band = L.chunk_band[chunk];
  const int n0 = G.u0 + band * G.R;
  const int nr = min(G.R, G.u1 - n0);
  const int L0 = max(G.u0, n0 - 1);
  const int L1 = min(G.u1, n0 + nr + 2);
  const int W = G.W;
  const float4* src = reinterpret_cast<const float4*>(G.Cr + static_cast<size_t>(L0 - G.u0) * W);
  float4* rows4 = reinterpret_cast<float4*>(rows);
  for (int i = threadIdx.x; i < (L1 - L0) * W / 4; i += kNtBand) rows4[i] = src[i];
  __syncthreads();
  const int64_t e0 = L.chunk_off[chunk], e1 = L.chunk_off[chunk + 1];
  const int shift = n0 - L0;  // held row of lattice row n0
  const int nheld = L1 - L0;
  float vmax = 0.0f;  // largest |output| of this thread (forward)
  // each thread's next entry is in flight while it interpolates the current
  // one (indices clamped into the chunk, into entry 0 for an empty chunk:
  // every device list holds at least one entry; a load past the end is
  // never used)
  const int64_t last = e1 > 0 ? e1 - 1 : 0;
  // (the forward's Radon points come as compact entries, expanded once
  // they have arrived)
  auto raw = [&](int64_t k) {
    if (MODE == 0) {
      const uint2 c = L.ent2[k];
      return make_uint4(c.x, c.y, 0u, 0u);
    }
    return L.ent[k];
  };
  uint4 En = raw(min(e0 + static_cast<int64_t>(threadIdx.x), last));
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kNtBand) {
    const uint4 E = MODE == 0 ? radon_entry(G, make_uint2(En.x, En.y)) : En;
    En = raw(min(e + kNtBand, last));
    const EntryTaps tp = decode_entry(E.y, E.z, G.x_frac_bits);
    float acc = 0.0f;
    // the four tap rows without branches: a row outside the held ones
    // (beyond the used lattice rows) reads held row 0 with weight 0
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      const int rl = tp.cy + shift + bb;
      const bool held = rl >= 0 && rl < nheld;
      const float* r = rows + (held ? rl : 0) * W + tp.cx;
      const float wy = held ? tp.wy[bb] : 0.0f;
      acc += wy * (r[0] * tp.wx[0] + r[1] * tp.wx[1] + r[2] * tp.wx[2] + r[3] * tp.wx[3]);
    }
    const float v = __uint_as_float(E.w) * acc;
    out[E.x] = G.accumulate ? out[E.x] + v : v;
    if (MODE == 0) vmax = fmaxf(vmax, fabsf(v) <= 3.0e38f ? fabsf(v) : INFINITY);
  }
  if (MODE == 0 && G.gmax) {
    vmax = block_max(vmax, s_wave);
    if (threadIdx.x == 0) G.gmax[chunk] = vmax;
  }
  if (MODE == 1 && !G.accumulate) {
    for (int k = chunk; k < G.nx_fill; k += L.nchunks) {
      float* fk = out + static_cast<size_t>(k) * G.data_ld;
      const int j1 = min(G.jmin[k], G.j_hi);
      for (int j = G.j_lo + threadIdx.x; j < j1; j += kNtBand) fk[j] = 0.0f;
    }
  }
}

}  // namespace hrt
