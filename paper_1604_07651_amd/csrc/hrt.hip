// gfx950 kernels and C ABI of the log-polar hyperbolic Radon transform.
//
// One direction of the transform is three kernels over an Mt x Mr lattice
// (angle theta x log radius rho) whose rows [u0, u1) are all that any point
// touches.  Only the non-negative half spectrum along theta inside the band
// limit L (k1 < K1) ever reaches HBM, stored column-major as S[k1][row]:
//
//   spread_rowfft    one workgroup per band of R rows: cubic B-spline smearing
//                    of every point whose stencil reaches the band into LDS
//                    (eq. B3tx2 for data samples, or the Radon samples for
//                    the adjoint), two real rows per complex FFT along theta,
//                    store k1 < K1.
//   colfft           one workgroup per kept k1: FFT along rho, multiply by the
//                    kernel multiplier K (eq. lok / B3tauq; its conjugate for
//                    the adjoint), inverse FFT along rho.
//   rowifft_gather   one workgroup per band: Hermitian completion and inverse
//                    FFT along theta of the band plus a 3-row halo, then the
//                    4x4 B-spline interpolation at every point the band owns
//                    (eq. B3tauq for Radon samples; data samples times their
//                    smear weight for the adjoint).
//
// Point coordinates are generated in float64 from the closed-form maps
// (eqs. transformT, transformP; the Radon side e^rho = A_l + B_l tau^2) and
// split into an integer cell and a float32 fraction; everything on the
// lattice is float32 with float32 accumulation.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "fft.hpp"
#include "hrt.h"
#include "plan.hpp"

namespace hrt {

constexpr int kNtBand = 512;                // threads of the band kernels
constexpr int kNtCol = 256;                 // threads of the column kernel
constexpr int kAbsMaxBlocks = 256;          // partial maxima of the input
constexpr uint64_t kMagic = 0x6872745f706c616eull;

struct DevGeo {
  int nt, nx, ntau, nq;
  double dt, x0, dx, tau0, dtau, T, X;
  double a, O1, O2, ca, sa, AeA;
  double inv_dtheta, inv_drho, drho, ctheta, crho;
  double wconst;  // 2 a^2 (dt/T)(dx/X): smear weight without t^, trapezoid, 1/|p|
  int Mt, Mr, K1, K2, u0, u1, R, nbands;
  int grp1, grp3;  // FFT scratch sequences after the band data in LDS
  float knorm;
  float wmax_data, wmax_radon;  // bounds on the smear weights of the two point sets    // 1/(Mt Mr): both inverse FFTs are unnormalised
  const int* jmin;
  const double* qA;
  const double* qB;
  const int* q_i0;
  const float4* q_w;
  const float* q_scale;
};

// ---------------------------------------------------------------- points --

__device__ __forceinline__ void bspline4(float f, float w[4]) {
  const float g = 1.0f - f;
  w[0] = g * g * g * (1.0f / 6.0f);
  w[1] = 2.0f / 3.0f - f * f + 0.5f * f * f * f;
  w[2] = 2.0f / 3.0f - g * g + 0.5f * g * g * g;
  w[3] = f * f * f * (1.0f / 6.0f);
}

// The point cursors below move from an anchor sample by small increments;
// these series are exact to float64 rounding for increments up to kSmall.
constexpr double kSmall = 0.01;

// atan(z), |z| <= 0.01: Taylor series to z^9 (truncation < 1e-19 |z|).
__device__ __forceinline__ double atan_small(double z) {
  const double z2 = z * z;
  double p = 1.0 / 9.0;
  p = fma(p, -z2, 1.0 / 7.0);
  p = fma(p, -z2, 1.0 / 5.0);
  p = fma(p, -z2, 1.0 / 3.0);
  p = fma(p, -z2, 1.0);
  return z * p;
}

// log(1 + x), |x| <= 0.01: Taylor series to x^8 (truncation < 2e-17 |x|).
__device__ __forceinline__ double log1p_small(double x) {
  double p = -1.0 / 8.0;
  p = fma(p, x, 1.0 / 7.0);
  p = fma(p, x, -1.0 / 6.0);
  p = fma(p, x, 1.0 / 5.0);
  p = fma(p, x, -1.0 / 4.0);
  p = fma(p, x, 1.0 / 3.0);
  p = fma(p, x, -1.0 / 2.0);
  p = fma(p, x, 1.0);
  return x * p;
}

// 1/d for d within 10 % of 1: hardware reciprocal and two Newton steps.
__device__ __forceinline__ double rcp_near1(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return r;
}

// round(v * scale) as a 64-bit integer for |v * scale| < 2^51: adding
// 1.5 * 2^52 leaves the rounded integer in the low mantissa bits.
__device__ __forceinline__ unsigned long long to_fixed(float v, double scale) {
  const double d = fma(static_cast<double>(v), scale, 6755399441055744.0);
  return static_cast<unsigned long long>(__double_as_longlong(d) - 0x4338000000000000ll);
}

// Data sample (j, k) of one trace: lattice coordinates of
// (t^2, x^2) -> T -> P1 and the smear weight 2 a^2 t^ e^-eta w_t w_x dt^ dx^
// (the 1/(2 sqrt y) of eq. f times the Jacobian, trapezoid rule).
//
// A thread walks consecutive samples of a trace.  Along trace k the mapped
// point moves on a straight line, p_j = p_a + delta e_alpha with
// delta = a (s_j - s_a), so from an anchor sample a evaluated in full
// (atan2, log) the next samples follow from
//   tan(phi_j - phi_a) = delta q1 / (1 + delta q2),
//   |p_j|^2 / |p_a|^2 = 1 + delta (2 q2 + delta / |p_a|^2),
// q1 = (p_a x e_alpha)/|p_a|^2, q2 = (p_a . e_alpha)/|p_a|^2, with short
// float64 series for atan and log1p.  Exact to float64 rounding; a new
// anchor is taken on a new trace or when the increments leave the series'
// range.
struct DataCursor {
  int k = -1;
  double tha, xga, yga, q1, q2;
  float inv_r2;  // enters only the second-order term of |p_j|^2
  float wa;      // wconst * (trapezoid weight in x of trace k) / |p_a|

  __device__ __forceinline__ void anchor(const DevGeo& G, int j, int kk) {
    k = kk;
    tha = (static_cast<double>(j) * G.dt) / G.T;
    const double xh = (G.x0 + static_cast<double>(kk) * G.dx) / G.X;
    const double ds = tha * tha - 0.5, dy = xh * xh - 0.5;
    const double u = G.a * (G.ca * ds - G.sa * dy) + G.O1;
    const double v = G.a * (G.sa * ds + G.ca * dy) + G.O2;
    const double r2 = u * u + v * v;
    xga = atan2(v, u) * G.inv_dtheta + G.ctheta;
    yga = 0.5 * log(r2) * G.inv_drho + G.crho;
    const double ir2 = 1.0 / r2;
    inv_r2 = static_cast<float>(ir2);
    q1 = (u * G.sa - v * G.ca) * ir2;
    q2 = (u * G.ca + v * G.sa) * ir2;
    wa = static_cast<float>(G.wconst * ((kk == 0 || kk == G.nx - 1) ? 0.5 : 1.0) * sqrt(ir2));
  }

  __device__ __forceinline__ void eval(const DevGeo& G, int j, int kk, double& xg,
                                       double& yg, float& w) {
    const double th = (static_cast<double>(j) * G.dt) / G.T;
    const double wt = (j == G.nt - 1) ? 0.5 : 1.0;
    if (kk == k) {
      const double delta = G.a * ((th - tha) * (th + tha));
      const double z = delta * q1 * rcp_near1(1.0 + delta * q2);
      const double x = delta * (2.0 * q2 + delta * static_cast<double>(inv_r2));
      if (fabs(z) <= kSmall && fabs(x) <= kSmall) {
        xg = xga + atan_small(z) * G.inv_dtheta;
        yg = yga + 0.5 * log1p_small(x) * G.inv_drho;
        w = wa * static_cast<float>(th * wt) * rsqrtf(1.0f + static_cast<float>(x));
        return;
      }
    }
    anchor(G, j, kk);
    xg = xga;
    yg = yga;
    w = wa * static_cast<float>(th * wt);
  }
};

// Radon sample (l, i) of one slowness column: e^rho = A_l + B_l tau^2, from
// an anchor sample by log1p of the relative change (the same anchoring as
// DataCursor).
struct RadonCursor {
  int l = -1;
  double A, B, tha, inv_ea, yga;

  __device__ __forceinline__ double eval(const DevGeo& G, double Al, double Bl, int i,
                                         int ll) {
    const double th = (G.tau0 + static_cast<double>(i) * G.dtau) / G.T;
    if (ll == l) {
      const double x = B * ((th - tha) * (th + tha)) * inv_ea;
      if (fabs(x) <= kSmall) return yga + log1p_small(x) * G.inv_drho;
    }
    l = ll;
    A = Al;
    B = Bl;
    tha = th;
    const double ea = A + B * (th * th);
    inv_ea = 1.0 / ea;
    yga = log(ea) * G.inv_drho + G.crho;
    return yga;
  }
};

// Time samples j of trace k whose log radius may fall in [Ylo, Yhi)
// (lattice units), from |p(s)|^2 = c0 + c1 s + c2 s^2 along the trace,
// s = t^2.  A superset with a one-sample margin: the kernels re-check every
// point.
__device__ __forceinline__ double trace_j_at(const DevGeo& G, double c0,
                                             double c1, double c2, double Y) {
  const double r2 = exp(2.0 * (Y - G.crho) * G.drho);
  const double disc = c1 * c1 + 4.0 * c2 * (r2 - c0);
  if (disc <= 0.0) return 0.0;
  const double s = 2.0 * (r2 - c0) / (c1 + sqrt(disc));
  if (s <= 0.0) return 0.0;
  return fmin(sqrt(s) * (G.nt - 1), 1e9);
}

__device__ __forceinline__ void data_range(const DevGeo& G, int k, double Ylo,
                                           double Yhi, int& jlo, int& jhi) {
  const double xh = (G.x0 + static_cast<double>(k) * G.dx) / G.X;
  const double dy = xh * xh - 0.5;
  const double pu = G.a * (G.ca * -0.5 - G.sa * dy) + G.O1;
  const double pv = G.a * (G.sa * -0.5 + G.ca * dy) + G.O2;
  const double c0 = pu * pu + pv * pv;
  const double c1 = 2.0 * G.a * (pu * G.ca + pv * G.sa);
  const double c2 = G.a * G.a;
  const int lo = static_cast<int>(ceil(trace_j_at(G, c0, c1, c2, Ylo))) - 1;
  const int hi = static_cast<int>(ceil(trace_j_at(G, c0, c1, c2, Yhi))) + 1;
  jlo = max(G.jmin[k], lo);
  jhi = min(G.nt, hi);
}

__device__ __forceinline__ void radon_range(const DevGeo& G, double A, double B,
                                            double Ylo, double Yhi, int& ilo,
                                            int& ihi) {
  auto i_at = [&](double Y) {
    const double e = exp((Y - G.crho) * G.drho);
    const double t2 = (e - A) / B;
    if (t2 <= 0.0) return -1e9;
    return fmin((sqrt(t2) * G.T - G.tau0) / G.dtau, 1e9);
  };
  ilo = max(0, static_cast<int>(ceil(i_at(Ylo))) - 1);
  ihi = min(G.ntau, static_cast<int>(ceil(i_at(Yhi))) + 1);
}

// Per-thread accumulator of the 4x4 B-spline taps of consecutive points that
// fall on the same lattice cell (a thread walks consecutive samples of one
// trace or slowness column, and where the lattice is coarse many of them
// share a cell): their taps are summed in registers and reach LDS as one set
// of 16 atomic adds.
//
// The band accumulates in 64-bit fixed point: a tap value v enters as
// round(v * scale) with scale = 2^40 / (bound on |v|), added with the
// integer LDS atomic (float LDS atomics are some 25x slower on gfx950).
// Integer sums are exact and order-independent, so the band is
// deterministic; the quantum is 2^-40 of the largest possible tap.  Rows
// outside the band [n0, n0+nr) are dropped; row r of the band is
// acc64[r * Mt ...].
struct TapAcc {
  int ix = INT_MIN, iy = 0;
  float a[4][4];

  __device__ __forceinline__ void flush(unsigned long long* acc64, int Mt, int n0,
                                        int nr, double scale) {
    if (ix == INT_MIN) return;
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      const int rl = iy - 1 + bb - n0;
      if (rl < 0 || rl >= nr) continue;
      unsigned long long* base = acc64 + rl * Mt + ix;
#pragma unroll
      for (int aa = 0; aa < 4; ++aa)
        atomicAdd(base + aa, to_fixed(a[bb][aa], scale));
    }
    ix = INT_MIN;  // nothing pending
  }

  // add w * B3(x - xg) B3(y - yg) for the point at lattice (xg, yg)
  __device__ __forceinline__ void add(unsigned long long* acc64, int Mt, int n0, int nr,
                                      double scale, int nix, const float wx[4], double yg,
                                      float w) {
    const double fy0 = floor(yg);
    const int niy = static_cast<int>(fy0);
    if (niy + 2 < n0 || niy - 1 >= n0 + nr || nix < 0 || nix + 3 >= Mt) return;
    float wy[4];
    bspline4(static_cast<float>(yg - fy0), wy);
    if (nix != ix || niy != iy) {
      flush(acc64, Mt, n0, nr, scale);
      ix = nix;
      iy = niy;
#pragma unroll
      for (int bb = 0; bb < 4; ++bb)
#pragma unroll
        for (int aa = 0; aa < 4; ++aa) a[bb][aa] = 0.0f;
    }
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      const float wr = w * wy[bb];
#pragma unroll
      for (int aa = 0; aa < 4; ++aa) a[bb][aa] += wr * wx[aa];
    }
  }
};

// Taps outside the rows [L0, L1) held in LDS or outside the angle axis are
// skipped (no point the band owns reaches them).
__device__ __forceinline__ float gather_taps(const float* ldsf, int Mt, int L0,
                                             int L1, int ix, const float wx[4],
                                             int iy, const float wy[4]) {
  float acc = 0.0f;
  if (ix < 0 || ix + 3 >= Mt) return acc;
#pragma unroll
  for (int bb = 0; bb < 4; ++bb) {
    const int rl = iy - 1 + bb - L0;
    if (rl < 0 || iy - 1 + bb >= L1) continue;
    const float* base = ldsf + ((rl >> 1) * Mt + ix) * 2 + (rl & 1);
    float row = 0.0f;
#pragma unroll
    for (int aa = 0; aa < 4; ++aa) row += base[2 * aa] * wx[aa];
    acc += row * wy[bb];
  }
  return acc;
}

// ---------------------------------------------------------------- kernels --

// Exclusive prefix sum over the workgroup (kNtBand threads, 64-wide waves).
__device__ __forceinline__ int block_exclusive_scan(int v, int* s_wave, int& total) {
  constexpr int kWaves = kNtBand / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_wave[wid] = x;
  __syncthreads();
  if (wid == 0) {
    int w = (lane < kWaves) ? s_wave[lane] : 0;
#pragma unroll
    for (int o = 1; o < kWaves; o <<= 1) {
      const int y = __shfl_up(w, o, 64);
      if (lane >= o) w += y;
    }
    if (lane < kWaves) s_wave[lane] = w;
  }
  __syncthreads();
  total = s_wave[kWaves - 1];
  return (wid ? s_wave[wid - 1] : 0) + x - v;
}

// Maximum over the workgroup (uses s_wave as scratch).
__device__ __forceinline__ float block_max(float v, int* s_wave) {
  constexpr int kWaves = kNtBand / 64;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  float* sw = reinterpret_cast<float*>(s_wave);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = v;
  __syncthreads();
  float m = sw[0];
#pragma unroll
  for (int i = 1; i < kWaves; ++i) m = fmaxf(m, sw[i]);
  __syncthreads();
  return m;
}

// Shared memory of the balanced point walk.
struct WalkLds {
  int lo[kNtBand];
  int pre[kNtBand + 1];
  int wave[kNtBand / 64];
};

// static LDS of the band kernels (walk tables, twiddles) plus slack
constexpr int64_t kWalkLdsBytes = sizeof(WalkLds) + kTwLds * sizeof(float2) + 512;

// Visits every point idx in [lo_u, hi_u) of every unit u (a trace or a
// slowness column), range(u, lo, hi) giving the superset range of unit u.
// Units are taken kNtBand at a time; the points of a chunk are cut into
// equal contiguous segments, one per thread, so every thread does the same
// amount of work whatever the spread of range lengths.  A thread's segment
// arrives as runs of consecutive points of one unit: run(u, idx0, len).
// Segments are dealt to lanes 16 apart (lane-major), so the lanes of one
// wave work on points far from each other on the lattice.  done() runs once
// per chunk after the thread's last run.
template <class RangeF, class RunF, class DoneF>
__device__ __forceinline__ void balanced_walk(int nunits, WalkLds& w, RangeF range, RunF run,
                                              DoneF done) {
  for (int c0 = 0; c0 < nunits; c0 += kNtBand) {
    const int u = c0 + static_cast<int>(threadIdx.x);
    int lo = 0, cnt = 0;
    if (u < nunits) {
      int hi;
      range(u, lo, hi);
      cnt = max(0, hi - lo);
    }
    int total;
    const int excl = block_exclusive_scan(cnt, w.wave, total);
    w.lo[threadIdx.x] = lo;
    w.pre[threadIdx.x] = excl;
    if (threadIdx.x == 0) w.pre[kNtBand] = total;
    __syncthreads();
    const int per = (total + kNtBand - 1) / kNtBand;
    const int seg = (threadIdx.x & 63) * (kNtBand / 64) + (threadIdx.x >> 6);
    int p = seg * per;
    const int pend = min(p + per, total);
    if (p < pend) {
      int a = 0, b = kNtBand;  // w.pre[a] <= p < w.pre[b]
      while (b - a > 1) {
        const int m = (a + b) >> 1;
        if (w.pre[m] <= p) a = m;
        else b = m;
      }
      int unit = a;
      int next = w.pre[unit + 1];
      while (p < pend) {
        while (p >= next) {
          ++unit;
          next = w.pre[unit + 1];
        }
        const int len = min(pend, next) - p;
        run(c0 + unit, w.lo[unit] + (p - w.pre[unit]), len);
        p += len;
      }
    }
    done();
    __syncthreads();
  }
}

// Calls point(i, value) for the `len` consecutive values in[base + i],
// loading them four at a time so that their latencies overlap.
template <class PointF>
__device__ __forceinline__ void for_run_values(const float* __restrict__ in, size_t base,
                                               int len, PointF point) {
  for (int i0 = 0; i0 < len; i0 += 4) {
    float v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = (i0 + t < len) ? in[base + i0 + t] : 0.0f;
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (i0 + t < len) point(i0 + t, v[t]);
  }
}

// Largest |x| over n floats, as kAbsMaxBlocks partial maxima (no atomics,
// no clearing, so safe to replay); a non-finite input makes its block report
// +inf.
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
// (adjoint).
template <int MODE>
__global__ __launch_bounds__(kNtBand, 4) void k_spread_rowfft(
    DevGeo G, FftDev F, const float2* __restrict__ tw,
    const float* __restrict__ in, const float* __restrict__ absmax,
    float2* __restrict__ S) {
  extern __shared__ float2 lds[];
  __shared__ WalkLds walk;
  __shared__ float2 s_tw[kTwLds];
  load_twiddles<kNtBand>(s_tw, tw, G.Mt);
  unsigned long long* acc64 = reinterpret_cast<unsigned long long*>(lds);
  const int n0 = G.u0 + static_cast<int>(blockIdx.x) * G.R;
  const int nr = min(G.R, G.u1 - n0);
  const int npair = nr >> 1;
  const int Mt = G.Mt;
  const double Ylo = n0 - 2, Yhi = n0 + nr + 1;
  const int nunits = MODE == 0 ? G.nx : G.nq;
  auto range = [&](int u, int& lo, int& hi) {
    if (MODE == 0) data_range(G, u, Ylo, Yhi, lo, hi);
    else radon_range(G, G.qA[u], G.qB[u], Ylo, Yhi, lo, hi);
  };
  const size_t ustride = MODE == 0 ? G.nt : G.ntau;

  // largest |input| (from k_absmax) fixes the fixed-point scale
  float vmax = 0.0f;
  for (int i = threadIdx.x; i < kAbsMaxBlocks; i += kNtBand) vmax = fmaxf(vmax, absmax[i]);
  vmax = block_max(vmax, walk.wave);
  const float wmax = MODE == 0 ? G.wmax_data : G.wmax_radon;
  const bool finite = vmax <= 3.0e38f;  // false for inf and NaN
  const double scale =
      (vmax > 0.0f && finite) ? 1099511627776.0 / (static_cast<double>(wmax) * vmax) : 0.0;
  for (int i = threadIdx.x; i < nr * Mt; i += kNtBand) acc64[i] = 0ull;
  __syncthreads();

  // pass 2: smear every point of the band (skipped when all inputs are 0)
  TapAcc acc;
  auto done = [&]() { acc.flush(acc64, Mt, n0, nr, scale); };
  if (scale > 0.0) {
    if (MODE == 0) {
      DataCursor cur;
      balanced_walk(
          nunits, walk, range,
          [&](int k, int j0, int len) {
            for_run_values(in, static_cast<size_t>(k) * G.nt + j0, len, [&](int t, float val) {
              if (val == 0.0f) return;
              double xg, yg;
              float w;
              cur.eval(G, j0 + t, k, xg, yg, w);
              const double fx0 = floor(xg);
              float wx[4];
              bspline4(static_cast<float>(xg - fx0), wx);
              acc.add(acc64, Mt, n0, nr, scale, static_cast<int>(fx0) - 1, wx, yg, w * val);
            });
          },
          done);
    } else {
      // per-column constants, reloaded when a thread moves to the next column
      RadonCursor rc;
      balanced_walk(
          nunits, walk, range,
          [&](int l, int i0, int len) {
            const float4 q = G.q_w[l];
            const float wx[4] = {q.x, q.y, q.z, q.w};
            const int ix = G.q_i0[l];
            const float sc = G.q_scale[l];
            const double A = G.qA[l], B = G.qB[l];
            for_run_values(in, static_cast<size_t>(l) * G.ntau + i0, len, [&](int t, float val) {
              if (val == 0.0f) return;
              acc.add(acc64, Mt, n0, nr, scale, ix, wx, rc.eval(G, A, B, i0 + t, l), sc * val);
            });
          },
          done);
    }
  }
  __syncthreads();
  // fixed point -> float, rows (2p, 2p+1) into complex pair p, in place: the
  // float pair at index p*Mt + m overwrites 64-bit cell p*Mt + m, which this
  // same thread has already read (pairs in increasing order)
  const float inv = scale > 0.0 ? static_cast<float>(1.0 / scale) : 0.0f;
  const float bad = finite ? 0.0f : __int_as_float(0x7fc00000);
  for (int m = threadIdx.x; m < Mt; m += kNtBand) {
    for (int p = 0; p < npair; ++p) {
      const long long lo = static_cast<long long>(acc64[(2 * p) * Mt + m]);
      const long long hi = static_cast<long long>(acc64[(2 * p + 1) * Mt + m]);
      lds[p * Mt + m] = make_float2(static_cast<float>(lo) * inv + bad,
                                    static_cast<float>(hi) * inv + bad);
    }
  }
  __syncthreads();
  fft_batch<kNtBand, false>(lds, Mt, npair, lds + npair * Mt, npair, F, s_tw);
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
template <int MODE>
__global__ __launch_bounds__(kNtBand, 4) void k_rowifft_gather(
    DevGeo G, FftDev F, const float2* __restrict__ tw,
    const float2* __restrict__ S, float* __restrict__ out) {
  extern __shared__ float2 lds[];
  __shared__ WalkLds walk;
  __shared__ float2 s_tw[kTwLds];
  load_twiddles<kNtBand>(s_tw, tw, G.Mt);
  const float* ldsf = reinterpret_cast<const float*>(lds);
  const int n0 = G.u0 + static_cast<int>(blockIdx.x) * G.R;
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
  fft_batch<kNtBand, true>(lds, Mt, npair, lds + ((G.R + 4) / 2) * Mt, G.grp3, F, s_tw);
  const double Ylo = n0, Yhi = n0 + nr;
  if (MODE == 0) {
    RadonCursor rc;
    balanced_walk(
        G.nq, walk,
        [&](int l, int& lo, int& hi) {
          radon_range(G, G.qA[l], G.qB[l], Ylo, Yhi, lo, hi);
        },
        [&](int l, int i0, int len) {
          const float4 q = G.q_w[l];
          const float wx[4] = {q.x, q.y, q.z, q.w};
          const int ix = G.q_i0[l];
          const float sc = G.q_scale[l];
          const double A = G.qA[l], B = G.qB[l];
          float* orow = out + static_cast<size_t>(l) * G.ntau;
          for (int i = i0; i < i0 + len; ++i) {
            const double yg = rc.eval(G, A, B, i, l);
            const double fy0 = floor(yg);
            const int iy = static_cast<int>(fy0);
            if (iy < n0 || iy >= n0 + nr) continue;
            float wy[4];
            bspline4(static_cast<float>(yg - fy0), wy);
            orow[i] = sc * gather_taps(ldsf, Mt, L0, L1, ix, wx, iy, wy);
          }
        },
        []() {});
  } else {
    DataCursor cur;
    balanced_walk(
        G.nx, walk,
        [&](int k, int& lo, int& hi) { data_range(G, k, Ylo, Yhi, lo, hi); },
        [&](int k, int j0, int len) {
          float* orow = out + static_cast<size_t>(k) * G.nt;
          for (int j = j0; j < j0 + len; ++j) {
            double xg, yg;
            float w;
            cur.eval(G, j, k, xg, yg, w);
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
        []() {});
    // samples outside the trapezoid: each trace zeroed by one band
    for (int k = static_cast<int>(blockIdx.x); k < G.nx; k += G.nbands) {
      float* fk = out + static_cast<size_t>(k) * G.nt;
      for (int j = threadIdx.x; j < G.jmin[k]; j += kNtBand) fk[j] = 0.0f;
    }
  }
}

// ---------------------------------------------------- kernel spectrum (plan)

// E1[k1][n] = 2 w_n sec(theta_n) cos(2 pi k1 theta_n / P_theta),
// E2[n][k2] = exp(-2 pi i k2 ln cos(theta_n) / P_rho), nodes on [0, beta_k]
// (the integrand of eq. finiteconv's kernel spectrum is even in theta).
__global__ void k_zeta_tables(int N, int K1, int K2, const double* __restrict__ nodes,
                              const double* __restrict__ weights, double inv_pt,
                              double inv_pr, double* __restrict__ E1,
                              double2* __restrict__ E2) {
  const int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t n1 = static_cast<int64_t>(K1) * N;
  const int64_t n2 = static_cast<int64_t>(K2) * N;
  if (tid < n1) {
    const int k1 = static_cast<int>(tid / N);
    const int n = static_cast<int>(tid - static_cast<int64_t>(k1) * N);
    const double th = nodes[n];
    double x = static_cast<double>(k1) * th * inv_pt;
    x -= floor(x);
    E1[tid] = 2.0 * weights[n] / cos(th) * cospi(2.0 * x);
  } else if (tid < n1 + n2) {
    const int64_t t = tid - n1;
    const int n = static_cast<int>(t / K2);
    const int k2 = static_cast<int>(t - static_cast<int64_t>(n) * K2);
    double x = static_cast<double>(k2) * log(cos(nodes[n])) * inv_pr;
    x -= floor(x);
    double s, c;
    sincospi(2.0 * x, &s, &c);
    E2[t] = make_double2(c, -s);
  }
}

// K[k1][k2] = s1[k1] s2[k2] c * sum_n E1[k1][n] E2[n][k2] (float64, tiled)
__global__ __launch_bounds__(256) void k_zeta_gemm(int N, int K1, int K2,
                                                   const double* __restrict__ E1,
                                                   const double2* __restrict__ E2,
                                                   const double* __restrict__ s1,
                                                   const double* __restrict__ s2,
                                                   double c, float2* __restrict__ K) {
  constexpr int TB = 16, TN = 32;
  __shared__ double a[TB][TN + 1];
  __shared__ double2 b[TN][TB];
  const int tx = threadIdx.x % TB, ty = threadIdx.x / TB;
  const int k1 = blockIdx.y * TB + ty;
  const int k2 = blockIdx.x * TB + tx;
  double re = 0.0, im = 0.0;
  for (int n0 = 0; n0 < N; n0 += TN) {
    for (int i = threadIdx.x; i < TB * TN; i += 256) {
      const int r = i / TN, cc = i % TN;
      const int kk = blockIdx.y * TB + r;
      a[r][cc] = (kk < K1 && n0 + cc < N) ? E1[static_cast<int64_t>(kk) * N + n0 + cc] : 0.0;
      const int rr = i / TB, c2 = i % TB;
      const int kq = blockIdx.x * TB + c2;
      b[rr][c2] = (kq < K2 && n0 + rr < N) ? E2[static_cast<int64_t>(n0 + rr) * K2 + kq]
                                           : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 8
    for (int t = 0; t < TN; ++t) {
      re = fma(a[ty][t], b[t][tx].x, re);
      im = fma(a[ty][t], b[t][tx].y, im);
    }
    __syncthreads();
  }
  if (k1 < K1 && k2 < K2) {
    const double sc = s1[k1] * s2[k2] * c;
    K[static_cast<int64_t>(k1) * K2 + k2] =
        make_float2(static_cast<float>(re * sc), static_cast<float>(im * sc));
  }
}

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

// ==================================================================== ABI ==

using namespace hrt;

struct hrt_plan_s {
  uint64_t magic;
  int device;
  Geometry g;
  hrt_info info;
  DevGeo dg;
  DirectGeo dd;
  FftDev ft, fr;
  float2* S = nullptr;
  float2* K = nullptr;
  float2* tw_t = nullptr;
  float2* tw_r = nullptr;
  int* jmin = nullptr;
  double* qA = nullptr;
  double* qB = nullptr;
  int* q_i0 = nullptr;
  float4* q_w = nullptr;
  float* q_scale = nullptr;
  float* absmax = nullptr;  // kAbsMaxBlocks partial maxima of the current input
  size_t lds_k1 = 0, lds_k2 = 0, lds_k3 = 0;
  // per-kernel timing (hrt_profile_begin / hrt_profile_end)
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_stage;
  int prof_used = 0;
};

namespace {

thread_local std::string g_last_error;

hrt_status set_err(hrt_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

hrt_status hip_err(hipError_t e, const char* what) {
  return set_err(HRT_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HRT_HIP(call, what)                                        \
  do {                                                             \
    hipError_t e_ = (call);                                        \
    if (e_ != hipSuccess) return hip_err(e_, what);                \
  } while (0)

FftDev to_dev(const FftFactors& f) {
  FftDev d{};
  d.n = f.n;
  d.npass = f.npass;
  d.codes = 0;
  for (int i = 0; i < f.npass; ++i)
    d.codes |= static_cast<unsigned long long>(f.radix[i]) << (4 * i);
  return d;
}

// Two-level twiddle table of length n: exp(-2 pi i 64 a / n) for
// a < ceil(n / 64), then exp(-2 pi i b / n) for b < 64.
std::vector<float2> twiddles(int n) {
  const int nhi = (n + 63) / 64;
  std::vector<float2> t(nhi + 64);
  const double two_pi = 6.283185307179586476925286766559;
  auto put = [&](int i, double j) {
    const double a = -two_pi * j / n;
    t[i] = make_float2(static_cast<float>(std::cos(a)), static_cast<float>(std::sin(a)));
  };
  for (int a = 0; a < nhi; ++a) put(a, 64.0 * a);
  for (int b = 0; b < 64; ++b) put(nhi + b, b);
  return t;
}

template <typename T>
hrt_status dev_alloc(T** p, size_t count, size_t& total) {
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes);
  if (e != hipSuccess) return set_err(HRT_ERR_OOM, "hipMalloc failed");
  total += bytes;
  return HRT_OK;
}

template <typename T>
hrt_status upload(T* dst, const std::vector<T>& src) {
  if (src.empty()) return HRT_OK;
  HRT_HIP(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice),
          "upload");
  return HRT_OK;
}

void free_plan(hrt_plan_s* p) {
  void* ptrs[] = {p->S, p->K, p->tw_t, p->tw_r, p->jmin, p->qA, p->qB,
                  p->q_i0, p->q_w, p->q_scale, p->absmax};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
}

double b_squared(double xi) {  // (sinc^4)^2 of the cubic B-spline
  if (xi == 0.0) return 1.0;
  const double pi = 3.14159265358979323846;
  const double s = std::sin(pi * xi) / (pi * xi);
  const double s2 = s * s, s4 = s2 * s2;
  return s4 * s4;
}

// Kernel spectrum of eq. finiteconv, divided by the B-spline transforms of
// eq. B3tauq, restricted to L (k1 < K1, |k2| < K2), by composite
// Gauss-Legendre quadrature in float64 on the device.
hrt_status build_kernel(hrt_plan_s* p) {
  const Geometry& g = p->g;
  const double Pt = g.Mt * g.dtheta, Pr = g.Mr * g.drho;
  const double rate = (g.Mt / (2.0 * g.sigma)) / Pt +
                      (g.Mr / (2.0 * g.sigma)) * std::tan(g.beta_k) / Pr;
  const int panels = static_cast<int>(std::ceil(g.beta_k * rate)) + 4;
  std::vector<double> nodes, weights;
  gauss_legendre(20, panels, 0.0, g.beta_k, nodes, weights);
  const int N = static_cast<int>(nodes.size());
  std::vector<double> s1(g.K1), s2(g.K2);
  for (int k = 0; k < g.K1; ++k) s1[k] = 1.0 / b_squared(static_cast<double>(k) / g.Mt);
  for (int k = 0; k < g.K2; ++k) s2[k] = 1.0 / b_squared(static_cast<double>(k) / g.Mr);
  double *dn = nullptr, *dw = nullptr, *E1 = nullptr, *ds1 = nullptr, *ds2 = nullptr;
  double2* E2 = nullptr;
  size_t tmp = 0;
  hrt_status st = HRT_OK;
  auto cleanup = [&]() {
    void* ptrs[] = {dn, dw, E1, E2, ds1, ds2};
    for (void* q : ptrs)
      if (q) (void)hipFree(q);
  };
  if ((st = dev_alloc(&dn, N, tmp)) || (st = dev_alloc(&dw, N, tmp)) ||
      (st = dev_alloc(&E1, static_cast<size_t>(g.K1) * N, tmp)) ||
      (st = dev_alloc(&E2, static_cast<size_t>(g.K2) * N, tmp)) ||
      (st = dev_alloc(&ds1, g.K1, tmp)) || (st = dev_alloc(&ds2, g.K2, tmp)) ||
      (st = upload(dn, nodes)) || (st = upload(dw, weights)) ||
      (st = upload(ds1, s1)) || (st = upload(ds2, s2))) {
    cleanup();
    return st;
  }
  const int64_t total = static_cast<int64_t>(g.K1 + g.K2) * N;
  k_zeta_tables<<<static_cast<unsigned>((total + 255) / 256), 256>>>(
      N, g.K1, g.K2, dn, dw, 1.0 / Pt, 1.0 / Pr, E1, E2);
  dim3 grid((g.K2 + 15) / 16, (g.K1 + 15) / 16);
  k_zeta_gemm<<<grid, 256>>>(N, g.K1, g.K2, E1, E2, ds1, ds2,
                             1.0 / (g.dtheta * g.drho), p->K);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  cleanup();
  if (e != hipSuccess) return hip_err(e, "kernel spectrum");
  return HRT_OK;
}

// Live plans: a destroyed or foreign handle is recognised without touching
// the memory it points to.
std::mutex g_plans_mu;
std::set<const hrt_plan_s*> g_plans;

hrt_status check_plan(hrt_plan_t p) {
  if (!p) return set_err(HRT_ERR_INVALID_ARG, "null plan");
  {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    if (!g_plans.count(p)) return set_err(HRT_ERR_BAD_HANDLE, "not a live plan");
  }
  if (p->magic != kMagic) return set_err(HRT_ERR_BAD_HANDLE, "not a live plan");
  return HRT_OK;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

std::mutex g_attr_mu;

}  // namespace

extern "C" {

const char* hrt_status_string(hrt_status s) {
  switch (s) {
    case HRT_OK: return "ok";
    case HRT_ERR_INVALID_ARG: return "invalid argument";
    case HRT_ERR_GEOMETRY: return "geometry not representable";
    case HRT_ERR_OOM: return "out of device memory";
    case HRT_ERR_HIP: return "HIP error";
    case HRT_ERR_BAD_HANDLE: return "bad plan handle";
    case HRT_ERR_UNSUPPORTED: return "unsupported size";
  }
  return "unknown status";
}

const char* hrt_last_error(void) { return g_last_error.c_str(); }

hrt_status hrt_plan_describe(const hrt_desc* desc, hrt_info* out) {
  if (!desc || !out) return set_err(HRT_ERR_INVALID_ARG, "null argument");
  Geometry g;
  std::string err;
  hrt_status s = build_geometry(*desc, 163840 - kWalkLdsBytes, g, err);
  if (s != HRT_OK) return set_err(s, err);
  fill_info(g, out);
  return HRT_OK;
}

hrt_status hrt_plan_create(const hrt_desc* desc, hrt_plan_t* out) {
  if (!desc || !out) return set_err(HRT_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  int dev = 0;
  HRT_HIP(hipGetDevice(&dev), "hipGetDevice");
  hipDeviceProp_t prop;
  HRT_HIP(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
  int lds_max = 0;
  HRT_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
          "hipDeviceGetAttribute");
  // the band kernels also hold the balanced walk's tables in static LDS
  const int64_t lds = std::min<int64_t>(lds_max, 163840) - kWalkLdsBytes;
  (void)hipGetLastError();  // do not report an earlier, unrelated error

  auto* p = new hrt_plan_s();
  p->magic = kMagic;
  p->device = dev;
  std::string err;
  hrt_status s = build_geometry(*desc, lds, p->g, err);
  if (s != HRT_OK) {
    delete p;
    return set_err(s, err);
  }
  const Geometry& g = p->g;
  const int npair_band = g.R / 2;
  const int npair_gather = (g.R + 4) / 2;
  // band rows in 64-bit fixed point; the same bytes then hold the float
  // pairs and the FFT's scratch (grp1 = R/2)
  p->lds_k1 = static_cast<size_t>(g.R) * g.Mt * sizeof(unsigned long long);
  p->lds_k2 = 2 * static_cast<size_t>(g.Mr) * sizeof(float2);
  p->lds_k3 = static_cast<size_t>(npair_gather + g.grp3) * g.Mt * sizeof(float2);
  if (static_cast<int64_t>(p->lds_k2) > std::min<int64_t>(lds_max, 163840)) {
    delete p;
    return set_err(HRT_ERR_UNSUPPORTED, "log-radius axis too long for an LDS column");
  }

  size_t total = 0;
  const std::vector<float2> twt = twiddles(g.Mt), twr = twiddles(g.Mr);
  std::vector<float4> qw(g.d.nq);
  for (int l = 0; l < g.d.nq; ++l)
    qw[l] = make_float4(g.q_w[4 * l], g.q_w[4 * l + 1], g.q_w[4 * l + 2], g.q_w[4 * l + 3]);
  if ((s = dev_alloc(&p->S, static_cast<size_t>(g.K1) * g.Mr, total)) ||
      (s = dev_alloc(&p->K, static_cast<size_t>(g.K1) * g.K2, total)) ||
      (s = dev_alloc(&p->tw_t, twt.size(), total)) ||
      (s = dev_alloc(&p->tw_r, twr.size(), total)) ||
      (s = dev_alloc(&p->jmin, g.d.nx, total)) || (s = dev_alloc(&p->qA, g.d.nq, total)) ||
      (s = dev_alloc(&p->qB, g.d.nq, total)) || (s = dev_alloc(&p->q_i0, g.d.nq, total)) ||
      (s = dev_alloc(&p->q_w, g.d.nq, total)) || (s = dev_alloc(&p->q_scale, g.d.nq, total)) ||
      (s = dev_alloc(&p->absmax, kAbsMaxBlocks, total)) ||
      (s = upload(p->tw_t, twt)) || (s = upload(p->tw_r, twr)) ||
      (s = upload(p->jmin, g.jmin)) || (s = upload(p->qA, g.qA)) ||
      (s = upload(p->qB, g.qB)) || (s = upload(p->q_i0, g.q_i0)) ||
      (s = upload(p->q_w, qw)) || (s = upload(p->q_scale, g.q_scale))) {
    free_plan(p);
    delete p;
    return s;
  }
  hipError_t e = hipMemset(p->S, 0, static_cast<size_t>(g.K1) * g.Mr * sizeof(float2));
  if (e != hipSuccess) {
    free_plan(p);
    delete p;
    return hip_err(e, "hipMemset");
  }
  if ((s = build_kernel(p)) != HRT_OK) {
    free_plan(p);
    delete p;
    return s;
  }
  {
    // dynamic LDS above the default limit must be granted per kernel; the
    // grant is process-wide, so always the largest the kernel can take
    // (the device limit less its static LDS), whatever this plan needs
    std::lock_guard<std::mutex> lk(g_attr_mu);
    const int64_t cap = std::min<int64_t>(lds_max, 163840);
    const void* fns[] = {reinterpret_cast<const void*>(&k_spread_rowfft<0>),
                         reinterpret_cast<const void*>(&k_spread_rowfft<1>),
                         reinterpret_cast<const void*>(&k_colfft<false>),
                         reinterpret_cast<const void*>(&k_colfft<true>),
                         reinterpret_cast<const void*>(&k_rowifft_gather<0>),
                         reinterpret_cast<const void*>(&k_rowifft_gather<1>)};
    const size_t need[] = {p->lds_k1, p->lds_k1, p->lds_k2, p->lds_k2, p->lds_k3, p->lds_k3};
    struct {
      const void* fn;
      size_t bytes;
    } attrs[6];
    for (int i = 0; i < 6; ++i) {
      hipFuncAttributes fa;
      hipError_t r = hipFuncGetAttributes(&fa, fns[i]);
      if (r != hipSuccess) {
        (void)hipGetLastError();
        free_plan(p);
        delete p;
        return hip_err(r, "hipFuncGetAttributes");
      }
      const int64_t room = cap - static_cast<int64_t>(fa.sharedSizeBytes);
      if (static_cast<int64_t>(need[i]) > room) {
        free_plan(p);
        delete p;
        return set_err(HRT_ERR_UNSUPPORTED, "lattice rows exceed the LDS of a workgroup");
      }
      attrs[i] = {fns[i], static_cast<size_t>(room)};
    }
    for (const auto& a : attrs) {
      hipError_t r = hipFuncSetAttribute(a.fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         static_cast<int>(a.bytes));
      if (r != hipSuccess) {
        (void)hipGetLastError();
        free_plan(p);
        delete p;
        return hip_err(r, "hipFuncSetAttribute");
      }
    }
  }
  DevGeo& G = p->dg;
  G.nt = g.d.nt; G.nx = g.d.nx; G.ntau = g.d.ntau; G.nq = g.d.nq;
  G.dt = g.d.dt; G.x0 = g.d.x0; G.dx = g.d.dx; G.tau0 = g.d.tau0; G.dtau = g.d.dtau;
  G.T = g.T; G.X = g.X;
  G.a = g.a; G.O1 = g.O1; G.O2 = g.O2; G.ca = g.ca; G.sa = g.sa; G.AeA = g.AeA;
  G.inv_dtheta = 1.0 / g.dtheta; G.inv_drho = 1.0 / g.drho; G.drho = g.drho;
  G.ctheta = g.ctheta; G.crho = g.crho;
  G.wconst = 2.0 * g.a * g.a * (g.d.dt / g.T) * (g.d.dx / g.X);
  G.Mt = g.Mt; G.Mr = g.Mr; G.K1 = g.K1; G.K2 = g.K2; G.u0 = g.u0; G.u1 = g.u1;
  G.R = g.R; G.nbands = g.nbands; G.grp1 = g.grp1; G.grp3 = g.grp3;
  G.knorm = static_cast<float>(1.0 / (static_cast<double>(g.Mt) * g.Mr));
  // |W| <= 2 a^2 dt^ dx^ / a_r (t^ <= 1, |p| >= a_r inside the trapezoid);
  // the Radon weights are X cos(psi_l)/a; both padded by 1e-6 for rounding
  G.wmax_data = static_cast<float>(G.wconst / g.a_r * (1.0 + 1e-6));
  {
    double m = 0.0;
    for (float v : g.q_scale) m = std::max(m, static_cast<double>(v));
    G.wmax_radon = static_cast<float>(m * (1.0 + 1e-6));
  }
  G.jmin = p->jmin; G.qA = p->qA; G.qB = p->qB; G.q_i0 = p->q_i0;
  G.q_w = p->q_w; G.q_scale = p->q_scale;
  p->ft = to_dev(g.fft_t);
  p->fr = to_dev(g.fft_r);

  DirectGeo& D = p->dd;
  D.nt = g.d.nt; D.nx = g.d.nx; D.ntau = g.d.ntau; D.nq = g.d.nq;
  D.dt = static_cast<float>(g.d.dt); D.inv_dt = static_cast<float>(1.0 / g.d.dt);
  D.x0 = static_cast<float>(g.d.x0); D.dx = static_cast<float>(g.d.dx);
  D.tau0 = static_cast<float>(g.d.tau0); D.dtau = static_cast<float>(g.d.dtau);
  D.q0 = static_cast<float>(g.d.q0); D.dq = static_cast<float>(g.d.dq);

  fill_info(g, &p->info);
  p->info.workspace_bytes = static_cast<int64_t>(total);
  {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    g_plans.insert(p);
  }
  *out = p;
  return HRT_OK;
}

namespace {
// Records the profiling events around one kernel launch (no-op unless a
// profile is active and has room).
struct StageTimer {
  hrt_plan_s* p;
  hipStream_t st;
  int slot = -1;
  StageTimer(hrt_plan_s* plan, hipStream_t s, int stage) : p(plan), st(s) {
    if (p->prof_used < static_cast<int>(p->prof_stage.size())) {
      slot = p->prof_used++;
      p->prof_stage[slot] = stage;
      (void)hipEventRecord(p->prof_ev[2 * slot], st);
    }
  }
  ~StageTimer() {
    if (slot >= 0) (void)hipEventRecord(p->prof_ev[2 * slot + 1], st);
  }
};
}  // namespace

static hrt_status launch_chain(hrt_plan_t p, const float* in, float* out, void* stream,
                               bool adjoint) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  if (!in || !out) return set_err(HRT_ERR_INVALID_ARG, "null array");
  const size_t n_data = static_cast<size_t>(p->g.d.nx) * p->g.d.nt;
  const size_t n_radon = static_cast<size_t>(p->g.d.nq) * p->g.d.ntau;
  const size_t n_in = adjoint ? n_radon : n_data;
  const size_t n_out = adjoint ? n_data : n_radon;
  const char* ib = reinterpret_cast<const char*>(in);
  const char* ob = reinterpret_cast<const char*>(out);
  if (ib < ob + n_out * sizeof(float) && ob < ib + n_in * sizeof(float))
    return set_err(HRT_ERR_INVALID_ARG, "input and output overlap");
  DeviceGuard guard(p->device);
  (void)hipGetLastError();  // do not report an earlier, unrelated error
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const Geometry& g = p->g;
  const dim3 bands(g.nbands);
  if (!adjoint) {
    {
      StageTimer t(p, st, 0);
      k_absmax<<<kAbsMaxBlocks, 256, 0, st>>>(in, static_cast<int64_t>(n_in), p->absmax);
      k_spread_rowfft<0><<<bands, kNtBand, p->lds_k1, st>>>(p->dg, p->ft, p->tw_t, in,
                                                            p->absmax, p->S);
    }
    {
      StageTimer t(p, st, 1);
      k_colfft<false><<<g.K1, kNtCol, p->lds_k2, st>>>(p->dg, p->fr, p->tw_r, p->S, p->K);
    }
    {
      StageTimer t(p, st, 2);
      k_rowifft_gather<0><<<bands, kNtBand, p->lds_k3, st>>>(p->dg, p->ft, p->tw_t, p->S, out);
    }
  } else {
    {
      StageTimer t(p, st, 3);
      k_absmax<<<kAbsMaxBlocks, 256, 0, st>>>(in, static_cast<int64_t>(n_in), p->absmax);
      k_spread_rowfft<1><<<bands, kNtBand, p->lds_k1, st>>>(p->dg, p->ft, p->tw_t, in,
                                                            p->absmax, p->S);
    }
    {
      StageTimer t(p, st, 4);
      k_colfft<true><<<g.K1, kNtCol, p->lds_k2, st>>>(p->dg, p->fr, p->tw_r, p->S, p->K);
    }
    {
      StageTimer t(p, st, 5);
      k_rowifft_gather<1><<<bands, kNtBand, p->lds_k3, st>>>(p->dg, p->ft, p->tw_t, p->S, out);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, adjoint ? "adjoint launch" : "forward launch");
  return HRT_OK;
}

hrt_status hrt_forward(hrt_plan_t p, const float* f, float* g, void* stream) {
  return launch_chain(p, f, g, stream, false);
}

hrt_status hrt_adjoint(hrt_plan_t p, const float* g, float* f, void* stream) {
  return launch_chain(p, g, f, stream, true);
}

hrt_status hrt_direct_forward(hrt_plan_t p, const float* f, float* g, void* stream) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  if (!f || !g) return set_err(HRT_ERR_INVALID_ARG, "null array");
  DeviceGuard guard(p->device);
  const DirectGeo& D = p->dd;
  dim3 grid((D.ntau + 255) / 256, D.nq);
  k_direct_fwd<<<grid, 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(D, f, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, "direct forward launch");
  return HRT_OK;
}

hrt_status hrt_direct_adjoint(hrt_plan_t p, const float* g, float* f, void* stream) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  if (!f || !g) return set_err(HRT_ERR_INVALID_ARG, "null array");
  DeviceGuard guard(p->device);
  const DirectGeo& D = p->dd;
  dim3 grid((D.nt + 255) / 256, D.nx);
  k_direct_adj<<<grid, 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(D, g, f);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(e, "direct adjoint launch");
  return HRT_OK;
}

hrt_status hrt_query(hrt_plan_t p, hrt_info* out) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  if (!out) return set_err(HRT_ERR_INVALID_ARG, "null argument");
  *out = p->info;
  return HRT_OK;
}

hrt_status hrt_plan_kernel(hrt_plan_t p, float* host_out) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  if (!host_out) return set_err(HRT_ERR_INVALID_ARG, "null argument");
  DeviceGuard guard(p->device);
  HRT_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
  HRT_HIP(hipMemcpy(host_out, p->K,
                    static_cast<size_t>(p->g.K1) * p->g.K2 * sizeof(float2),
                    hipMemcpyDeviceToHost),
          "copy kernel");
  return HRT_OK;
}

static void release_profile(hrt_plan_t p) {
  for (hipEvent_t e : p->prof_ev) (void)hipEventDestroy(e);
  p->prof_ev.clear();
  p->prof_stage.clear();
  p->prof_used = 0;
}

hrt_status hrt_profile_begin(hrt_plan_t p, int32_t max_records) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  if (max_records < 1 || max_records > (1 << 20))
    return set_err(HRT_ERR_INVALID_ARG, "max_records out of range");
  DeviceGuard guard(p->device);
  release_profile(p);
  p->prof_ev.resize(2 * static_cast<size_t>(max_records));
  for (auto& e : p->prof_ev) {
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) {
      e = nullptr;
      p->prof_ev.clear();
      return hip_err(r, "hipEventCreate");
    }
  }
  p->prof_stage.assign(max_records, -1);
  p->prof_used = 0;
  return HRT_OK;
}

hrt_status hrt_profile_end(hrt_plan_t p, double* ms_sum, int64_t* count) {
  hrt_status s = check_plan(p);
  if (s != HRT_OK) return s;
  DeviceGuard guard(p->device);
  double ms[6] = {0, 0, 0, 0, 0, 0};
  int64_t cnt[6] = {0, 0, 0, 0, 0, 0};
  hrt_status out = HRT_OK;
  for (int i = 0; i < p->prof_used; ++i) {
    float t = 0.f;
    hipError_t r = hipEventSynchronize(p->prof_ev[2 * i + 1]);
    if (r == hipSuccess) r = hipEventElapsedTime(&t, p->prof_ev[2 * i], p->prof_ev[2 * i + 1]);
    if (r != hipSuccess) {
      out = hip_err(r, "hipEventElapsedTime");
      break;
    }
    ms[p->prof_stage[i]] += t;
    cnt[p->prof_stage[i]] += 1;
  }
  release_profile(p);
  for (int i = 0; i < 6; ++i) {
    if (ms_sum) ms_sum[i] = ms[i];
    if (count) count[i] = cnt[i];
  }
  return out;
}

void hrt_plan_destroy(hrt_plan_t p) {
  {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    if (!p || !g_plans.erase(p)) return;
  }
  DeviceGuard guard(p->device);
  (void)hipDeviceSynchronize();
  release_profile(p);
  free_plan(p);
  p->magic = 0;
  delete p;
}

}  // extern "C"
