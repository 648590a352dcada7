// Points on the log-polar lattice: the ranges of samples that reach a row
// band, the float64 anchors from which a band's samples are placed, the
// fixed-point tap accumulator of the spread, the 4x4 interpolation of the
// gather, and the balanced walk that deals a band's samples to threads.
#pragma once

#include "device_common.hpp"

namespace hrt {

// ------------------------------------------------------------ ranges --

// Time index j (fractional) where trace k reaches log radius Y (lattice
// units), from |p(s)|^2 = c0 + c1 s + c2 s^2 along the trace, s = t^2.
__device__ __forceinline__ double trace_j_at(const DevGeo& G, double c0, double c1,
                                             double c2, double Y) {
  const double r2 = exp(2.0 * (Y - G.crho) * G.drho);
  const double disc = c1 * c1 + 4.0 * c2 * (r2 - c0);
  if (disc <= 0.0) return 0.0;
  const double s = 2.0 * (r2 - c0) / (c1 + sqrt(disc));
  if (s <= 0.0) return 0.0;
  return fmin(sqrt(s) * (G.nt - 1), 1e9);
}

// Kept samples j of trace k whose log radius may lie in [Ylo, Yhi): a
// superset with a one-sample margin (every point is re-checked).
__device__ __forceinline__ void data_range(const DevGeo& G, int k, double Ylo, double Yhi,
                                           int& jlo, int& jhi) {
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

// Samples i of slowness column l whose log radius may lie in [Ylo, Yhi),
// from e^rho = A + B tau^2 (superset, one-sample margin).
__device__ __forceinline__ void radon_range(const DevGeo& G, double A, double B, double Ylo,
                                            double Yhi, int& ilo, int& ihi) {
  auto i_at = [&](double Y) {
    const double e = exp((Y - G.crho) * G.drho);
    const double t2 = (e - A) / B;
    if (t2 <= 0.0) return -1e9;
    return fmin((sqrt(t2) * G.T - G.tau0) / G.dtau, 1e9);
  };
  ilo = max(0, static_cast<int>(ceil(i_at(Ylo))) - 1);
  ihi = min(G.ntau, static_cast<int>(ceil(i_at(Yhi))) + 1);
}

// ----------------------------------------------------------- anchors --

// Data samples.  Along trace k the mapped point p = T(t^2, x^2) moves on a
// straight line, p_j = p_a + delta e_alpha with delta = a (s_j - s_a), so
// from an anchor sample a placed in full (atan2, log) every sample of the
// trace within the band follows from
//   tan(phi_j - phi_a) = delta q1 / (1 + delta q2),
//   |p_j|^2 / |p_a|^2 = 1 + x,   x = delta (2 q2 + delta / |p_a|^2),
// with q1 = (p_a x e_alpha) / |p_a|^2 and q2 = (p_a . e_alpha) / |p_a|^2,
// and float64 series for atan and log1p (exact to rounding; larger
// increments are first halved).  The smear
// weight 2 a^2 t^ e^-eta w_t w_x dt^ dx^ (the 1/(2 sqrt y) of eq. f times
// the Jacobian, trapezoid rule) is w_a t^ w_t (1 + x)^-1/2.
// One anchor per unit slot of the walk's current chunk, in LDS.
struct DataAnchors {
  double xg[kNtBand], yg[kNtBand], q1[kNtBand], q2[kNtBand], th[kNtBand];
  float inv_r2[kNtBand], wa[kNtBand];

  __device__ __forceinline__ static void place(const DevGeo& G, int j, int k, double& th,
                                               double& xg, double& yg, double& q1,
                                               double& q2, float& inv_r2, float& wa) {
    th = (static_cast<double>(j) * G.dt) / G.T;
    const double xh = (G.x0 + static_cast<double>(k) * G.dx) / G.X;
    const double ds = th * th - 0.5, dy = xh * xh - 0.5;
    const double u = G.a * (G.ca * ds - G.sa * dy) + G.O1;
    const double v = G.a * (G.sa * ds + G.ca * dy) + G.O2;
    const double r2 = u * u + v * v;
    xg = atan2(v, u) * G.inv_dtheta + G.ctheta;
    yg = 0.5 * log(r2) * G.inv_drho + G.crho;
    const double ir2 = 1.0 / r2;
    inv_r2 = static_cast<float>(ir2);
    q1 = (u * G.sa - v * G.ca) * ir2;
    q2 = (u * G.ca + v * G.sa) * ir2;
    wa = static_cast<float>(G.wconst * ((k == 0 || k == G.nx - 1) ? 0.5 : 1.0) * sqrt(ir2));
  }

  __device__ __forceinline__ void set(int slot, const DevGeo& G, int j, int k) {
    double t, x, y, a1, a2;
    float ir, w;
    place(G, j, k, t, x, y, a1, a2, ir, w);
    th[slot] = t;
    xg[slot] = x;
    yg[slot] = y;
    q1[slot] = a1;
    q2[slot] = a2;
    inv_r2[slot] = ir;
    wa[slot] = w;
  }

  // lattice coordinates and smear weight of sample j of slot's trace
  __device__ __forceinline__ void eval(int slot, const DevGeo& G, int j, double& x, double& y,
                                       float& w) const {
    const double t = (static_cast<double>(j) * G.dt) / G.T;
    const float wt = (j == G.nt - 1) ? 0.5f : 1.0f;
    const double ta = th[slot];
    const double delta = G.a * ((t - ta) * (t + ta));
    const double dq = delta * q2[slot];
    // p_a . p_j > 0 inside the sector; 1 / (1 + dq) by Newton when dq is
    // small, as it is for a band's samples
    const double r = fabs(dq) <= 0.15 ? rcp_near1(1.0 + dq) : 1.0 / (1.0 + dq);
    const double z = delta * q1[slot] * r;
    const double e = delta * fma(delta, static_cast<double>(inv_r2[slot]), 2.0 * q2[slot]);
    x = xg[slot] + atan_any(z) * G.inv_dtheta;
    y = yg[slot] + 0.5 * log1p_any(e) * G.inv_drho;
    w = wa[slot] * static_cast<float>(t) * wt * rsqrtf(1.0f + static_cast<float>(e));
  }

  // The same quantities placed in full, without an anchor.  A point whose
  // log-radius coordinate lies within rounding of a row boundary is placed
  // this way by every band that meets it, so that all of them agree on the
  // band that owns it (anchored values differ in the last bits from band to
  // band).
  __device__ static void exact(const DevGeo& G, int j, int k, double& x, double& y, float& w) {
    double th, q1, q2;
    float ir, wa;
    place(G, j, k, th, x, y, q1, q2, ir, wa);
    w = wa * static_cast<float>(th) * ((j == G.nt - 1) ? 0.5f : 1.0f);
  }
};

// Radon samples of slowness column l: angle from the per-column table,
// e^rho = A + B tau^2, from an anchor sample a by
// rho_i = rho_a + log1p(B (tau_i^2 - tau_a^2) / e^rho_a).
struct RadonAnchors {
  double yg[kNtBand], bi[kNtBand], th[kNtBand];  // bi = B / e^rho_a
  float4 qw[kNtBand];                            // angle tap weights
  int i0[kNtBand];                               // first angle tap
  float sc[kNtBand];                             // X cos(psi) / a

  __device__ __forceinline__ void set(int slot, const DevGeo& G, int i, int l) {
    const double A = G.qA[l], B = G.qB[l];
    const double t = (G.tau0 + static_cast<double>(i) * G.dtau) / G.T;
    const double ea = A + B * (t * t);
    yg[slot] = log(ea) * G.inv_drho + G.crho;
    bi[slot] = B / ea;
    th[slot] = t;
    qw[slot] = G.q_w[l];
    i0[slot] = G.q_i0[l];
    sc[slot] = G.q_scale[l];
  }

  // log-radius lattice coordinate of sample i of slot's column
  __device__ __forceinline__ double eval_y(int slot, const DevGeo& G, int i) const {
    const double t = (G.tau0 + static_cast<double>(i) * G.dtau) / G.T;
    const double ta = th[slot];
    return yg[slot] + log1p_any(bi[slot] * ((t - ta) * (t + ta))) * G.inv_drho;
  }

  // The same coordinate without an anchor (see DataAnchors::exact).
  __device__ static double exact_y(const DevGeo& G, int i, int l) {
    const double t = (G.tau0 + static_cast<double>(i) * G.dtau) / G.T;
    return log(G.qA[l] + G.qB[l] * (t * t)) * G.inv_drho + G.crho;
  }
};

// True when a log-radius coordinate is within rounding of a lattice row, where
// the band that owns the point must be decided from the exact placement.
__device__ __forceinline__ bool near_row(double yg) { return fabs(yg - rint(yg)) < 1e-8; }

// Bytes of LDS the anchors of one chunk take (the larger of the two kinds).
constexpr int kAnchorLdsBytes =
    sizeof(DataAnchors) > sizeof(RadonAnchors) ? sizeof(DataAnchors) : sizeof(RadonAnchors);

// -------------------------------------------------------------- taps --

// Per-thread accumulator of the 4x4 B-spline taps of consecutive points that
// fall on the same lattice cell (a thread walks consecutive samples of one
// trace or slowness column, and where the lattice is coarse many of them
// share a cell): their taps are summed in registers and reach LDS as one set
// of 16 atomic adds.
//
// The band accumulates in 64-bit fixed point: a tap value v enters as
// round(v * scale), scale = 2^40 / (bound on |v|), added with the integer
// LDS atomic (float LDS atomics are some 25x slower on gfx950).  Integer
// sums are exact and order-independent, so the band is deterministic; the
// quantum is 2^-40 of the largest possible tap.  Row r of the band, angle
// column c, is acc64[r * W + c - xw0]; rows outside [n0, n0+nr) are dropped.
struct TapAcc {
  int ix = INT_MIN, iy = 0;
  float a[4][4];

  __device__ __forceinline__ void flush(unsigned long long* acc64, const DevGeo& G, int n0,
                                        int nr, double scale) {
    if (ix == INT_MIN) return;
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      const int rl = iy - 1 + bb - n0;
      if (rl < 0 || rl >= nr) continue;
      unsigned long long* base = acc64 + rl * G.W + (ix - G.xw0);
#pragma unroll
      for (int aa = 0; aa < 4; ++aa) atomicAdd(base + aa, to_fixed(a[bb][aa], scale));
    }
    ix = INT_MIN;  // nothing pending
  }

  // add w * B3(x - xg) B3(y - yg) for the point at lattice (xg, yg); nix is
  // the first angle tap
  __device__ __forceinline__ void add(unsigned long long* acc64, const DevGeo& G, int n0,
                                      int nr, double scale, int nix, const float wx[4],
                                      double yg, float w) {
    const double fy0 = floor(yg);
    const int niy = static_cast<int>(fy0);
    if (niy + 2 < n0 || niy - 1 >= n0 + nr || nix < G.xw0 || nix + 4 > G.xw0 + G.W) return;
    float wy[4];
    bspline4(static_cast<float>(yg - fy0), wy);
    if (nix != ix || niy != iy) {
      flush(acc64, G, n0, nr, scale);
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

// Sum of C[m, n] B3(x - m) B3(y - n) over the 4x4 taps of a point, C being
// the band's lattice rows [L0, L1) held in LDS as complex pairs (row r at
// component r & 1 of pair r >> 1).  Taps outside the held rows or the angle
// axis are skipped (no point a band owns reaches them).
__device__ __forceinline__ float gather_taps(const float* ldsf, int Mt, int L0, int L1,
                                             int ix, const float wx[4], int iy,
                                             const float wy[4]) {
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

// -------------------------------------------------------------- walk --

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

// Visits every point of every unit (a trace or a slowness column) that may
// reach the band.  Units are taken kNtBand at a time; in each chunk thread
// `slot` handles unit c0 + slot in range(slot, u, lo, hi), which returns the
// unit's superset range and may leave per-unit data (the anchors) in LDS.
// The chunk's points are then cut into equal contiguous segments, one per
// thread, so every thread does the same amount of work whatever the spread
// of range lengths; a segment arrives as runs of consecutive points of one
// unit, run(acc, slot, u, idx0, len), with a fresh per-thread accumulator
// `acc` of type Acc that finish(acc) closes after the thread's last run (so
// the accumulator is not live while the next chunk's ranges are computed).
// Segments are dealt to lanes 16 apart (lane-major), so the lanes of one
// wave work on points far from each other on the lattice.
struct NoAcc {};

template <class Acc, class RangeF, class RunF, class FinishF>
__device__ __forceinline__ void balanced_walk(int nunits, WalkLds& w, RangeF range, RunF run,
                                              FinishF finish) {
  for (int c0 = 0; c0 < nunits; c0 += kNtBand) {
    const int slot = static_cast<int>(threadIdx.x);
    const int u = c0 + slot;
    int lo = 0, cnt = 0;
    if (u < nunits) {
      int hi;
      range(slot, u, lo, hi);
      cnt = max(0, hi - lo);
    }
    int total;
    const int excl = block_exclusive_scan(cnt, w.wave, total);
    w.lo[slot] = lo;
    w.pre[slot] = excl;
    if (slot == 0) w.pre[kNtBand] = total;
    __syncthreads();
    const int per = (total + kNtBand - 1) / kNtBand;
    const int seg = (slot & 63) * (kNtBand / 64) + (slot >> 6);
    int p = seg * per;
    const int pend = min(p + per, total);
    Acc acc;
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
        run(acc, unit, c0 + unit, w.lo[unit] + (p - w.pre[unit]), len);
        p += len;
      }
    }
    finish(acc);
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

}  // namespace hrt
