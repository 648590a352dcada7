// Workgroup-wide mixed-radix Stockham FFTs on sequences held in LDS.
//
// A batch of B complex sequences of length n (n = product of the radices in
// an FftDev) sits in LDS at data + b*stride.  Element e of a sequence is
// stored at lpad(e) = e + e/16: one unused slot after every 16 elements
// spreads the strided stores of the early passes (stride R*Ns complex
// values) over all LDS banks.  Each pass reads one LDS buffer
// and writes the other (Stockham autosort order), so a thread only holds the
// R values of the butterfly it is working on.  Twiddles exp(-2 pi i m / n)
// come from a two-level table in LDS, tw[m >> 6] * tw[nhi + (m & 63)] with
// nhi = ceil(n / 64), each level computed in float64 on the host and rounded
// once (about 1.5 ulp for the product).  Forward transforms use
// exp(-2 pi i ...); INV selects exp(+2 pi i ...), unnormalised.
#pragma once

#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace hrt {


constexpr int kTwLds = 256;  // two-level twiddle entries: n <= 64 * (256 - 64)

// Length and radix sequence of one transform; the radix of pass p sits in
// bits [8p, 8p+8) of `codes` (small enough to travel in registers).
struct FftDev {
  int n;
  int npass;
  unsigned long long codes;
};

__host__ __device__ inline int fft_radix(const FftDev& f, int p) {
  return static_cast<int>((f.codes >> (8 * p)) & 0xFF);
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) {
  return make_float2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ float2 csub(float2 a, float2 b) {
  return make_float2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) {
  return make_float2(a.x * s, a.y * s);
}
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 rot(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV>
struct Dft<3, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    const float s = 0.86602540378443864676f;  // sin(2 pi/3)
    float2 t1 = cadd(v[1], v[2]);
    float2 t2 = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
    float2 t3 = cscale(csub(v[1], v[2]), s);
    v[0] = cadd(v[0], t1);
    float2 r = rot<INV>(t3);
    v[1] = cadd(t2, r);
    v[2] = csub(t2, r);
  }
};

template <bool INV>
struct Dft<4, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    float2 b0 = cadd(v[1], v[3]), b1 = rot<INV>(csub(v[1], v[3]));
    v[0] = cadd(a0, b0);
    v[2] = csub(a0, b0);
    v[1] = cadd(a1, b1);
    v[3] = csub(a1, b1);
  }
};

template <bool INV>
struct Dft<5, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    const float c1 = 0.30901699437494742410f;   // cos(2 pi/5)
    const float c2 = -0.80901699437494742410f;  // cos(4 pi/5)
    const float s1 = 0.95105651629515357212f;   // sin(2 pi/5)
    const float s2 = 0.58778525229247312917f;   // sin(4 pi/5)
    float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    float2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    float2 x0 = v[0];
    v[0] = cadd(x0, cadd(t1, t2));
    float2 a1 = make_float2(x0.x + c1 * t1.x + c2 * t2.x, x0.y + c1 * t1.y + c2 * t2.y);
    float2 a2 = make_float2(x0.x + c2 * t1.x + c1 * t2.x, x0.y + c2 * t1.y + c1 * t2.y);
    float2 b1 = make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y);
    float2 b2 = make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y);
    float2 r1 = rot<INV>(b1), r2 = rot<INV>(b2);
    v[1] = cadd(a1, r1);
    v[4] = csub(a1, r1);
    v[2] = cadd(a2, r2);
    v[3] = csub(a2, r2);
  }
};

template <bool INV>
struct Dft<8, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    const float h = 0.70710678118654752440f;
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, INV>::run(e);
    Dft<4, INV>::run(o);
    // o[k] *= w8^k, w8 = exp(-+ 2 pi i / 8)
    float2 w1 = INV ? make_float2(h, h) : make_float2(h, -h);
    float2 w3 = INV ? make_float2(-h, h) : make_float2(-h, -h);
    o[1] = cmul(o[1], w1);
    o[2] = rot<INV>(o[2]);
    o[3] = cmul(o[3], w3);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = cadd(e[k], o[k]);
      v[k + 4] = csub(e[k], o[k]);
    }
  }
};

// cos and sin of 2 pi num / den in float64 by their Taylor series after
// reduction to [-pi, pi] (30 terms: truncation below 1e-17), for tables built
// at compile time.
constexpr double cx_trig2pi(int num, int den, bool sine) {
  const double pi = 3.14159265358979323846;
  double x = 2.0 * pi * static_cast<double>(num % den) / den;
  if (x > pi) x -= 2.0 * pi;
  double term = sine ? x : 1.0, sum = term;
  for (int i = 1; i < 30; ++i) {
    const double a = sine ? 2.0 * i : 2.0 * i - 1.0;
    term *= -x * x / (a * (a + 1.0));
    sum += term;
  }
  return sum;
}

// exp(-2 pi i m / R) for m < R, as float.
template <int R>
struct RootTable {
  float c[R], s[R];
  constexpr RootTable() : c(), s() {
    for (int m = 0; m < R; ++m) {
      c[m] = static_cast<float>(cx_trig2pi(m, R, false));
      s[m] = static_cast<float>(-cx_trig2pi(m, R, true));
    }
  }
};

// Composite radix R = A*B in registers (Cooley-Tukey): with n = a + A b and
// k = B k1 + k2, X[k] = sum_a W_A^(a k1) W_R^(a k2) sum_b x[a + A b] W_B^(b k2).
// The inner twiddles W_R^(a k2) are compile-time constants.
template <int A, int B, bool INV>
struct DftAB {
  __device__ __forceinline__ static void run(float2* v) {
    constexpr int R = A * B;
    constexpr RootTable<R> W{};
    float2 y[A][B];
#pragma unroll
    for (int a = 0; a < A; ++a) {
#pragma unroll
      for (int b = 0; b < B; ++b) y[a][b] = v[a + A * b];
      Dft<B, INV>::run(y[a]);
#pragma unroll
      for (int k2 = 1; k2 < B; ++k2) {
        if (a == 0) continue;
        const int m = (a * k2) % R;
        y[a][k2] = cmul(y[a][k2], make_float2(W.c[m], INV ? -W.s[m] : W.s[m]));
      }
    }
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) {
      float2 z[A];
#pragma unroll
      for (int a = 0; a < A; ++a) z[a] = y[a][k2];
      Dft<A, INV>::run(z);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) v[B * k1 + k2] = z[k1];
    }
  }
};

template <bool INV> struct Dft<6, INV> : DftAB<2, 3, INV> {};
template <bool INV> struct Dft<9, INV> : DftAB<3, 3, INV> {};
template <bool INV> struct Dft<10, INV> : DftAB<2, 5, INV> {};
template <bool INV> struct Dft<12, INV> : DftAB<4, 3, INV> {};
template <bool INV> struct Dft<15, INV> : DftAB<3, 5, INV> {};
template <bool INV> struct Dft<16, INV> : DftAB<4, 4, INV> {};

// floor(x / d) for 0 <= x < 2^16, 1 <= d < 2^16 by a multiply-high with
// m = ceil(2^32 / d); m = 0 stands for d = 1 (2^32 does not fit).
__device__ __forceinline__ int div_small(int x, unsigned m) {
  return m ? static_cast<int>(__umulhi(static_cast<unsigned>(x), m)) : x;
}
__device__ __forceinline__ unsigned div_magic(int d) {
  return d == 1 ? 0u : 0xFFFFFFFFu / static_cast<unsigned>(d) + 1u;
}

// One out-of-place radix-R Stockham pass over B sequences of length n:
// src sequences at src + b*ss, results to dst + b*sd.  Ns is the length of
// the sub-transforms already combined.  A thread takes U butterflies at a
// time (as many as the in-place form holds) and issues all their loads before
// any arithmetic, so that the LDS latencies overlap.  The twiddles w^r of a
// butterfly are products of the table values w^(2^i), at most four factors.
template <int R, int NT, bool INV>
__device__ __forceinline__ void stockham_pass(const float2* __restrict__ src, int ss,
                                              float2* __restrict__ dst, int sd, int n,
                                              int B, int Ns,
                                              const float2* __restrict__ tw) {
  constexpr int U = inplace_units(R, kInplaceValues) > 0 ? inplace_units(R, kInplaceValues) : 1;
  constexpr int NB2 = R > 8 ? 4 : (R > 4 ? 3 : (R > 2 ? 2 : 1));  // powers w^(2^i) needed
  const int nb = n / R;
  const int total = B * nb;
  const int twstep = n / (Ns * R);
  const int nhi = (n + 63) >> 6;
  const unsigned m_nb = div_magic(nb), m_ns = div_magic(Ns);
  for (int i0 = threadIdx.x; i0 < total; i0 += NT * U) {
    float2 v[U][R];
    int ob[U], oo[U], kk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = i0 + u * NT;
      const int b = div_small(idx, m_nb);
      const int j = idx - b * nb;
      const int k = j - div_small(j, m_ns) * Ns;
      kk[u] = k;
      ob[u] = b * sd;
      oo[u] = (j - k) * R + k;
      if (idx < total) {
        const float2* in = src + b * ss;
#pragma unroll
        for (int r = 0; r < R; ++r) v[u][r] = in[lpad(j + r * nb)];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i0 + u * NT < total) {
        if (kk[u] != 0) {
          float2 p2[NB2];
#pragma unroll
          for (int i = 0; i < NB2; ++i) {
            const int m = (kk[u] * twstep) << i;
            p2[i] = cmul(tw[m >> 6], tw[nhi + (m & 63)]);
            if (INV) p2[i].y = -p2[i].y;
          }
#pragma unroll
          for (int r = 1; r < R; ++r) {
            float2 w = make_float2(1.0f, 0.0f);
            bool first = true;
#pragma unroll
            for (int i = 0; i < NB2; ++i) {
              if (r & (1 << i)) {
                w = first ? p2[i] : cmul(w, p2[i]);
                first = false;
              }
            }
            v[u][r] = cmul(v[u][r], w);
          }
        }
        Dft<R, INV>::run(v[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i0 + u * NT < total) {
        float2* out = dst + ob[u];
#pragma unroll
        for (int r = 0; r < R; ++r) out[lpad(oo[u] + r * Ns)] = v[u][r];
      }
    }
  }
}

// A pass's outputs as they are: the default of the passes' `post` hook.
// A hook sees (sequence b, output index, unrolled output r of the thread's
// butterfly, value) before the value is stored; with kStores the hook
// stores the value itself and the pass leaves LDS as it was.
struct NoPost {
  static constexpr bool kStores = false;
  __device__ __forceinline__ void operator()(int, int, int, float2&) const {}
};

// The first pass's inputs as they are in LDS: the default of the passes'
// `pre` hook.  A hook with kLoads gives input `index` of sequence b itself
// (from global memory, say), and the pass reads no LDS.
struct NoPre {
  static constexpr bool kLoads = false;
  __device__ __forceinline__ float2 operator()(int, int) const { return make_float2(0.f, 0.f); }
};
template <class F>
struct PreFn {
  static constexpr bool kLoads = true;
  F f;
  __device__ __forceinline__ float2 operator()(int b, int i) const { return f(b, i); }
};
template <class F>
__device__ __forceinline__ PreFn<F> make_pre(F f) {
  return PreFn<F>{f};
}

// A hook from a callable f(b, index, r, value&).
template <bool STORES, class F>
struct PostFn {
  static constexpr bool kStores = STORES;
  F f;
  __device__ __forceinline__ void operator()(int b, int i, int r, float2& v) const { f(b, i, r, v); }
};
template <bool STORES, class F>
__device__ __forceinline__ PostFn<STORES, F> make_post(F f) {
  return PostFn<STORES, F>{f};
}

// In-place form of the same pass for a batch small enough that every thread
// can hold all of its butterflies at once (U*R <= VALUES; the plan checks
// ceil(B*n/R / NT) <= VALUES/R for every radix): all loads, a
// barrier, then twiddles, DFTs and stores into the same buffer.  It needs no
// scratch, so a workgroup takes half the LDS of the ping-pong form.
// post(b, index, r, value) sees output r of the thread's butterfly (r a
// compile-time constant once unrolled), output `index` of sequence b, just
// before its store (see NoPost).
template <int R, int NT, int VALUES, bool INV, class Post = NoPost, class Pre = NoPre>
__device__ __forceinline__ void inplace_pass(float2* data, int stride, int n, int B, int Ns,
                                             const float2* __restrict__ tw,
                                             const Post& post = Post(), const Pre& pre = Pre()) {
  constexpr int U = inplace_units(R, VALUES);
  constexpr int NB2 = R > 8 ? 4 : (R > 4 ? 3 : (R > 2 ? 2 : 1));
  const int nb = n / R;
  const int total = B * nb;
  const int twstep = n / (Ns * R);
  const int nhi = (n + 63) >> 6;
  const unsigned m_nb = div_magic(nb), m_ns = div_magic(Ns);
  float2 v[U][R];
  int ob[U], oo[U], kk[U], bq[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int idx = threadIdx.x + u * NT;
    const int b = div_small(idx, m_nb);
    const int j = idx - b * nb;
    const int k = j - div_small(j, m_ns) * Ns;
    kk[u] = k;
    bq[u] = b;
    ob[u] = b * stride;
    oo[u] = (j - k) * R + k;
    if (idx < total) {
      const float2* in = data + b * stride;
#pragma unroll
      for (int r = 0; r < R; ++r) v[u][r] = Pre::kLoads ? pre(b, j + r * nb) : in[lpad(j + r * nb)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (threadIdx.x + u * NT < total) {
      if (kk[u] != 0) {
        float2 p2[NB2];
#pragma unroll
        for (int i = 0; i < NB2; ++i) {
          const int m = (kk[u] * twstep) << i;
          p2[i] = cmul(tw[m >> 6], tw[nhi + (m & 63)]);
          if (INV) p2[i].y = -p2[i].y;
        }
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = make_float2(1.0f, 0.0f);
          bool first = true;
#pragma unroll
          for (int i = 0; i < NB2; ++i) {
            if (r & (1 << i)) {
              w = first ? p2[i] : cmul(w, p2[i]);
              first = false;
            }
          }
          v[u][r] = cmul(v[u][r], w);
        }
      }
      Dft<R, INV>::run(v[u]);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        post(bq[u], oo[u] + r * Ns, r, v[u][r]);
        if (!Post::kStores) data[ob[u] + lpad(oo[u] + r * Ns)] = v[u][r];
      }
    }
  }
  __syncthreads();
}

// One in-place pass of the radix `R` (runtime) with the given hooks.
template <int NT, int VALUES, bool INV, class Pre, class Post>
__device__ __forceinline__ void hooked_pass(int R, float2* data, int stride, int n, int B, int Ns,
                                            const float2* __restrict__ tw, const Pre& pre,
                                            const Post& post) {
  switch (R) {
    case 16: inplace_pass<16, NT, VALUES, INV, Post, Pre>(data, stride, n, B, Ns, tw, post, pre); break;
    case 15: inplace_pass<15, NT, VALUES, INV, Post, Pre>(data, stride, n, B, Ns, tw, post, pre); break;
    case 12: inplace_pass<12, NT, VALUES, INV, Post, Pre>(data, stride, n, B, Ns, tw, post, pre); break;
    case 10: inplace_pass<10, NT, VALUES, INV, Post, Pre>(data, stride, n, B, Ns, tw, post, pre); break;
    case 9: inplace_pass<9, NT, VALUES, INV, Post, Pre>(data, stride, n, B, Ns, tw, post, pre); break;
    case 8: inplace_pass<8, NT, VALUES, INV, Post, Pre>(data, stride, n, B, Ns, tw, post, pre); break;
    case 6: inplace_pass<6, NT, VALUES, INV, Post, Pre>(data, stride, n, B, Ns, tw, post, pre); break;
    case 5: inplace_pass<5, NT, VALUES, INV, Post, Pre>(data, stride, n, B, Ns, tw, post, pre); break;
    case 4: inplace_pass<4, NT, VALUES, INV, Post, Pre>(data, stride, n, B, Ns, tw, post, pre); break;
    case 3: inplace_pass<3, NT, VALUES, INV, Post, Pre>(data, stride, n, B, Ns, tw, post, pre); break;
    default: inplace_pass<2, NT, VALUES, INV, Post, Pre>(data, stride, n, B, Ns, tw, post, pre); break;
  }
}

// B sequences at data + b*stride in place, all in one group (see
// inplace_pass for the size condition), the first pass's inputs from `pre`
// and the last pass's outputs through `post` (see NoPre, NoPost).  The
// caller synchronises before the call; the call ends synchronised.
template <int NT, int VALUES, bool INV, class Pre, class Post>
__device__ __forceinline__ void fft_inplace_hooks(float2* data, int stride, int B, const FftDev& f,
                                                  const float2* __restrict__ tw, const Pre& pre,
                                                  const Post& post) {
  const int n = f.n, last = f.npass - 1;
  if (last == 0) {
    hooked_pass<NT, VALUES, INV>(fft_radix(f, 0), data, stride, n, B, 1, tw, pre, post);
    return;
  }
  hooked_pass<NT, VALUES, INV>(fft_radix(f, 0), data, stride, n, B, 1, tw, pre, NoPost());
  int Ns = fft_radix(f, 0);
  for (int p = 1; p < last; ++p) {
    hooked_pass<NT, VALUES, INV>(fft_radix(f, p), data, stride, n, B, Ns, tw, NoPre(), NoPost());
    Ns *= fft_radix(f, p);
  }
  hooked_pass<NT, VALUES, INV>(fft_radix(f, last), data, stride, n, B, Ns, tw, NoPre(), post);
}

// Transform B sequences at data + b*stride in place, `group` sequences at a
// time (see inplace_pass for the size condition on a group).  The caller
// synchronises before the call; the call ends synchronised.
template <int NT, int VALUES, bool INV>
__device__ void fft_inplace(float2* data, int stride, int B, int group, const FftDev& f,
                            const float2* __restrict__ tw) {
  const int n = f.n;
  for (int b0 = 0; b0 < B; b0 += group) {
    float2* a = data + b0 * stride;
    const int Bg = min(group, B - b0);
    int Ns = 1;
    for (int p = 0; p < f.npass; ++p) {
      switch (fft_radix(f, p)) {
        case 16: inplace_pass<16, NT, VALUES, INV>(a, stride, n, Bg, Ns, tw); break;
        case 15: inplace_pass<15, NT, VALUES, INV>(a, stride, n, Bg, Ns, tw); break;
        case 12: inplace_pass<12, NT, VALUES, INV>(a, stride, n, Bg, Ns, tw); break;
        case 10: inplace_pass<10, NT, VALUES, INV>(a, stride, n, Bg, Ns, tw); break;
        case 9: inplace_pass<9, NT, VALUES, INV>(a, stride, n, Bg, Ns, tw); break;
        case 8: inplace_pass<8, NT, VALUES, INV>(a, stride, n, Bg, Ns, tw); break;
        case 6: inplace_pass<6, NT, VALUES, INV>(a, stride, n, Bg, Ns, tw); break;
        case 5: inplace_pass<5, NT, VALUES, INV>(a, stride, n, Bg, Ns, tw); break;
        case 4: inplace_pass<4, NT, VALUES, INV>(a, stride, n, Bg, Ns, tw); break;
        case 3: inplace_pass<3, NT, VALUES, INV>(a, stride, n, Bg, Ns, tw); break;
        default: inplace_pass<2, NT, VALUES, INV>(a, stride, n, Bg, Ns, tw); break;
      }
      Ns *= fft_radix(f, p);
    }
  }
}

// Either form: in place when `scratch` is null (`group` sequences at a time,
// at most VALUES values per thread), else ping-pong through `scratch` (room
// for `group` sequences).
template <int NT, int VALUES, bool INV>
__device__ __forceinline__ void fft_rows(float2* data, int stride, int B, float2* scratch,
                                         int group, const FftDev& f,
                                         const float2* __restrict__ tw);

// Transform B sequences held at data + b*stride (padded layout), using
// `scratch` (room for `group` padded sequences, padded_len(n) apart) as the
// other half of the ping-pong; the results end in place.  The caller synchronises before the call; the call
// ends synchronised.
template <int NT, bool INV>
__device__ void fft_batch(float2* data, int stride, int B, float2* scratch, int group,
                          const FftDev& f, const float2* __restrict__ tw) {
  const int n = f.n;
  for (int b0 = 0; b0 < B; b0 += group) {
    const int Bg = min(group, B - b0);
    float2* a = data + b0 * stride;
    float2* c = scratch;
    int sa = stride, sc = padded_len(n);
    int Ns = 1;
    for (int p = 0; p < f.npass; ++p) {
      switch (fft_radix(f, p)) {
        case 16: stockham_pass<16, NT, INV>(a, sa, c, sc, n, Bg, Ns, tw); break;
        case 15: stockham_pass<15, NT, INV>(a, sa, c, sc, n, Bg, Ns, tw); break;
        case 12: stockham_pass<12, NT, INV>(a, sa, c, sc, n, Bg, Ns, tw); break;
        case 10: stockham_pass<10, NT, INV>(a, sa, c, sc, n, Bg, Ns, tw); break;
        case 9: stockham_pass<9, NT, INV>(a, sa, c, sc, n, Bg, Ns, tw); break;
        case 8: stockham_pass<8, NT, INV>(a, sa, c, sc, n, Bg, Ns, tw); break;
        case 6: stockham_pass<6, NT, INV>(a, sa, c, sc, n, Bg, Ns, tw); break;
        case 5: stockham_pass<5, NT, INV>(a, sa, c, sc, n, Bg, Ns, tw); break;
        case 4: stockham_pass<4, NT, INV>(a, sa, c, sc, n, Bg, Ns, tw); break;
        case 3: stockham_pass<3, NT, INV>(a, sa, c, sc, n, Bg, Ns, tw); break;
        default: stockham_pass<2, NT, INV>(a, sa, c, sc, n, Bg, Ns, tw); break;
      }
      __syncthreads();
      Ns *= fft_radix(f, p);
      float2* t = a; a = c; c = t;
      const int ts = sa; sa = sc; sc = ts;
    }
    if (a == scratch) {  // odd number of passes: copy the results back
      for (int i = threadIdx.x; i < Bg * n; i += NT) {
        const int b = i / n;
        const int e = lpad(i - b * n);
        data[(b0 + b) * stride + e] = scratch[b * padded_len(n) + e];
      }
      __syncthreads();
    }
  }
}

}  // namespace hrt

namespace hrt {
// Copy the two-level twiddle table (ceil(n/64) + 64 entries) into LDS.
template <int NT>
__device__ __forceinline__ void load_twiddles(float2* s_tw, const float2* __restrict__ tw,
                                              int n) {
  const int cnt = ((n + 63) >> 6) + 64;
  for (int i = threadIdx.x; i < cnt; i += NT) s_tw[i] = tw[i];
}
}  // namespace hrt

namespace hrt {
template <int NT, int VALUES, bool INV>
__device__ __forceinline__ void fft_rows(float2* data, int stride, int B, float2* scratch,
                                         int group, const FftDev& f,
                                         const float2* __restrict__ tw) {
  if (scratch == nullptr) fft_inplace<NT, VALUES, INV>(data, stride, B, group, f, tw);
  else fft_batch<NT, INV>(data, stride, B, scratch, group, f, tw);
}
}  // namespace hrt
