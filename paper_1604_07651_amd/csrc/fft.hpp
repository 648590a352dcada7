// Workgroup-wide mixed-radix Stockham FFTs on sequences held in LDS.
//
// A batch of B complex sequences of length n (n = product of the radices in
// an FftDev) sits in LDS at buf + b*stride.  Every pass reads all of a
// thread's butterfly inputs into registers, synchronises, then writes the
// outputs back in place (the Stockham autosort order), so one LDS buffer is
// enough.  Twiddles come from a table tw[j] = exp(-2 pi i j / n) computed in
// float64 on the host and rounded once.  Forward transforms use
// exp(-2 pi i ...); INV selects exp(+2 pi i ...), unnormalised.
#pragma once

#include <hip/hip_runtime.h>

namespace hrt {

constexpr int kMaxPassesDev = 24;

struct FftDev {
  int n;
  int npass;
  int radix[kMaxPassesDev];
};

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

// One radix-R Stockham pass over B sequences of length n.  Ns is the length
// of the sub-transforms already combined; CAP bounds B*n (it sizes the
// per-thread register staging).
template <int R, int NT, int CAP, bool INV>
__device__ __forceinline__ void stockham_pass(float2* buf, int n, int stride,
                                              int B, int Ns,
                                              const float2* __restrict__ tw) {
  constexpr int MAXB = (CAP + R * NT - 1) / (R * NT);
  const int nb = n / R;
  const int total = B * nb;
  const int twstep = n / (Ns * R);
  float2 v[MAXB][R];
#pragma unroll
  for (int t = 0; t < MAXB; ++t) {
    const int idx = static_cast<int>(threadIdx.x) + t * NT;
    if (idx < total) {
      const int b = idx / nb;
      const int j = idx - b * nb;
      const int k = j % Ns;
      const float2* src = buf + b * stride + j;
#pragma unroll
      for (int r = 0; r < R; ++r) v[t][r] = src[r * nb];
      if (k != 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[r * k * twstep];
          if (INV) w.y = -w.y;
          v[t][r] = cmul(v[t][r], w);
        }
      }
      Dft<R, INV>::run(v[t]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < MAXB; ++t) {
    const int idx = static_cast<int>(threadIdx.x) + t * NT;
    if (idx < total) {
      const int b = idx / nb;
      const int j = idx - b * nb;
      const int k = j % Ns;
      float2* dst = buf + b * stride + (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * Ns] = v[t][r];
    }
  }
  __syncthreads();
}

// Full transform of B sequences (caller synchronises before the call).
template <int NT, int CAP, bool INV>
__device__ void fft_batch(float2* buf, int stride, int B, const FftDev& f,
                          const float2* __restrict__ tw) {
  int Ns = 1;
  for (int p = 0; p < f.npass; ++p) {
    const int R = f.radix[p];
    switch (R) {
      case 8: stockham_pass<8, NT, CAP, INV>(buf, f.n, stride, B, Ns, tw); break;
      case 4: stockham_pass<4, NT, CAP, INV>(buf, f.n, stride, B, Ns, tw); break;
      case 2: stockham_pass<2, NT, CAP, INV>(buf, f.n, stride, B, Ns, tw); break;
      case 3: stockham_pass<3, NT, CAP, INV>(buf, f.n, stride, B, Ns, tw); break;
      default: stockham_pass<5, NT, CAP, INV>(buf, f.n, stride, B, Ns, tw); break;
    }
    Ns *= R;
  }
}

}  // namespace hrt
