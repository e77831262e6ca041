// Device-side FFT building blocks for gfx950: complex arithmetic and the in-register
// radix-2/3/4/8 DFTs that the register FFT (fft_pencil.hpp) is built from.
#pragma once

#include <hip/hip_runtime.h>

namespace cola {

__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 c_conj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 c_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// Multiply by S*i, S = -1 for the forward transform, +1 for the inverse.
template <int S>
__device__ __forceinline__ float2 mul_si(float2 a) {
  return S < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

template <int S>
__device__ __forceinline__ void dft2(float2* x) {
  float2 t = x[0];
  x[0] = c_add(t, x[1]);
  x[1] = c_sub(t, x[1]);
}

template <int S>
__device__ __forceinline__ void dft3(float2* x) {
  const float c1 = -0.5f;
  const float s1 = S * 0.866025403784438647f;  // sin(S * 2 pi / 3)
  float2 t = c_add(x[1], x[2]);
  float2 d = c_sub(x[1], x[2]);
  float2 m = make_float2(x[0].x + c1 * t.x, x[0].y + c1 * t.y);
  float2 r = make_float2(-s1 * d.y, s1 * d.x);  // i * s1 * d
  x[0] = c_add(x[0], t);
  x[1] = c_add(m, r);
  x[2] = c_sub(m, r);
}

template <int S>
__device__ __forceinline__ void dft4(float2* x) {
  float2 a0 = c_add(x[0], x[2]);
  float2 a1 = c_sub(x[0], x[2]);
  float2 a2 = c_add(x[1], x[3]);
  float2 a3 = mul_si<S>(c_sub(x[1], x[3]));
  x[0] = c_add(a0, a2);
  x[2] = c_sub(a0, a2);
  x[1] = c_add(a1, a3);
  x[3] = c_sub(a1, a3);
}

// Radix 8 as a radix-2 split followed by two radix-4 DFTs.
template <int S>
__device__ __forceinline__ void dft8(float2* x) {
  const float r = 0.707106781186547524f;
  float2 a[4], b[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    a[n] = c_add(x[n], x[n + 4]);
    b[n] = c_sub(x[n], x[n + 4]);
  }
  b[1] = c_mul(b[1], make_float2(r, S * r));
  b[2] = mul_si<S>(b[2]);
  b[3] = c_mul(b[3], make_float2(-r, S * r));
  dft4<S>(a);
  dft4<S>(b);
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    x[2 * n] = a[n];
    x[2 * n + 1] = b[n];
  }
}

template <int R, int S>
__device__ __forceinline__ void dft(float2* x) {
  if constexpr (R == 2) dft2<S>(x);
  else if constexpr (R == 3) dft3<S>(x);
  else if constexpr (R == 4) dft4<S>(x);
  else dft8<S>(x);
}


}  // namespace cola
