// Register-resident two-level FFT for gfx950.
//
// A transform of length L = R1 * R2 (R1, R2 <= 32) runs as two rounds of register
// DFTs with one LDS exchange between them (the "four-step" split):
//   x[i1 + R1 i2]  --DFT_R2 over i2, twiddle W_L^(i1 j2)-->  Y[i1][j2]   (A-layout unit i1)
//   Y[i1][j2]      --exchange through LDS, DFT_R1 over i1--> X[j2 + R2 j1] (B-layout unit j2)
// The same routine run from B-layout to A-layout ("inv_like") takes natural-order
// input at positions j2 + R2 j1 to natural-order output at positions b2 + R1 b1, so a
// forward transform followed by an inverse needs no reordering in between.
//
// A tile holds NT independent transforms and runs on T = NT * R1 threads: one A-layout
// unit per thread, ceil(R2 / R1) B-layout units per thread.  ROW tiles keep each
// transform contiguous in memory (rows); COL tiles interleave NT contiguous columns
// (element m of column b at m * stride + b).  Global loads and stores go straight
// between registers and memory; the LDS holds only the exchange (padded so the lanes of
// a wave fall in distinct banks) and the twiddle table.
//
// Twiddles inside a register DFT are compile-time constants (a constexpr sine/cosine
// series evaluated in double and rounded once to float); the cross twiddles W_L^e come
// from the host's FP64 table in LDS.
#pragma once

#include <utility>

#include "fft_device.hpp"

namespace cola {

// ---------------------------------------------------------------------------------
// Compile-time trigonometry: sin / cos of 2 pi e / r by their Taylor series on the
// reduced angle in (-pi, pi].
// ---------------------------------------------------------------------------------
constexpr double kTwoPiD = 6.283185307179586476925286766559;

constexpr double ct_series(double x, bool cosine) {
  double term = cosine ? 1.0 : x, sum = term;
  for (int n = cosine ? 2 : 3; n < 64; n += 2) {
    term *= -x * x / ((double)(n - 1) * (double)n);
    sum += term;
  }
  return sum;
}
constexpr double ct_angle(int e, int r) {
  e %= r;
  if (e < 0) e += r;
  if (2 * e > r) e -= r;
  return kTwoPiD * (double)e / (double)r;
}
constexpr float ct_cos(int e, int r) { return (float)ct_series(ct_angle(e, r), true); }
constexpr float ct_sin(int e, int r) { return (float)ct_series(ct_angle(e, r), false); }

// Compile-time loop: f(std::integral_constant<int, i>) for i = 0 .. N-1.
template <class F, int... I>
__device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// v * exp(S 2 pi i E / R), E a compile-time exponent.  Multiples of a quarter turn are
// exact swaps and negations.
template <int R, int S, int E>
__device__ __forceinline__ float2 tw_const(float2 v) {
  constexpr int e = ((S * E) % R + R) % R;
  if constexpr (e == 0) {
    return v;
  } else if constexpr (4 * e == R) {
    return make_float2(-v.y, v.x);        // * i
  } else if constexpr (2 * e == R) {
    return make_float2(-v.x, -v.y);       // * -1
  } else if constexpr (4 * e == 3 * R) {
    return make_float2(v.y, -v.x);        // * -i
  } else {
    constexpr float c = ct_cos(e, R), s = ct_sin(e, R);
    return make_float2(v.x * c - v.y * s, v.x * s + v.y * c);
  }
}

// In-register DFT of length R (natural order in and out):
//   x[k] <- sum_n x[n] exp(S 2 pi i n k / R).
// R in {1, 2, 3, 4, 8} directly; otherwise R = P * Q with P = 3 or 4, as sub-DFTs of
// length Q over the P interleaved subsequences, constant twiddles, then length-P DFTs.
template <int R, int S>
__device__ __forceinline__ void dft_reg(float2* x) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2 || R == 3 || R == 4 || R == 8) {
    dft<R, S>(x);
  } else {
    constexpr int P = (R % 3 == 0) ? 3 : 4;
    constexpr int Q = R / P;
    float2 y[P][Q];
    sfor<P>([&](auto a1_) {
      constexpr int a1 = decltype(a1_)::value;
#pragma unroll
      for (int a2 = 0; a2 < Q; ++a2) y[a1][a2] = x[a1 + P * a2];
      dft_reg<Q, S>(y[a1]);
      sfor<Q>([&](auto b2_) {
        constexpr int b2 = decltype(b2_)::value;
        y[a1][b2] = tw_const<R, S, a1 * b2>(y[a1][b2]);
      });
    });
#pragma unroll
    for (int b2 = 0; b2 < Q; ++b2) {
      float2 z[P];
#pragma unroll
      for (int a1 = 0; a1 < P; ++a1) z[a1] = y[a1][b2];
      dft_reg<P, S>(z);
#pragma unroll
      for (int b1 = 0; b1 < P; ++b1) x[b2 + Q * b1] = z[b1];
    }
  }
}

// Split L = R1 * R2 with R2 a power of two (so a row's B-layout units share a wave).
constexpr int pencil_r2(int L) {
  return L == 8 ? 4 : L == 12 ? 4 : L == 16 ? 4 : L == 24 ? 8 : L == 32 ? 8 : L == 48 ? 8 : L == 64 ? 8
       : L == 96 ? 16 : L == 128 ? 16 : L == 192 ? 16 : L == 256 ? 16 : L == 384 ? 16 : L == 512 ? 32
       : L == 768 ? 24 : L == 1024 ? 32 : 0;
}
constexpr int pmax(int a, int b) { return a > b ? a : b; }
constexpr int round_up(int a, int m) { return (a + m - 1) / m * m; }

// Twiddle W_L^e from the FP64-rounded table (tab[m] = exp(-2 pi i m / (L * TWS))),
// conjugated for S = +1.
template <int S, int TWS>
__device__ __forceinline__ float2 tw_table(const float2* tab, int e) {
  float2 w = tab[e * TWS];
  if constexpr (S > 0) w.y = -w.y;
  return w;
}

template <int L_, int NT_, bool ROW_>
struct Pencil {
  static constexpr int L = L_, NT = NT_;
  static constexpr bool ROW = ROW_;
  static constexpr int R2 = pencil_r2(L), R1 = L / R2;
  static constexpr int T = NT * R1;                       // threads per tile
  static constexpr int UB = (NT * R2 + T - 1) / T;        // B-layout units per thread
  static constexpr bool B_FULL = (NT * R2) % T == 0;
  // LDS geometry.  ROW: per transform, [j2][i1] (stride R1+1) for the forward split and
  // [b2][j2] (stride R2+1) for the inverse one.  COL: [i1][j2][b] with i1 stride PF.
  static constexpr int SF = R2 * (R1 + 1), SI = R1 * (R2 + 1);
  static constexpr int PF = round_up(R2 * NT, 32) + NT;
  // COL tiles with several B-layout units per thread exchange in UB chunks of R1
  // j2-columns (the j2 of B-layout slice u is in [u R1, (u+1) R1)), which divides the
  // LDS of the exchange by UB and lets more tiles share a CU.
  static constexpr bool CHUNK = !ROW && UB > 1;
  static constexpr int PC = round_up(R1 * NT, 32) + NT;
  static constexpr int LDS = ROW ? NT * pmax(SF, SI) : (CHUNK ? R1 * PC : R1 * PF);

  static_assert(R2 > 0 && R1 * R2 == L, "unsupported transform length");
  static_assert(R1 <= 32 && R2 <= 32, "register DFTs are at most 32 long");

  // A-layout unit of this thread: transform b, index i1 (< R1).
  __device__ static void a_unit(int& b, int& i1) {
    const int t = threadIdx.x;
    if constexpr (ROW) { b = t / R1; i1 = t % R1; } else { b = t % NT; i1 = t / NT; }
  }
  // B-layout unit u of this thread: transform b, index j2 (< R2); false if unused.
  __device__ static bool b_unit(int u, int& b, int& j2) {
    const int ub = threadIdx.x + T * u;
    if constexpr (ROW) { b = ub / R2; j2 = ub % R2; } else { b = ub % NT; j2 = ub / NT; }
    return B_FULL || ub < NT * R2;
  }
  __device__ static int addr_f(int b, int i1, int j2) {
    if constexpr (ROW) return b * SF + j2 * (R1 + 1) + i1;
    else return i1 * PF + j2 * NT + b;
  }
  __device__ static int addr_i(int b, int j2, int b2) {
    if constexpr (ROW) return b * SI + b2 * (R2 + 1) + j2;
    else return b2 * PF + j2 * NT + b;
  }
  // Offset (in elements) of element m of transform b; `stride` is the row length (ROW)
  // or the column stride (COL).
  __device__ static long elem(int b, int m, long stride) {
    if constexpr (ROW) return (long)b * stride + m;
    else return (long)m * stride + b;
  }

  // A-layout load: a[i2] = element i1 + R1 i2.
  __device__ static void load_a(float2 (&a)[R2], const float2* src, long stride) {
    int b, i1;
    a_unit(b, i1);
#pragma unroll
    for (int i2 = 0; i2 < R2; ++i2) a[i2] = src[elem(b, i1 + R1 * i2, stride)];
  }
  // A-layout store: element b2 + R1 b1 = a[b1].
  __device__ static void store_a(const float2 (&a)[R2], float2* dst, long stride) {
    int b, i1;
    a_unit(b, i1);
#pragma unroll
    for (int i2 = 0; i2 < R2; ++i2) dst[elem(b, i1 + R1 * i2, stride)] = a[i2];
  }
  // B-layout load / store: q[u][j1] is element j2 + R2 j1 of unit u.
  __device__ static void load_b(float2 (&q)[UB][R1], const float2* src, long stride) {
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      int b, j2;
      if (!b_unit(u, b, j2)) continue;
#pragma unroll
      for (int j1 = 0; j1 < R1; ++j1) q[u][j1] = src[elem(b, j2 + R2 * j1, stride)];
    }
  }
  __device__ static void store_b(const float2 (&q)[UB][R1], float2* dst, long stride) {
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      int b, j2;
      if (!b_unit(u, b, j2)) continue;
#pragma unroll
      for (int j1 = 0; j1 < R1; ++j1) dst[elem(b, j2 + R2 * j1, stride)] = q[u][j1];
    }
  }
  // COL tiles whose rows are not evenly spaced: element m of column b sits at
  // src[row(m) + b], row(m) an element offset.
  template <class RowF>
  __device__ static void load_a_rows(float2 (&a)[R2], const float2* src, RowF row) {
    static_assert(!ROW, "row maps are for column tiles");
    int b, i1;
    a_unit(b, i1);
#pragma unroll
    for (int i2 = 0; i2 < R2; ++i2) a[i2] = src[row(i1 + R1 * i2) + b];
  }
  template <class RowF>
  __device__ static void store_a_rows(const float2 (&a)[R2], float2* dst, RowF row) {
    static_assert(!ROW, "row maps are for column tiles");
    int b, i1;
    a_unit(b, i1);
#pragma unroll
    for (int i2 = 0; i2 < R2; ++i2) dst[row(i1 + R1 * i2) + b] = a[i2];
  }
  template <class RowF>
  __device__ static void store_b_rows(const float2 (&q)[UB][R1], float2* dst, RowF row) {
    static_assert(!ROW, "row maps are for column tiles");
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      int b, j2;
      if (!b_unit(u, b, j2)) continue;
#pragma unroll
      for (int j1 = 0; j1 < R1; ++j1) dst[row(j2 + R2 * j1) + b] = q[u][j1];
    }
  }

  // A-layout (positions i1 + R1 i2) -> B-layout (positions j2 + R2 j1), sign S.
  // Destroys a.  The caller has the LDS exchange free on entry (a barrier since its last
  // reads) and the twiddle table visible; returns without a trailing barrier.
  template <int S, int TWS>
  __device__ static void fwd_like(float2 (&a)[R2], float2 (&q)[UB][R1], float2* ex, const float2* tab) {
    int b, i1;
    a_unit(b, i1);
    dft_reg<R2, S>(a);
#pragma unroll
    for (int j2 = 1; j2 < R2; ++j2) a[j2] = c_mul(a[j2], tw_table<S, TWS>(tab, i1 * j2));
    if constexpr (CHUNK) {
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        if (u > 0) __syncthreads();   // the previous chunk has been read
#pragma unroll
        for (int jj = 0; jj < R1; ++jj)
          if (u * R1 + jj < R2) ex[i1 * PC + jj * NT + b] = a[u * R1 + jj];
        __syncthreads();
        int bb, j2;
        if (!b_unit(u, bb, j2)) continue;
#pragma unroll
        for (int k = 0; k < R1; ++k) q[u][k] = ex[k * PC + (j2 - u * R1) * NT + bb];
        dft_reg<R1, S>(q[u]);
      }
    } else {
#pragma unroll
      for (int j2 = 0; j2 < R2; ++j2) ex[addr_f(b, i1, j2)] = a[j2];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        int bb, j2;
        if (!b_unit(u, bb, j2)) continue;
#pragma unroll
        for (int k = 0; k < R1; ++k) q[u][k] = ex[addr_f(bb, k, j2)];
        dft_reg<R1, S>(q[u]);
      }
    }
  }

  // B-layout (positions j2 + R2 j1) -> A-layout (positions b2 + R1 b1), sign S.
  // Destroys q.  Same LDS contract as fwd_like.
  template <int S, int TWS>
  __device__ static void inv_like(float2 (&q)[UB][R1], float2 (&a)[R2], float2* ex, const float2* tab) {
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      int b, j2;
      if (!b_unit(u, b, j2)) continue;
      dft_reg<R1, S>(q[u]);
#pragma unroll
      for (int b2 = 1; b2 < R1; ++b2) q[u][b2] = c_mul(q[u][b2], tw_table<S, TWS>(tab, j2 * b2));
    }
    int b, b2;
    a_unit(b, b2);
    if constexpr (CHUNK) {
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        if (u > 0) __syncthreads();   // the previous chunk has been read
        int bu, j2;
        if (b_unit(u, bu, j2)) {
#pragma unroll
          for (int k = 0; k < R1; ++k) ex[k * PC + (j2 - u * R1) * NT + bu] = q[u][k];
        }
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < R1; ++jj)
          if (u * R1 + jj < R2) a[u * R1 + jj] = ex[b2 * PC + jj * NT + b];
      }
    } else {
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        int bu, j2;
        if (!b_unit(u, bu, j2)) continue;
#pragma unroll
        for (int k = 0; k < R1; ++k) ex[addr_i(bu, j2, k)] = q[u][k];
      }
      __syncthreads();
#pragma unroll
      for (int j2 = 0; j2 < R2; ++j2) a[j2] = ex[addr_i(b, j2, b2)];
    }
    dft_reg<R2, S>(a);
  }

  // ROW tiles: the partner of B-layout unit (b, j2) holding position k = j2 + R2 j1 for
  // position (L - k) mod L is unit (b, (R2 - j2) mod R2) of the same wave, register
  // R1 - 1 - j1 (j2 != 0), or this unit's own register (R1 - j1) mod R1 (j2 == 0).
  // Returns element (L - k) mod L for every register of unit u.
  __device__ static void partner(const float2 (&q)[UB][R1], int u, float2 (&m)[R1]) {
    static_assert(ROW, "partner exchange is for row tiles");
    const int lane = __lane_id();
    const int j2 = (threadIdx.x + T * u) % R2;
    const int src = lane - j2 + ((R2 - j2) & (R2 - 1));
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) {
      const float2 o = q[u][R1 - 1 - j1];
      const float2 s = make_float2(__shfl(o.x, src), __shfl(o.y, src));
      m[j1] = (j2 == 0) ? q[u][(R1 - j1) % R1] : s;
    }
  }
};

}  // namespace cola
