// Pencil passes of the 3D real FFT on gfx950, with the k-space operator fused into
// the last forward / first inverse pass.
//
// Mesh layout: a real field is [x][y][z] with z fastest (n floats per row).  Its
// half spectrum uses the same memory as [x][y][kz] complex with kz = 0..n/2-1
// (n/2 complex per row): the kz = n/2 plane is never stored because every
// k-space operator of the method zeroes Nyquist-index modes.
//
// Passes (each reads and writes every element once, HBM-bound):
//   z forward   rows of n reals -> n/2 complex (half-length complex FFT + split)
//   y / x       strided column FFTs over tiles of B contiguous kz columns
//   x multiply  forward x FFT, multiplier, inverse x FFT into several outputs
//   z inverse   rows of n/2 complex -> n reals, with fused epilogues
#include "fft_device.hpp"
#include "internal.hpp"

namespace cola {

constexpr int kThreads = 256;

// ---------------------------------------------------------------------------------
// Tile shapes per transform length.
// ---------------------------------------------------------------------------------
constexpr int pow2_factor(int v) { return (v & (-v)); }
constexpr int floor_pow2(int v) { return v < 2 ? 1 : 2 * floor_pow2(v / 2); }
constexpr int min_i(int a, int b) { return a < b ? a : b; }
constexpr int max_i(int a, int b) { return a > b ? a : b; }

// Rows per block of the z passes: a 32 KB LDS tile of n/2 complex rows.
template <int N>
constexpr int z_rows() { return min_i(64, floor_pow2(4096 / (N / 2))); }
// Rows per block of the Hessian z pass (keeps several fields in registers).
template <int N>
constexpr int zh_rows() { return min_i(64, floor_pow2(1024 / (N / 2))); }
// Columns per block of the strided passes: 16 (128-byte segments) while the tile
// stays within 64 KB, limited to a power of two dividing n/2.
template <int N>
constexpr int col_width() {
  return min_i(pow2_factor(N / 2), min_i(16, max_i(2, floor_pow2(8192 / N))));
}

// Threads per block of the strided passes: 512 for tiles of >= 8192 elements so
// each lane holds at most 16 complex values.
constexpr int col_threads_for(int n, int b) { return n * b >= 8192 ? 512 : 256; }
// A column width is usable when it divides n/2 and the tile fits in 64 KB.
template <int N, int B>
constexpr bool col_ok() { return B >= 2 && B <= pow2_factor(N / 2) && N * B <= 8192; }

__device__ __forceinline__ int pick_comp(int c, int nx, int ny, int nz) {
  return c == 0 ? nx : (c == 1 ? ny : nz);
}
// Hessian components in output order xx, yy, zz, xy, yz, zx.
__device__ __forceinline__ int hess_a(int p) { return p < 3 ? p : p - 3; }
__device__ __forceinline__ int hess_b(int p) { return p < 3 ? p : (p - 2) % 3; }

__device__ __forceinline__ void load_twiddles(float2* stw, const float2* __restrict__ tw, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) stw[i] = tw[i];
}

// ---------------------------------------------------------------------------------
// z forward: real rows -> half complex rows.
// X[k] = (Z[k] + conj Z[M-k]) / 2 - i W^k (Z[k] - conj Z[M-k]) / 2, W = exp(-2 pi i / N),
// where Z is the length-M = N/2 DFT of z[m] = x[2m] + i x[2m+1].
// ---------------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(kThreads) void k_zfwd(const float* in, float2* out, const float2* __restrict__ tw) {
  constexpr int M = N / 2;
  constexpr int BR = z_rows<N>();
  __shared__ __align__(16) float2 tile[BR * M];
  __shared__ float2 stw[N];
  load_twiddles(stw, tw, N);
  const long row0 = (long)blockIdx.x * BR;
  const float4* src = reinterpret_cast<const float4*>(in + row0 * N);
  for (int idx = threadIdx.x; idx < BR * M / 2; idx += kThreads) reinterpret_cast<float4*>(tile)[idx] = src[idx];
  __syncthreads();
  fft_tile<M, BR, kThreads, 1, M, true, -1, 2>(tile, stw);
  // X[k] and X[M-k] both come from the pair (Z[k], Z[M-k]).
  constexpr int Q = M / 2 + 1;
  for (int idx = threadIdx.x; idx < BR * Q; idx += kThreads) {
    const int b = idx / Q, k = idx % Q;
    float2* dst = out + (row0 + b) * M;
    const float2 zk = tile[b * M + k];
    const float2 zm = tile[b * M + ((M - k) % M)];
    const float2 a = c_scale(c_add(zk, c_conj(zm)), 0.5f);
    const float2 d = c_scale(c_sub(zk, c_conj(zm)), 0.5f);
    dst[k] = c_add(a, mul_si<-1>(c_mul(stw[k], d)));
    if (k != 0 && k != M - k) {
      const float2 a2 = c_scale(c_add(zm, c_conj(zk)), 0.5f);
      const float2 d2 = c_scale(c_sub(zm, c_conj(zk)), 0.5f);
      dst[M - k] = c_add(a2, mul_si<-1>(c_mul(stw[M - k], d2)));
    }
  }
}

// ---------------------------------------------------------------------------------
// z inverse: half complex rows -> real rows (unnormalised, times `scale`).
// Z'[k] = (X[k] + conj X[M-k]) + i W^-k (X[k] - conj X[M-k]) with X[M] = 0;
// its unnormalised inverse length-M DFT is x[2m] + i x[2m+1].
// ---------------------------------------------------------------------------------
// Requires stw to be visible to the whole block on entry (callers synchronise
// after loading it).
template <int N, int BR>
__device__ __forceinline__ void zinv_tile(float2* tile, const float2* stw, const float2* src) {
  constexpr int M = N / 2;
  constexpr int Q = M / 2 + 1;   // work items per row: k = 0..M/2, each also producing M - k
  // Each item loads X[k] and X[M-k] straight from memory and writes Z'[k], Z'[M-k].
  for (int idx = threadIdx.x; idx < BR * Q; idx += kThreads) {
    const int b = idx / Q, k = idx % Q;
    const float2* row = src + b * M;
    float2* out = tile + b * M;
    const float2 xk = row[k];
    if (k == 0) {
      out[0] = c_add(xk, mul_si<1>(xk));                         // X[M] = 0
    } else {
      const float2 xm = row[M - k];
      out[k] = c_add(c_add(xk, c_conj(xm)), mul_si<1>(c_mul(c_conj(stw[k]), c_sub(xk, c_conj(xm)))));
      if (k != M - k)
        out[M - k] = c_add(c_add(xm, c_conj(xk)), mul_si<1>(c_mul(c_conj(stw[M - k]), c_sub(xm, c_conj(xk)))));
    }
  }
  __syncthreads();
  fft_tile<M, BR, kThreads, 1, M, true, 1, 2>(tile, stw);
}

template <int N, int EPI>
__global__ __launch_bounds__(kThreads) void k_zinv(FieldPtrs in, FieldPtrs out, const float2* __restrict__ tw,
                                                   EpiArgs e) {
  constexpr int M = N / 2;
  constexpr int BR = z_rows<N>();
  __shared__ __align__(16) float2 tile[BR * M];
  __shared__ float2 stw[N];
  load_twiddles(stw, tw, N);
  __syncthreads();   // zinv_tile reads the twiddles before its first barrier
  const int f = blockIdx.y;
  const long row0 = (long)blockIdx.x * BR;
  zinv_tile<N, BR>(tile, stw, in.p[f] + row0 * M);
  float4* dst = reinterpret_cast<float4*>(reinterpret_cast<float*>(out.p[f]) + row0 * N);
  if constexpr (EPI == kEpiStore) {
    for (int idx = threadIdx.x; idx < BR * M / 2; idx += kThreads) {
      const float4 ab = reinterpret_cast<const float4*>(tile)[idx];
      dst[idx] = make_float4(ab.x * e.scale, ab.y * e.scale, ab.z * e.scale, ab.w * e.scale);
    }
  } else {
    const long off = f * e.comp_stride + row0 * N;
    const float4* s1 = reinterpret_cast<const float4*>(e.s1 + off);
    float4* s = reinterpret_cast<float4*>(e.s + off);
    float4* v = reinterpret_cast<float4*>(e.v + off);
    for (int idx = threadIdx.x; idx < BR * M / 2; idx += kThreads) {
      const float4 ab = reinterpret_cast<const float4*>(tile)[idx];
      const float4 x2 = make_float4(ab.x * e.scale, ab.y * e.scale, ab.z * e.scale, ab.w * e.scale);
      const float4 x1 = s1[idx];
      dst[idx] = x2;
      s[idx] = make_float4(e.d1 * x1.x + e.d2 * x2.x, e.d1 * x1.y + e.d2 * x2.y,
                           e.d1 * x1.z + e.d2 * x2.z, e.d1 * x1.w + e.d2 * x2.w);
      v[idx] = make_float4(e.v1 * x1.x + e.v2 * x2.x, e.v1 * x1.y + e.v2 * x2.y,
                           e.v1 * x1.z + e.v2 * x2.z, e.v1 * x1.w + e.v2 * x2.w);
    }
  }
}

// Six Hessian fields -> S, one field at a time through the same LDS tile.
template <int N>
__global__ __launch_bounds__(kThreads) void k_zinv_hess(FieldPtrs in, float* out, const float2* __restrict__ tw,
                                                        float scale) {
  constexpr int M = N / 2;
  constexpr int BR = zh_rows<N>();
  constexpr int PER = ceil_div(BR * M, kThreads);
  __shared__ __align__(16) float2 tile[BR * M];
  __shared__ float2 stw[N];
  load_twiddles(stw, tw, N);
  __syncthreads();   // zinv_tile reads the twiddles before its first barrier
  const long row0 = (long)blockIdx.x * BR;
  float2 dg[3][PER];
  float2 acc[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) acc[i] = make_float2(0.f, 0.f);
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    zinv_tile<N, BR>(tile, stw, in.p[f] + row0 * M);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = threadIdx.x + i * kThreads;
      if ((BR * M) % kThreads == 0 || idx < BR * M) {
        const float2 t = c_scale(tile[idx], scale);
        if (f < 3) {
          dg[f][i] = t;
        } else {
          acc[i].x -= t.x * t.x;
          acc[i].y -= t.y * t.y;
        }
      }
    }
    __syncthreads();
  }
  float2* dst = reinterpret_cast<float2*>(out + row0 * N);
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int idx = threadIdx.x + i * kThreads;
    if ((BR * M) % kThreads == 0 || idx < BR * M) {
      float2 r = acc[i];
      r.x += dg[0][i].x * dg[1][i].x + dg[1][i].x * dg[2][i].x + dg[2][i].x * dg[0][i].x;
      r.y += dg[0][i].y * dg[1][i].y + dg[1][i].y * dg[2][i].y + dg[2][i].y * dg[0][i].y;
      dst[idx] = r;
    }
  }
}

// ---------------------------------------------------------------------------------
// Strided column pass: tile = n elements along inner_stride x B contiguous columns.
// LDS layout [m][b] (b fastest): global float4 loads cover 2 columns each.
// ---------------------------------------------------------------------------------
template <int N, int B, int T>
__device__ __forceinline__ void col_load(float2* tile, const float2* src, long inner_stride) {
  for (int idx = threadIdx.x; idx < N * B / 2; idx += T) {
    const int m = idx / (B / 2), q = idx % (B / 2);
    reinterpret_cast<float4*>(tile)[idx] = *reinterpret_cast<const float4*>(src + m * inner_stride + 2 * q);
  }
}

template <int N, int B, int T>
__device__ __forceinline__ void col_store(const float2* tile, float2* dst, long inner_stride) {
  for (int idx = threadIdx.x; idx < N * B / 2; idx += T) {
    const int m = idx / (B / 2), q = idx % (B / 2);
    *reinterpret_cast<float4*>(dst + m * inner_stride + 2 * q) = reinterpret_cast<const float4*>(tile)[idx];
  }
}

template <int N, int B, int S, int T = col_threads_for(N, B)>
__global__ __launch_bounds__(T) void k_col(FieldPtrs in, FieldPtrs out, long outer_stride, long inner_stride,
                                           int ntiles_c, const float2* __restrict__ tw) {
  __shared__ __align__(16) float2 tile[N * B];
  __shared__ float2 stw[N];
  load_twiddles(stw, tw, N);
  const int f = blockIdx.y;
  const int tc = blockIdx.x % ntiles_c;
  const long o = blockIdx.x / ntiles_c;
  const long origin = o * outer_stride + (long)tc * B;
  col_load<N, B, T>(tile, in.p[f] + origin, inner_stride);
  __syncthreads();
  fft_tile<N, B, T, B, 1, false, S, 1>(tile, stw);
  col_store<N, B, T>(tile, out.p[f] + origin, inner_stride);
}

// ---------------------------------------------------------------------------------
// x pass with multiplier.  Tile = n elements along x (stride n * n/2) x B kz columns
// at fixed y.  Mode numbers: nx from the row m, ny from y, nz = kz (< n/2).
// Modes with nx or ny equal to n/2, and the k = 0 mode, get multiplier 0.
// ---------------------------------------------------------------------------------
template <int N, int B, int MODE, int T = col_threads_for(N, B)>
__global__ __launch_bounds__(T) void k_xmul(const float2* in, FieldPtrs out, int nout, MulArgs ma,
                                            const float2* __restrict__ tw) {
  constexpr int H = N / 2;
  constexpr int NT = H / B;
  constexpr int PER = ceil_div(N * B, T);
  constexpr bool FULL = (N * B) % T == 0;
  __shared__ __align__(16) float2 tile[N * B];
  __shared__ float2 stw[N];
  load_twiddles(stw, tw, N);
  const int tc = blockIdx.x % NT;
  const int y = blockIdx.x / NT;
  const long inner = (long)N * H;
  const long origin = (long)y * H + tc * B;
  col_load<N, B, T>(tile, in + origin, inner);
  __syncthreads();
  fft_tile<N, B, T, B, 1, false, -1, 1>(tile, stw);
  // The forward spectrum stays in registers; mode numbers are recomputed per use.
  float2 xs[PER];
  const int ny = (y <= H) ? y : y - N;
  const bool ny_ok = (y != H);
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int idx = threadIdx.x + i * T;
    const int m = idx / B, b = idx % B;
    const int nx = (m <= H) ? m : m - N;
    const int nz = tc * B + b;
    const bool keep = (FULL || idx < N * B) && ny_ok && (m != H) && (nx != 0 || ny != 0 || nz != 0);
    xs[i] = keep ? tile[idx] : make_float2(0.f, 0.f);
  }
  for (int o = 0; o < nout; ++o) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = threadIdx.x + i * T;
      if (!FULL && idx >= N * B) continue;
      const int m = idx / B, b = idx % B;
      const int nx = (m <= H) ? m : m - N;
      const int nz = tc * B + b;
      const int nsq = max_i(1, nx * nx + ny * ny + nz * nz);
      float2 r;
      if constexpr (MODE == kMulGrad) {
        const int nj = pick_comp(o, nx, ny, nz);
        r = mul_si<1>(c_scale(xs[i], ma.c * (float)nj / (float)nsq));   // i c n_j / n^2 X
      } else {
        const float t = ma.tab[nsq];
        if (o < 3) {
          const int nj = pick_comp(o, nx, ny, nz);
          r = mul_si<1>(c_scale(xs[i], t * (float)nj));                  // s1_j
        } else {
          const int na = pick_comp(hess_a(o - 3), nx, ny, nz);
          const int nb = pick_comp(hess_b(o - 3), nx, ny, nz);
          r = c_scale(xs[i], ma.kf * t * (float)(na * nb));              // phi_ab
        }
      }
      tile[idx] = r;
    }
    __syncthreads();
    fft_tile<N, B, T, B, 1, false, 1, 1>(tile, stw);
    col_store<N, B, T>(tile, out.p[o] + origin, inner);
  }
}

// ---------------------------------------------------------------------------------
// Transposed x pass (adjoint of k_xmul): every input is forward transformed along x,
// multiplied by the complex conjugate of its multiplier and accumulated; the sum is
// inverse transformed into the single output.
// ---------------------------------------------------------------------------------
template <int N, int B, int MODE, int T = col_threads_for(N, B)>
__global__ __launch_bounds__(T) void k_xmul_adj(FieldPtrs in, int nin, float2* out, MulArgs ma,
                                                const float2* __restrict__ tw) {
  constexpr int H = N / 2;
  constexpr int NT = H / B;
  constexpr int PER = ceil_div(N * B, T);
  constexpr bool FULL = (N * B) % T == 0;
  __shared__ __align__(16) float2 tile[N * B];
  __shared__ float2 stw[N];
  load_twiddles(stw, tw, N);
  const int tc = blockIdx.x % NT;
  const int y = blockIdx.x / NT;
  const long inner = (long)N * H;
  const long origin = (long)y * H + tc * B;
  const int ny = (y <= H) ? y : y - N;
  const bool ny_ok = (y != H);
  float2 acc[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) acc[i] = make_float2(0.f, 0.f);
  for (int f = 0; f < nin; ++f) {
    if (f > 0) __syncthreads();
    col_load<N, B, T>(tile, in.p[f] + origin, inner);
    __syncthreads();
    fft_tile<N, B, T, B, 1, false, -1, 1>(tile, stw);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = threadIdx.x + i * T;
      if (!FULL && idx >= N * B) continue;
      const int m = idx / B, b = idx % B;
      const int nx = (m <= H) ? m : m - N;
      const int nz = tc * B + b;
      const bool keep = ny_ok && (m != H) && (nx != 0 || ny != 0 || nz != 0);
      if (!keep) continue;
      const int nsq = nx * nx + ny * ny + nz * nz;
      const float2 x = tile[idx];
      float2 r;
      if constexpr (MODE == kMulGrad) {
        const int nj = pick_comp(f, nx, ny, nz);
        r = mul_si<-1>(c_scale(x, ma.c * (float)nj / (float)nsq));    // conj(i c n_j / n^2) X
      } else {
        const float t = ma.tab[nsq];
        if (f < 3) {
          const int nj = pick_comp(f, nx, ny, nz);
          r = mul_si<-1>(c_scale(x, t * (float)nj));                     // conj(i n_j t) X
        } else {
          const int na = pick_comp(hess_a(f - 3), nx, ny, nz);
          const int nb = pick_comp(hess_b(f - 3), nx, ny, nz);
          r = c_scale(x, ma.kf * t * (float)(na * nb));                   // real multiplier
        }
      }
      acc[i] = c_add(acc[i], r);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int idx = threadIdx.x + i * T;
    if (FULL || idx < N * B) tile[idx] = acc[i];
  }
  __syncthreads();
  fft_tile<N, B, T, B, 1, false, 1, 1>(tile, stw);
  col_store<N, B, T>(tile, out + origin, inner);
}

// ---------------------------------------------------------------------------------
// Host dispatch.
// ---------------------------------------------------------------------------------
#define COLA_FOR_EACH_SIZE(X) \
  X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

bool fft_size_supported(int n) {
  switch (n) {
#define COLA_CASE(N) case N:
    COLA_FOR_EACH_SIZE(COLA_CASE)
#undef COLA_CASE
    return true;
    default:
      return false;
  }
}

template <int N>
static hipError_t zfwd_t(const float* in, float2* out, long nrows, const float2* tw, hipStream_t st) {
  constexpr int BR = z_rows<N>();
  if (nrows % BR) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_zfwd<N>, dim3(nrows / BR), dim3(kThreads), 0, st, in, out, tw);
  return hipGetLastError();
}

template <int N>
static hipError_t zinv_t(FieldPtrs in, FieldPtrs out, int nf, long nrows, const float2* tw, int epi,
                         EpiArgs e, hipStream_t st) {
  constexpr int BR = z_rows<N>();
  if (nrows % BR) return hipErrorInvalidValue;
  dim3 grid(nrows / BR, nf);
  if (epi == kEpiStore)
    hipLaunchKernelGGL((k_zinv<N, kEpiStore>), grid, dim3(kThreads), 0, st, in, out, tw, e);
  else
    hipLaunchKernelGGL((k_zinv<N, kEpiLptFinal>), grid, dim3(kThreads), 0, st, in, out, tw, e);
  return hipGetLastError();
}

template <int N>
static hipError_t zinv_hess_t(FieldPtrs in, float* out, long nrows, const float2* tw, float scale,
                              hipStream_t st) {
  constexpr int BR = zh_rows<N>();
  if (nrows % BR) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_zinv_hess<N>, dim3(nrows / BR), dim3(kThreads), 0, st, in, out, tw, scale);
  return hipGetLastError();
}

template <int N, int B>
static hipError_t col_tb(int dir, FieldPtrs in, FieldPtrs out, int nf, int n_outer, long outer_stride,
                         long inner_stride, int ncols, const float2* tw, hipStream_t st) {
  if constexpr (col_ok<N, B>()) {
    if (ncols % B) return hipErrorInvalidValue;
    constexpr int T = col_threads_for(N, B);
    const int ntc = ncols / B;
    dim3 grid((unsigned)((long)n_outer * ntc), nf);
    if (dir < 0)
      hipLaunchKernelGGL((k_col<N, B, -1>), grid, dim3(T), 0, st, in, out, outer_stride, inner_stride, ntc, tw);
    else
      hipLaunchKernelGGL((k_col<N, B, 1>), grid, dim3(T), 0, st, in, out, outer_stride, inner_stride, ntc, tw);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int N>
static hipError_t col_t(int dir, FieldPtrs in, FieldPtrs out, int nf, int n_outer, long outer_stride,
                        long inner_stride, int ncols, const float2* tw, int width, hipStream_t st) {
  switch (width ? width : col_width<N>()) {
    case 4: return col_tb<N, 4>(dir, in, out, nf, n_outer, outer_stride, inner_stride, ncols, tw, st);
    case 8: return col_tb<N, 8>(dir, in, out, nf, n_outer, outer_stride, inner_stride, ncols, tw, st);
    case 16: return col_tb<N, 16>(dir, in, out, nf, n_outer, outer_stride, inner_stride, ncols, tw, st);
    default: return hipErrorInvalidValue;
  }
}

template <int N, int B>
static hipError_t xmul_tb(int mode, const float2* in, FieldPtrs out, int nout, MulArgs m, const float2* tw,
                          hipStream_t st) {
  if constexpr (col_ok<N, B>()) {
    constexpr int T = col_threads_for(N, B);
    dim3 grid(N * ((N / 2) / B));
    if (mode == kMulGrad)
      hipLaunchKernelGGL((k_xmul<N, B, kMulGrad>), grid, dim3(T), 0, st, in, out, nout, m, tw);
    else
      hipLaunchKernelGGL((k_xmul<N, B, kMulLpt1>), grid, dim3(T), 0, st, in, out, nout, m, tw);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

// Default x-pass width: 8 columns where valid (the multi-output x pass holds the
// forward spectrum in registers, so narrower tiles keep more blocks resident).
template <int N>
constexpr int xmul_width() { return col_ok<N, 8>() ? 8 : col_width<N>(); }

template <int N>
static hipError_t xmul_t(int mode, const float2* in, FieldPtrs out, int nout, MulArgs m, const float2* tw,
                         int width, hipStream_t st) {
  switch (width ? width : xmul_width<N>()) {
    case 4: return xmul_tb<N, 4>(mode, in, out, nout, m, tw, st);
    case 8: return xmul_tb<N, 8>(mode, in, out, nout, m, tw, st);
    case 16: return xmul_tb<N, 16>(mode, in, out, nout, m, tw, st);
    default: return hipErrorInvalidValue;
  }
}

template <int N>
static hipError_t xmul_adj_t(int mode, FieldPtrs in, int nin, float2* out, MulArgs m, const float2* tw,
                             hipStream_t st) {
  constexpr int B = xmul_width<N>();
  constexpr int T = col_threads_for(N, B);
  dim3 grid(N * ((N / 2) / B));
  if (mode == kMulGrad)
    hipLaunchKernelGGL((k_xmul_adj<N, B, kMulGrad>), grid, dim3(T), 0, st, in, nin, out, m, tw);
  else
    hipLaunchKernelGGL((k_xmul_adj<N, B, kMulLpt1>), grid, dim3(T), 0, st, in, nin, out, m, tw);
  return hipGetLastError();
}

template <int N>
static bool width_ok(int w) {
  switch (w) {
    case 0: return true;
    case 4: return col_ok<N, 4>();
    case 8: return col_ok<N, 8>();
    case 16: return col_ok<N, 16>();
    default: return false;
  }
}

bool fft_width_supported(int n, int width) {
  switch (n) {
#define COLA_CASE(N) \
  case N:            \
    return width_ok<N>(width);
    COLA_FOR_EACH_SIZE(COLA_CASE)
#undef COLA_CASE
    default:
      return false;
  }
}

hipError_t launch_zfwd(int n, const float* in, float2* out, long nrows, const float2* tw, hipStream_t st) {
  switch (n) {
#define COLA_CASE(N) \
  case N:            \
    return zfwd_t<N>(in, out, nrows, tw, st);
    COLA_FOR_EACH_SIZE(COLA_CASE)
#undef COLA_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_zinv(int n, FieldPtrs in, FieldPtrs out, int nf, long nrows, const float2* tw, int epi,
                       EpiArgs e, hipStream_t st) {
  switch (n) {
#define COLA_CASE(N) \
  case N:            \
    return zinv_t<N>(in, out, nf, nrows, tw, epi, e, st);
    COLA_FOR_EACH_SIZE(COLA_CASE)
#undef COLA_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_zinv_hessian(int n, FieldPtrs in, float* out, long nrows, const float2* tw, float scale,
                               hipStream_t st) {
  switch (n) {
#define COLA_CASE(N) \
  case N:            \
    return zinv_hess_t<N>(in, out, nrows, tw, scale, st);
    COLA_FOR_EACH_SIZE(COLA_CASE)
#undef COLA_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_col(int n, int dir, FieldPtrs in, FieldPtrs out, int nf, int n_outer, long outer_stride,
                      long inner_stride, int ncols, const float2* tw, int width, hipStream_t st) {
  switch (n) {
#define COLA_CASE(N) \
  case N:            \
    return col_t<N>(dir, in, out, nf, n_outer, outer_stride, inner_stride, ncols, tw, width, st);
    COLA_FOR_EACH_SIZE(COLA_CASE)
#undef COLA_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_xmul_adj(int n, int mode, FieldPtrs in, int nin, float2* out, MulArgs m, const float2* tw,
                           hipStream_t st) {
  switch (n) {
#define COLA_CASE(N) \
  case N:            \
    return xmul_adj_t<N>(mode, in, nin, out, m, tw, st);
    COLA_FOR_EACH_SIZE(COLA_CASE)
#undef COLA_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_xmul(int n, int mode, const float2* in, FieldPtrs out, int nout, MulArgs m, const float2* tw,
                       int width, hipStream_t st) {
  switch (n) {
#define COLA_CASE(N) \
  case N:            \
    return xmul_t<N>(mode, in, out, nout, m, tw, width, st);
    COLA_FOR_EACH_SIZE(COLA_CASE)
#undef COLA_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace cola
