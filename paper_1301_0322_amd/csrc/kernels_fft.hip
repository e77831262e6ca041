// Pencil passes of the 3D real FFT on gfx950, with the k-space operator fused into
// the last forward / first inverse pass.
//
// Mesh layout: a real field is [x][y][z] with z fastest (n floats per row).  Its
// half spectrum uses the same memory as [x][y][kz] complex with kz = 0..n/2-1
// (n/2 complex per row): the kz = n/2 plane is never stored because every
// k-space operator of the method zeroes Nyquist-index modes.
//
// Rotated planes: between the y passes and the x pass the half spectrum may be held
// with the rows of every x-plane rotated by `rot` rows per plane: row y of plane x at
// row (y + rot x) mod n.  The x pass reads one row from each of the n planes; with
// rot = 0 those rows lie exactly n^2/2 complex apart (4 MB at n = 1024), a power-of-
// two stride that sends a column's loads to the same few HBM channels, and a rotation
// spreads them.  A y pass owns whole columns of a plane, so the forward one stores
// rotated and the inverse one loads rotated, in place.  The x passes take rot as a
// multiple of R2 = n / R1 (their register DFT split n = R1 R2): a thread holds planes
// x = i1 + R1 i2, whose rows (y + rot i1) mod n then do not depend on i2, so each
// thread's 2 R2 loads and stores keep one stride.
//
// Passes (each reads and writes every element once, HBM-bound):
//   z forward   rows of n reals -> n/2 complex (half-length complex FFT + split)
//   y / x       strided column FFTs over tiles of B contiguous kz columns
//   x multiply  forward x FFT, multiplier, inverse x FFT into several outputs
//   z inverse   rows of n/2 complex -> n reals, with fused epilogues
// Every pass is a tile of the two-level register FFT (fft_pencil.hpp): data moves
// between HBM and registers directly, with one LDS exchange per transform.
#include "fft_pencil.hpp"
#include "internal.hpp"

namespace cola {

constexpr int pow2_factor(int v) { return (v & (-v)); }
constexpr int kXcdsFft = 8;   // XCDs; blocks b and b + 8 run on the same one
constexpr int min_i(int a, int b) { return a < b ? a : b; }

// Rows per block of the z passes: a power of two with at most 256 threads and an LDS
// exchange of at most 36 KB.
template <int M>
constexpr int z_rows() {
  constexpr int r2 = pencil_r2(M), r1 = M / r2;
  constexpr int per_row = pmax(r2 * (r1 + 1), r1 * (r2 + 1));
  int rows = 1;
  while (2 * rows * r1 <= 256 && 2 * rows * per_row <= 4608) rows *= 2;
  return rows;
}
template <int N>
using ZPencil = Pencil<N / 2, z_rows<N / 2>(), true>;

// Rows per block of the Hessian z pass (two accumulators stay in registers): at most
// 128 threads, a power of two so it divides the row count.
constexpr int floor_pow2(int v) { return v < 2 ? 1 : 2 * floor_pow2(v / 2); }
template <int N>
using ZHPencil = Pencil<N / 2, floor_pow2(min_i(z_rows<N / 2>(), pmax(1, 128 / (N / 2 / pencil_r2(N / 2))))), true>;

// A column width is usable when it divides n/2, the LDS exchange fits in kColLdsMax
// and the block stays within 1024 threads.
constexpr size_t kColLdsMax = 144 * 1024;
template <int N, int B>
constexpr bool col_ok() {
  return B >= 2 && B <= pow2_factor(N / 2) && B * (N / pencil_r2(N)) <= 1024 &&
         Pencil<N, B, false>::LDS * sizeof(float2) <= kColLdsMax;
}
// The widest of 16, 8, 4 columns that is usable: 16 columns are 128-byte runs per row,
// the width at which the strided passes reach full HBM bandwidth.
template <int N>
constexpr int col_width_default() {
  return col_ok<N, 16>() ? 16 : col_ok<N, 8>() ? 8 : 4;
}

// Stored row of logical row y of x-plane x in a rotated half spectrum.
template <int N>
__device__ __forceinline__ int rot_row(int y, int x, int rot) {
  return (int)((unsigned)(y + rot * x) % (unsigned)N);
}

__device__ __forceinline__ int pick_comp(int c, int nx, int ny, int nz) {
  return c == 0 ? nx : (c == 1 ? ny : nz);
}
// Hessian components in output order xx, yy, zz, xy, yz, zx.
__device__ __forceinline__ int hess_a(int p) { return p < 3 ? p : p - 3; }
__device__ __forceinline__ int hess_b(int p) { return p < 3 ? p : (p - 2) % 3; }

__device__ __forceinline__ void load_twiddles(float2* stw, const float2* __restrict__ tw, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) stw[i] = tw[i];
}

// The z passes at n >= 1024 read their twiddles from the global table (8 KB, held in
// the caches) instead of an LDS copy: their blocks are single waves, and a per-block
// copy would be a third of the block's LDS and cap a CU at six of them.
template <int N>
constexpr bool z_twiddles_global() { return N >= 1024; }
template <int N>
constexpr int z_stw_len() { return z_twiddles_global<N>() ? 1 : N; }
template <int N>
__device__ __forceinline__ const float2* z_twiddles(float2* stw, const float2* __restrict__ tw) {
  if constexpr (z_twiddles_global<N>()) {
    return tw;
  } else {
    load_twiddles(stw, tw, N);
    return stw;
  }
}

// ---------------------------------------------------------------------------------
// z forward: real rows -> half complex rows.
// X[k] = (Z[k] + conj Z[M-k]) / 2 - i W^k (Z[k] - conj Z[M-k]) / 2, W = exp(-2 pi i / N),
// where Z is the length-M = N/2 DFT of z[m] = x[2m] + i x[2m+1].  Z[M-k] sits in the
// partner lane of the same wave (Pencil::partner).
// ---------------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(ZPencil<N>::T) void k_zfwd(const float* in, float2* out, const float2* __restrict__ tw) {
  using P = ZPencil<N>;
  constexpr int M = N / 2;
  __shared__ __align__(16) float2 ex[P::LDS];
  __shared__ float2 stw_l[z_stw_len<N>()];
  const long row0 = (long)blockIdx.x * P::NT;
  float2 a[P::R2];
  P::load_a(a, reinterpret_cast<const float2*>(in) + row0 * M, M);
  const float2* stw = z_twiddles<N>(stw_l, tw);
  __syncthreads();
  float2 q[P::UB][P::R1];
  P::template fwd_like<-1, 2>(a, q, ex, stw);
#pragma unroll
  for (int u = 0; u < P::UB; ++u) {
    int b, j2;
    const bool ok = P::b_unit(u, b, j2);
    float2 zm[P::R1];
    P::partner(q, u, zm);
    if (!ok) continue;
#pragma unroll
    for (int j1 = 0; j1 < P::R1; ++j1) {
      const int k = j2 + P::R2 * j1;
      const float2 zk = q[u][j1];
      const float2 s = c_scale(c_add(zk, c_conj(zm[j1])), 0.5f);
      const float2 d = c_scale(c_sub(zk, c_conj(zm[j1])), 0.5f);
      q[u][j1] = c_add(s, mul_si<-1>(c_mul(stw[k], d)));
    }
  }
  P::store_b(q, out + row0 * M, M);
}

// ---------------------------------------------------------------------------------
// z inverse: half complex rows -> real rows (unnormalised, times `scale`).
// Z'[k] = (X[k] + conj X[M-k]) + i W^-k (X[k] - conj X[M-k]) with X[M] = 0;
// its unnormalised inverse length-M DFT is x[2m] + i x[2m+1].
// ---------------------------------------------------------------------------------
// Pre-processing of loaded B-layout registers, then the inverse half-length transform.
template <class P, int N>
__device__ __forceinline__ void zinv_regs(float2 (&q)[P::UB][P::R1], float2 (&a)[P::R2], float2* ex,
                                          const float2* stw) {
#pragma unroll
  for (int u = 0; u < P::UB; ++u) {
    int b, j2;
    const bool ok = P::b_unit(u, b, j2);
    float2 xm[P::R1];
    P::partner(q, u, xm);
    if (!ok) continue;
#pragma unroll
    for (int j1 = 0; j1 < P::R1; ++j1) {
      const int k = j2 + P::R2 * j1;
      const float2 xk = q[u][j1];
      const float2 m = (j1 == 0 && j2 == 0) ? make_float2(0.f, 0.f) : xm[j1];
      q[u][j1] = c_add(c_add(xk, c_conj(m)), mul_si<1>(c_mul(c_conj(stw[k]), c_sub(xk, c_conj(m)))));
    }
  }
  P::template inv_like<1, 2>(q, a, ex, stw);
}

template <int N, int EPI>
__global__ __launch_bounds__(ZPencil<N>::T) void k_zinv(FieldPtrs in, FieldPtrs out, const float2* __restrict__ tw,
                                                         EpiArgs e) {
  using P = ZPencil<N>;
  constexpr int M = N / 2;
  __shared__ __align__(16) float2 ex[P::LDS];
  __shared__ float2 stw_l[z_stw_len<N>()];
  // the fields' blocks alternate (field fastest), so fields written together by the
  // previous pass are read together
  const int nf = e.nfields;
  const int f = (int)(blockIdx.x % nf);
  const long blk = blockIdx.x / nf, nblk = gridDim.x / nf;
  const long row0 = (e.reverse ? nblk - 1 - blk : blk) * P::NT;
  float2 q[P::UB][P::R1];
  P::load_b(q, in.p[f] + row0 * M, M);
  const float2* stw = z_twiddles<N>(stw_l, tw);
  if ((e.deriv >> f) & 1) {
    // z derivative: mode k (0 <= k < n/2) times i k, before the Hermitian pairing
#pragma unroll
    for (int u = 0; u < P::UB; ++u) {
      int b, j2;
      P::b_unit(u, b, j2);
#pragma unroll
      for (int j1 = 0; j1 < P::R1; ++j1) q[u][j1] = mul_si<1>(c_scale(q[u][j1], (float)(j2 + P::R2 * j1)));
    }
  }
  __syncthreads();
  float2 a[P::R2];
  zinv_regs<P, N>(q, a, ex, stw);
#pragma unroll
  for (int i = 0; i < P::R2; ++i) a[i] = c_scale(a[i], e.scale);
  float2* dst = out.p[f] + row0 * M;
  if constexpr (EPI == kEpiStore) {
    P::store_a(a, dst, M);
  } else {
    // s2 = x; s = d1 s1 + d2 s2; v = v1 s1 + v2 s2 (component f)
    const long off = f * e.comp_stride + row0 * N;
    const float2* s1 = reinterpret_cast<const float2*>(e.s1 + off);
    float2 x1[P::R2], sv[P::R2], vv[P::R2];
    P::load_a(x1, s1, M);
#pragma unroll
    for (int i = 0; i < P::R2; ++i) {
      sv[i] = make_float2(e.d1 * x1[i].x + e.d2 * a[i].x, e.d1 * x1[i].y + e.d2 * a[i].y);
      vv[i] = make_float2(e.v1 * x1[i].x + e.v2 * a[i].x, e.v1 * x1[i].y + e.v2 * a[i].y);
    }
    P::store_a(a, dst, M);
    P::store_a(sv, reinterpret_cast<float2*>(e.s + off), M);
    P::store_a(vv, reinterpret_cast<float2*>(e.v + off), M);
  }
}

// Six Hessian fields -> S, accumulated in registers one field at a time.
template <int N>
__global__ __launch_bounds__(ZHPencil<N>::T) void k_zinv_hess(FieldPtrs in, float* out, const float2* __restrict__ tw,
                                                              float scale) {
  using P = ZHPencil<N>;
  constexpr int M = N / 2;
  __shared__ __align__(16) float2 ex[P::LDS];
  __shared__ float2 stw_l[z_stw_len<N>()];
  const float2* stw = z_twiddles<N>(stw_l, tw);
  const long row0 = (long)blockIdx.x * P::NT;
  // S = xx yy + zz (xx + yy) - xy^2 - yz^2 - zx^2, accumulated as the fields arrive:
  // sum holds xx (+ yy), acc the products.
  float2 sum[P::R2], acc[P::R2];
#pragma unroll 1
  for (int f = 0; f < 6; ++f) {
    float2 q[P::UB][P::R1];
    P::load_b(q, in.p[f] + row0 * M, M);
    __syncthreads();   // twiddles visible / previous exchange consumed
    float2 a[P::R2];
    zinv_regs<P, N>(q, a, ex, stw);
#pragma unroll
    for (int i = 0; i < P::R2; ++i) {
      const float2 t = c_scale(a[i], scale);
      if (f == 0) {
        sum[i] = t;
        acc[i] = make_float2(0.f, 0.f);
      } else if (f < 3) {
        acc[i].x += sum[i].x * t.x;
        acc[i].y += sum[i].y * t.y;
        sum[i] = c_add(sum[i], t);
      } else {
        acc[i].x -= t.x * t.x;
        acc[i].y -= t.y * t.y;
      }
    }
  }
  P::store_a(acc, reinterpret_cast<float2*>(out) + row0 * M, M);
}

// ---------------------------------------------------------------------------------
// Strided column pass: tile = n elements along inner_stride x B contiguous columns.
// ---------------------------------------------------------------------------------
// reverse: blocks walk the tiles from the last to the first, so a pass that follows
// one which wrote the same array in ascending order starts on the data written last
// (still in the memory-side cache).
// rot: the k-space side (the output of a forward pass, the input of an inverse one) is
// a rotated half spectrum whose plane index is the outer index o (y passes only).
template <int N, int B, int S>
__global__ __launch_bounds__((Pencil<N, B, false>::T)) void k_col(FieldPtrs in, FieldPtrs out, long outer_stride,
                                                                long inner_stride, int ntiles_c,
                                                                const float2* __restrict__ tw, int reverse,
                                                                int rot) {
  using P = Pencil<N, B, false>;
  __shared__ __align__(16) float2 ex[P::LDS];
  __shared__ float2 stw[N];
  const int f = blockIdx.y;
  const unsigned blk = reverse ? gridDim.x - 1 - blockIdx.x : blockIdx.x;
  const int tc = blk % ntiles_c;
  const long o = blk / ntiles_c;
  const long origin = o * outer_stride + (long)tc * B;
  const int rot_in = S > 0 ? rot : 0, rot_out = S < 0 ? rot : 0;
  float2 a[P::R2];
  P::load_a_rows(a, in.p[f] + origin, [&](int m) { return (long)rot_row<N>(m, (int)o, rot_in) * inner_stride; });
  load_twiddles(stw, tw, N);
  __syncthreads();
  float2 q[P::UB][P::R1];
  P::template fwd_like<S, 1>(a, q, ex, stw);
  P::store_b_rows(q, out.p[f] + origin, [&](int m) { return (long)rot_row<N>(m, (int)o, rot_out) * inner_stride; });
}

// Inverse column pass with two outputs from one tile of columns: out_d gets the
// inverse transform of i n X (n = m for m <= n/2, else m - n, m the position along
// the column) and out_p that of X; neither may alias in.  Each tile is read by two
// blocks, one per output, 8 block indices apart (the same XCD, dispatched together),
// so the second read is served by that XCD's L2.  At n >= 768 a tile (n rows of B
// columns, 96 or 128 KB) takes a CU's whole LDS budget for its exchange, 32 of them
// fill an XCD's L2 and the partner's read would miss; there one block keeps the tile
// in registers and writes both outputs (the LDS already limits the pass to two waves
// per SIMD, which leave room for the second copy).  in may be a rotated half spectrum
// (rot, plane index o); the outputs are not rotated.
template <int N>
constexpr bool col_pair_one_block() { return N >= 768; }

template <int N, int B>
__global__ __launch_bounds__((Pencil<N, B, false>::T)) void k_col_pair(const float2* __restrict__ in,
                                                                     float2* __restrict__ out_p,
                                                                     float2* __restrict__ out_d, long outer_stride,
                                                                     long inner_stride, int ntiles_c, long ntiles,
                                                                     const float2* __restrict__ tw, int reverse,
                                                                     int rot) {
  using P = Pencil<N, B, false>;
  __shared__ __align__(16) float2 ex[P::LDS];
  __shared__ float2 stw[N];
  constexpr bool ONE = col_pair_one_block<N>();
  long tile;
  int deriv;
  if (ONE) {
    tile = blockIdx.x;
    deriv = 1;
  } else if (ntiles % kXcdsFft == 0) {
    const long g = blockIdx.x / (2 * kXcdsFft), w = blockIdx.x % (2 * kXcdsFft);
    tile = g * kXcdsFft + w % kXcdsFft;
    deriv = w < kXcdsFft;
  } else {
    tile = blockIdx.x / 2;
    deriv = (blockIdx.x % 2) == 0;
  }
  if (reverse) tile = ntiles - 1 - tile;
  const int tc = (int)(tile % ntiles_c);
  const long o = tile / ntiles_c;
  const long origin = o * outer_stride + (long)tc * B;
  float2 a[P::R2];
  P::load_a_rows(a, in + origin, [&](int m) { return (long)rot_row<N>(m, (int)o, rot) * inner_stride; });
  load_twiddles(stw, tw, N);
  // i n X of A-layout register i2 (position m = i1 + R1 i2)
  auto times_in = [&](int i2, float2 v) {
    int b, i1;
    P::a_unit(b, i1);
    const int m = i1 + P::R1 * i2;
    return mul_si<1>(c_scale(v, (float)(m <= N / 2 ? m : m - N)));
  };
  float2 q[P::UB][P::R1];
  if constexpr (ONE) {
    float2 d[P::R2];
#pragma unroll
    for (int i2 = 0; i2 < P::R2; ++i2) d[i2] = times_in(i2, a[i2]);
    __syncthreads();
    P::template fwd_like<1, 1>(d, q, ex, stw);
    P::store_b(q, out_d + origin, inner_stride);
    __syncthreads();   // the exchange has been read
    P::template fwd_like<1, 1>(a, q, ex, stw);
    P::store_b(q, out_p + origin, inner_stride);
  } else {
    if (deriv) {
#pragma unroll
      for (int i2 = 0; i2 < P::R2; ++i2) a[i2] = times_in(i2, a[i2]);
    }
    __syncthreads();
    P::template fwd_like<1, 1>(a, q, ex, stw);
    P::store_b(q, (deriv ? out_d : out_p) + origin, inner_stride);
  }
}

// ---------------------------------------------------------------------------------
// x pass with multiplier.  Tile = n elements along x (stride n * n/2) x B kz columns
// at fixed y.  Mode numbers: nx from the row m, ny from y, nz = kz (< n/2).
// Modes with nx or ny equal to n/2, and the k = 0 mode, get multiplier 0.
// The forward spectrum is held in registers, pre-scaled by the part of the multiplier
// shared by all outputs (c / n^2, or tab[n^2]); each output then applies its own
// factor and is inverse transformed.  Input and outputs are rotated half spectra
// (rot); row x of the tile is row rot_row(y, x) of plane x.  At n >= 1024, where a
// field is many times the memory-side cache, consecutive blocks take consecutive y
// of one kz tile, so the rows that one wave of blocks reads in a plane lie together.
// ---------------------------------------------------------------------------------
// Offset of this thread's first element (plane i1, A layout) in a rotated half spectrum
// at row y, column kz0; the thread's planes i1 + R1 i2 follow at stride n^2/2.
template <class P, int N>
__device__ __forceinline__ long xmul_origin(int y, int kz0, int rot) {
  static_assert(P::R1 * P::R2 == N, "x pass tiles are one transform of length n");
  int b, i1;
  P::a_unit(b, i1);
  return (long)rot_row<N>(y, i1, rot) * (N / 2) + kz0;
}

template <int N>
__device__ __forceinline__ void xmul_tile(int nt, int& tc, int& y) {
  if constexpr (N >= 1024) {
    tc = blockIdx.x / N;
    y = blockIdx.x % N;
  } else {
    tc = blockIdx.x % nt;
    y = blockIdx.x / nt;
  }
}

template <int N, int B, int MODE>
__global__ __launch_bounds__((Pencil<N, B, false>::T)) void k_xmul(const float2* in, FieldPtrs out, int nout,
                                                                 MulArgs ma, const float2* __restrict__ tw, int rot) {
  using P = Pencil<N, B, false>;
  constexpr int H = N / 2;
  constexpr int NT = H / B;
  __shared__ __align__(16) float2 ex[P::LDS];
  __shared__ float2 stw[N];
  int tc, y;
  xmul_tile<N>(NT, tc, y);
  const long inner = (long)N * H;
  const long origin = xmul_origin<P, N>(y, tc * B, rot);
  float2 a[P::R2];
  P::load_a(a, in + origin, inner);
  load_twiddles(stw, tw, N);
  __syncthreads();
  float2 xs[P::UB][P::R1];
  P::template fwd_like<-1, 1>(a, xs, ex, stw);
  const int ny = (y <= H) ? y : y - N;
  const bool ny_ok = (y != H);
#pragma unroll
  for (int u = 0; u < P::UB; ++u) {
    int b, j2;
    P::b_unit(u, b, j2);
    const int nz = tc * B + b;
#pragma unroll
    for (int j1 = 0; j1 < P::R1; ++j1) {
      const int m = j2 + P::R2 * j1;
      const int nx = (m <= H) ? m : m - N;
      const int nsq = nx * nx + ny * ny + nz * nz;
      const bool keep = ny_ok && (m != H) && nsq != 0;
      float w;
      if constexpr (MODE != kMulLpt1) w = ma.c / (float)max(nsq, 1);
      else w = ma.tab[nsq];
      xs[u][j1] = keep ? c_scale(xs[u][j1], w) : make_float2(0.f, 0.f);
    }
  }
  // One output: c = factor(o) * X', inverse x transform, store.
  auto emit = [&](int o, auto factor) {
    float2 c[P::UB][P::R1];
#pragma unroll
    for (int u = 0; u < P::UB; ++u) {
      int b, j2;
      P::b_unit(u, b, j2);
#pragma unroll
      for (int j1 = 0; j1 < P::R1; ++j1) c[u][j1] = factor(xs[u][j1], b, j2 + P::R2 * j1);
    }
    __syncthreads();   // the previous exchange has been read
    float2 r[P::R2];
    P::template inv_like<1, 1>(c, r, ex, stw);
    P::store_a(r, out.p[o] + origin, inner);
  };
  auto nx_of = [](int m) { return (m <= H) ? m : m - N; };
  if constexpr (MODE == kMulGrad) {
    // i n_j X' for j = x, y, z; n_y is uniform over the tile and n_z over a column.
    emit(0, [&](float2 v, int, int m) { return mul_si<1>(c_scale(v, (float)nx_of(m))); });
    emit(1, [&](float2 v, int, int) { return mul_si<1>(c_scale(v, (float)ny)); });
    emit(2, [&](float2 v, int b, int) { return mul_si<1>(c_scale(v, (float)(tc * B + b))); });
  } else if constexpr (MODE == kMulGradPair) {
    // i n_x X' and X' itself: the y and z components are i n_y X' and i n_z X', whose
    // factors are constant along x, so they are applied in the y and z passes instead
    emit(0, [&](float2 v, int, int m) { return mul_si<1>(c_scale(v, (float)nx_of(m))); });
    emit(1, [&](float2 v, int, int) { return v; });
  } else {
    for (int o = 0; o < nout; ++o) {
      emit(o, [&](float2 v, int b, int m) {
        const int nx = nx_of(m), nz = tc * B + b;
        if (o < 3) return mul_si<1>(c_scale(v, (float)pick_comp(o, nx, ny, nz)));     // s1_j: i n_j X'
        const int na = pick_comp(hess_a(o - 3), nx, ny, nz);
        const int nb = pick_comp(hess_b(o - 3), nx, ny, nz);
        return c_scale(v, ma.kf * (float)(na * nb));                                   // phi_ab: kf n_a n_b X'
      });
    }
  }
}

// ---------------------------------------------------------------------------------
// Transposed x pass (adjoint of k_xmul): every input is forward transformed along x,
// multiplied by the complex conjugate of its multiplier and accumulated; the sum is
// inverse transformed into the single output.
// ---------------------------------------------------------------------------------
template <int N, int B, int MODE>
__global__ __launch_bounds__((Pencil<N, B, false>::T)) void k_xmul_adj(FieldPtrs in, int nin, float2* out, MulArgs ma,
                                                                     const float2* __restrict__ tw, int rot) {
  using P = Pencil<N, B, false>;
  constexpr int H = N / 2;
  constexpr int NT = H / B;
  __shared__ __align__(16) float2 ex[P::LDS];
  __shared__ float2 stw[N];
  load_twiddles(stw, tw, N);
  int tc, y;
  xmul_tile<N>(NT, tc, y);
  const long inner = (long)N * H;
  const long origin = xmul_origin<P, N>(y, tc * B, rot);
  const int ny = (y <= H) ? y : y - N;
  const bool ny_ok = (y != H);
  float2 acc[P::UB][P::R1];
#pragma unroll
  for (int u = 0; u < P::UB; ++u)
#pragma unroll
    for (int j1 = 0; j1 < P::R1; ++j1) acc[u][j1] = make_float2(0.f, 0.f);
  // Adds conj(multiplier_f) * FFT_x(in_f) to acc; conj_mul(x, b, m, nsq) is the product.
  auto absorb = [&](int f, auto conj_mul) {
    float2 a[P::R2];
    P::load_a(a, in.p[f] + origin, inner);
    __syncthreads();   // twiddles visible / previous exchange consumed
    float2 q[P::UB][P::R1];
    P::template fwd_like<-1, 1>(a, q, ex, stw);
#pragma unroll
    for (int u = 0; u < P::UB; ++u) {
      int b, j2;
      P::b_unit(u, b, j2);
      const int nz = tc * B + b;
#pragma unroll
      for (int j1 = 0; j1 < P::R1; ++j1) {
        const int m = j2 + P::R2 * j1;
        const int nx = (m <= H) ? m : m - N;
        const int nsq = nx * nx + ny * ny + nz * nz;
        const bool keep = ny_ok && (m != H) && nsq != 0;
        if (keep) acc[u][j1] = c_add(acc[u][j1], conj_mul(q[u][j1], nx, nz, nsq));
      }
    }
  };
  if constexpr (MODE == kMulGrad) {
    // conj(i c n_j / n^2) X
    absorb(0, [&](float2 x, int nx, int, int nsq) { return mul_si<-1>(c_scale(x, ma.c * (float)nx / (float)nsq)); });
    absorb(1, [&](float2 x, int, int, int nsq) { return mul_si<-1>(c_scale(x, ma.c * (float)ny / (float)nsq)); });
    absorb(2, [&](float2 x, int, int nz, int nsq) { return mul_si<-1>(c_scale(x, ma.c * (float)nz / (float)nsq)); });
  } else {
    for (int f = 0; f < nin; ++f) {
      absorb(f, [&](float2 x, int nx, int nz, int nsq) {
        const float t = ma.tab[nsq];
        if (f < 3) return mul_si<-1>(c_scale(x, t * (float)pick_comp(f, nx, ny, nz)));   // conj(i n_j t) X
        const int na = pick_comp(hess_a(f - 3), nx, ny, nz);
        const int nb = pick_comp(hess_b(f - 3), nx, ny, nz);
        return c_scale(x, ma.kf * t * (float)(na * nb));                                   // real multiplier
      });
    }
  }
  __syncthreads();
  float2 r[P::R2];
  P::template inv_like<1, 1>(acc, r, ex, stw);
  P::store_a(r, out + origin, inner);
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
  using P = ZPencil<N>;
  if (nrows % P::NT) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_zfwd<N>, dim3(nrows / P::NT), dim3(P::T), 0, st, in, out, tw);
  return hipGetLastError();
}

template <int N>
static hipError_t zinv_t(FieldPtrs in, FieldPtrs out, int nf, long nrows, const float2* tw, int epi,
                         EpiArgs e, hipStream_t st) {
  using P = ZPencil<N>;
  if (nrows % P::NT) return hipErrorInvalidValue;
  if (nf < 1 || nf > kMaxFields) return hipErrorInvalidValue;
  e.nfields = nf;
  dim3 grid((unsigned)(nrows / P::NT * nf));
  if (epi == kEpiStore)
    hipLaunchKernelGGL((k_zinv<N, kEpiStore>), grid, dim3(P::T), 0, st, in, out, tw, e);
  else
    hipLaunchKernelGGL((k_zinv<N, kEpiLptFinal>), grid, dim3(P::T), 0, st, in, out, tw, e);
  return hipGetLastError();
}

template <int N>
static hipError_t zinv_hess_t(FieldPtrs in, float* out, long nrows, const float2* tw, float scale,
                              hipStream_t st) {
  using P = ZHPencil<N>;
  if (nrows % P::NT) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_zinv_hess<N>, dim3(nrows / P::NT), dim3(P::T), 0, st, in, out, tw, scale);
  return hipGetLastError();
}

template <int N, int B>
static hipError_t col_tb(int dir, FieldPtrs in, FieldPtrs out, int nf, int n_outer, long outer_stride,
                         long inner_stride, int ncols, const float2* tw, int reverse, int rot, hipStream_t st) {
  if constexpr (col_ok<N, B>()) {
    if (ncols % B) return hipErrorInvalidValue;
    constexpr int T = Pencil<N, B, false>::T;
    const int ntc = ncols / B;
    dim3 grid((unsigned)((long)n_outer * ntc), nf);
    if (dir < 0)
      hipLaunchKernelGGL((k_col<N, B, -1>), grid, dim3(T), 0, st, in, out, outer_stride, inner_stride, ntc, tw,
                         reverse, rot);
    else
      hipLaunchKernelGGL((k_col<N, B, 1>), grid, dim3(T), 0, st, in, out, outer_stride, inner_stride, ntc, tw,
                         reverse, rot);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int N>
static hipError_t col_t(int dir, FieldPtrs in, FieldPtrs out, int nf, int n_outer, long outer_stride,
                        long inner_stride, int ncols, const float2* tw, int width, int reverse, int rot,
                        hipStream_t st) {
  switch (width ? width : col_width_default<N>()) {
    case 4: return col_tb<N, 4>(dir, in, out, nf, n_outer, outer_stride, inner_stride, ncols, tw, reverse, rot, st);
    case 8: return col_tb<N, 8>(dir, in, out, nf, n_outer, outer_stride, inner_stride, ncols, tw, reverse, rot, st);
    case 16: return col_tb<N, 16>(dir, in, out, nf, n_outer, outer_stride, inner_stride, ncols, tw, reverse, rot, st);
    default: return hipErrorInvalidValue;
  }
}

template <int N, int B>
static hipError_t col_pair_tb(const float2* in, float2* out_p, float2* out_d, int n_outer, long outer_stride,
                              long inner_stride, int ncols, const float2* tw, int reverse, int rot, hipStream_t st) {
  if constexpr (col_ok<N, B>()) {
    if (ncols % B) return hipErrorInvalidValue;
    constexpr int T = Pencil<N, B, false>::T;
    const int ntc = ncols / B;
    const long ntiles = (long)n_outer * ntc;
    const long nblocks = col_pair_one_block<N>() ? ntiles : 2 * ntiles;
    hipLaunchKernelGGL((k_col_pair<N, B>), dim3((unsigned)nblocks), dim3(T), 0, st, in, out_p, out_d,
                       outer_stride, inner_stride, ntc, ntiles, tw, reverse, rot);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int N>
static hipError_t col_pair_t(const float2* in, float2* out_p, float2* out_d, int n_outer, long outer_stride,
                             long inner_stride, int ncols, const float2* tw, int width, int reverse, int rot,
                             hipStream_t st) {
  switch (width ? width : col_width_default<N>()) {
    case 4:
      return col_pair_tb<N, 4>(in, out_p, out_d, n_outer, outer_stride, inner_stride, ncols, tw, reverse, rot, st);
    case 8:
      return col_pair_tb<N, 8>(in, out_p, out_d, n_outer, outer_stride, inner_stride, ncols, tw, reverse, rot, st);
    case 16:
      return col_pair_tb<N, 16>(in, out_p, out_d, n_outer, outer_stride, inner_stride, ncols, tw, reverse, rot, st);
    default: return hipErrorInvalidValue;
  }
}

template <int N, int B>
static hipError_t xmul_tb(int mode, const float2* in, FieldPtrs out, int nout, MulArgs m, const float2* tw,
                          int rot, hipStream_t st) {
  if constexpr (col_ok<N, B>()) {
    constexpr int T = Pencil<N, B, false>::T;
    if (rot % Pencil<N, B, false>::R2) return hipErrorInvalidValue;
    if (mode == kMulGrad ? nout != 3
        : mode == kMulGradPair ? nout != 2
        : (mode != kMulLpt1 || nout < 1 || nout > kMaxFields))
      return hipErrorInvalidValue;
    dim3 grid(N * ((N / 2) / B));
    if (mode == kMulGrad)
      hipLaunchKernelGGL((k_xmul<N, B, kMulGrad>), grid, dim3(T), 0, st, in, out, nout, m, tw, rot);
    else if (mode == kMulGradPair)
      hipLaunchKernelGGL((k_xmul<N, B, kMulGradPair>), grid, dim3(T), 0, st, in, out, nout, m, tw, rot);
    else
      hipLaunchKernelGGL((k_xmul<N, B, kMulLpt1>), grid, dim3(T), 0, st, in, out, nout, m, tw, rot);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

// Default x-pass width: the widest valid tile (128-byte row segments at 16 columns).
template <int N>
constexpr int xmul_width() { return col_width_default<N>(); }

template <int N>
static hipError_t xmul_t(int mode, const float2* in, FieldPtrs out, int nout, MulArgs m, const float2* tw,
                         int width, int rot, hipStream_t st) {
  switch (width ? width : xmul_width<N>()) {
    case 4: return xmul_tb<N, 4>(mode, in, out, nout, m, tw, rot, st);
    case 8: return xmul_tb<N, 8>(mode, in, out, nout, m, tw, rot, st);
    case 16: return xmul_tb<N, 16>(mode, in, out, nout, m, tw, rot, st);
    default: return hipErrorInvalidValue;
  }
}

template <int N>
static hipError_t xmul_adj_t(int mode, FieldPtrs in, int nin, float2* out, MulArgs m, const float2* tw,
                             int rot, hipStream_t st) {
  // the transposed pass holds three inputs: 16 columns of 1024 would spill, and the
  // nine-input LPT form spills with 16 columns of 768
  constexpr int BG = (N >= 1024 && xmul_width<N>() > 8) ? 8 : xmul_width<N>();
  constexpr int BL = (N >= 768 && BG > 8) ? 8 : BG;
  if (rot % pencil_r2(N)) return hipErrorInvalidValue;
  if (mode != kMulGrad && mode != kMulLpt1) return hipErrorInvalidValue;
  if (mode == kMulGrad ? nin != 3 : (nin < 1 || nin > kMaxFields)) return hipErrorInvalidValue;
  if (mode == kMulGrad)
    hipLaunchKernelGGL((k_xmul_adj<N, BG, kMulGrad>), dim3(N * ((N / 2) / BG)), dim3(Pencil<N, BG, false>::T), 0, st,
                       in, nin, out, m, tw, rot);
  else
    hipLaunchKernelGGL((k_xmul_adj<N, BL, kMulLpt1>), dim3(N * ((N / 2) / BL)), dim3(Pencil<N, BL, false>::T), 0, st,
                       in, nin, out, m, tw, rot);
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

int fft_rot_rows(int n) { return fft_size_supported(n) ? pencil_r2(n) : 0; }
// Rotated where the plane stride is 4 MB or more (n >= 1024): there copies with the x
// pass's access pattern move 2.7 TB/s over plain planes and 3.7 TB/s over rotated ones.
bool fft_rot_default_on(int n) { return n >= 1024; }

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
                      long inner_stride, int ncols, const float2* tw, int width, int rot, hipStream_t st,
                      int reverse) {
  if (rot < 0 || rot >= n) return hipErrorInvalidValue;
  switch (n) {
#define COLA_CASE(N) \
  case N:            \
    return col_t<N>(dir, in, out, nf, n_outer, outer_stride, inner_stride, ncols, tw, width, reverse, rot, st);
    COLA_FOR_EACH_SIZE(COLA_CASE)
#undef COLA_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------------
// Shell statistics of two half spectra a, b ([x][y][kz], n/2 kz per row; the kz = n/2
// plane is not stored, so shells s = round(|n|) with 1 <= s < n/2 are complete).
// Per shell: the mode count and the sums of |a|^2, |b|^2 and Re(a conj b), each mode
// with kz > 0 counted twice (it stands for its conjugate partner too).  The shell is
// decided in integers.  Blocks accumulate in LDS (FP64 atomics) over a contiguous
// range of elements and write partial sums; k_shell_reduce adds the partials block
// by block in a fixed order and forms P, rho = P_ab / sqrt(P_aa P_bb) and
// n_max = (2/3) rho / sqrt(1 - rho^2).
// ---------------------------------------------------------------------------------
constexpr int kShellThreads = 256;

__device__ __forceinline__ int shell_of(int n2) {
  int s = (int)sqrtf((float)n2);
  while (s * s > n2) --s;
  while ((s + 1) * (s + 1) <= n2) ++s;
  return n2 > s * s + s ? s + 1 : s;   // round(sqrt(n2)): sqrt(n2) >= s + 1/2 iff n2 > s^2 + s
}

__global__ __launch_bounds__(kShellThreads) void k_shell_sums(int n, const float2* __restrict__ a,
                                                              const float2* __restrict__ b, long chunk,
                                                              double* __restrict__ part) {
  extern __shared__ double acc[];   // [4][h]: count, aa, bb, ab
  const int h = n / 2;
  for (int i = threadIdx.x; i < 4 * h; i += kShellThreads) acc[i] = 0.0;
  __syncthreads();
  const long total = (long)n * n * h;
  const long beg = (long)blockIdx.x * chunk;
  const long end = beg + chunk < total ? beg + chunk : total;
  for (long e = beg + threadIdx.x; e < end; e += kShellThreads) {
    const int kz = (int)(e % h);
    const long r = e / h;
    const int y = (int)(r % n), x = (int)(r / n);
    const int nx = x <= h ? x : x - n, ny = y <= h ? y : y - n;
    const int sh = shell_of(nx * nx + ny * ny + kz * kz);
    if (sh < 1 || sh >= h) continue;
    const double w = kz > 0 ? 2.0 : 1.0;
    const float2 va = a[e];
    atomicAdd(&acc[sh], w);
    atomicAdd(&acc[h + sh], w * ((double)va.x * va.x + (double)va.y * va.y));
    if (b) {
      const float2 vb = b[e];
      atomicAdd(&acc[2 * h + sh], w * ((double)vb.x * vb.x + (double)vb.y * vb.y));
      atomicAdd(&acc[3 * h + sh], w * ((double)va.x * vb.x + (double)va.y * vb.y));
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 4 * h; i += kShellThreads) part[(long)blockIdx.x * 4 * h + i] = acc[i];
}

__global__ __launch_bounds__(kShellThreads) void k_shell_reduce(int h, const double* __restrict__ part, int nblocks,
                                                                double norm, int cross, double* __restrict__ out) {
  const int sh = blockIdx.x * kShellThreads + threadIdx.x;
  if (sh >= h) return;
  double c = 0.0, aa = 0.0, bb = 0.0, ab = 0.0;
  for (int k = 0; k < nblocks; ++k) {
    const double* q = part + (long)k * 4 * h;
    c += q[sh];
    aa += q[h + sh];
    bb += q[2 * h + sh];
    ab += q[3 * h + sh];
  }
  double paa = 0.0, pbb = 0.0, pab = 0.0, rho = 0.0, nmax = 0.0;
  if (c > 0.0) {
    paa = aa / c * norm;
    pbb = bb / c * norm;
    pab = ab / c * norm;
    if (cross && paa > 0.0 && pbb > 0.0) {
      rho = pab / sqrt(paa * pbb);
      nmax = (2.0 / 3.0) * rho / sqrt(fmax(1.0 - rho * rho, 0.0));
    }
  }
  out[sh] = c;
  out[h + sh] = paa;
  out[2 * h + sh] = pbb;
  out[3 * h + sh] = pab;
  out[4 * h + sh] = rho;
  out[5 * h + sh] = nmax;
}

hipError_t launch_shell_stats(int n, const float2* a, const float2* b, double* part, long part_doubles, double norm,
                              double* out, hipStream_t st) {
  if (n < 4 || n % 2 || !a || !part || !out) return hipErrorInvalidValue;
  const int h = n / 2;
  const long total = (long)n * n * h;
  long nb = part_doubles / (4L * h);
  nb = nb < 1024 ? nb : 1024;
  if (nb < 1) return hipErrorInvalidValue;
  const long chunk = (total + nb - 1) / nb;
  nb = (total + chunk - 1) / chunk;
  hipLaunchKernelGGL(k_shell_sums, dim3((unsigned)nb), dim3(kShellThreads), 4 * h * sizeof(double), st, n, a, b, chunk,
                     part);
  hipLaunchKernelGGL(k_shell_reduce, dim3((unsigned)((h + kShellThreads - 1) / kShellThreads)), dim3(kShellThreads), 0,
                     st, h, part, (int)nb, norm, b != nullptr ? 1 : 0, out);
  return hipGetLastError();
}

hipError_t launch_col_pair(int n, const float2* in, float2* out_p, float2* out_d, int n_outer, long outer_stride,
                           long inner_stride, int ncols, const float2* tw, int width, int rot, hipStream_t st,
                           int reverse) {
  if (out_d == in || out_p == in || out_d == out_p) return hipErrorInvalidValue;
  if (rot < 0 || rot >= n) return hipErrorInvalidValue;
  switch (n) {
#define COLA_CASE(N) \
  case N:            \
    return col_pair_t<N>(in, out_p, out_d, n_outer, outer_stride, inner_stride, ncols, tw, width, reverse, rot, st);
    COLA_FOR_EACH_SIZE(COLA_CASE)
#undef COLA_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_xmul_adj(int n, int mode, FieldPtrs in, int nin, float2* out, MulArgs m, const float2* tw,
                           int rot, hipStream_t st) {
  if (rot < 0 || rot >= n) return hipErrorInvalidValue;
  switch (n) {
#define COLA_CASE(N) \
  case N:            \
    return xmul_adj_t<N>(mode, in, nin, out, m, tw, rot, st);
    COLA_FOR_EACH_SIZE(COLA_CASE)
#undef COLA_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_xmul(int n, int mode, const float2* in, FieldPtrs out, int nout, MulArgs m, const float2* tw,
                       int width, int rot, hipStream_t st) {
  if (rot < 0 || rot >= n) return hipErrorInvalidValue;
  switch (n) {
#define COLA_CASE(N) \
  case N:            \
    return xmul_t<N>(mode, in, out, nout, m, tw, width, rot, st);
    COLA_FOR_EACH_SIZE(COLA_CASE)
#undef COLA_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace cola
