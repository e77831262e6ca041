// Per-particle kernels on gfx950: Eulerian binning, cloud-in-cell deposit, the
// fused CIC gather + COLA kick + drift, Philox white noise and a fill kernel.
//
// Particles are in Lagrangian order p = (i np + j) np + k (k fastest) with SoA
// components [3][np^3]; the Lagrangian position q = (i, j, k) L / np is implicit.
// Cell-centred mesh: the mesh coordinate of a particle is
//   u = ratio * (i, j, k) + (s / dx - 1/2),
// evaluated as an exact integer plus a small FP32 remainder so the CIC weights keep
// full FP32 precision on large meshes.
//
// Tile blocks are remapped so that each of the 8 XCDs (which receive blocks
// round-robin) works on one contiguous slab of tiles and shares its L2 with the
// neighbouring tiles whose halo rows it reads.
#include <type_traits>

#include "internal.hpp"


namespace cola {

constexpr int kPartThreads = 256;
constexpr int kXcds = 8;

__device__ __forceinline__ long xcd_block(long nblocks_padded, long b = blockIdx.x) {
  return (b % kXcds) * (nblocks_padded / kXcds) + b / kXcds;
}

__device__ __forceinline__ int wrap(int c, int n) {
  c %= n;
  return c < 0 ? c + n : c;
}

// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(kPartThreads) void k_fill(float4* p, long n4, float value) {
  const long i = (long)blockIdx.x * kPartThreads + threadIdx.x;
  if (i < n4) p[i] = make_float4(value, value, value, value);
}

// ---------------------------------------------------------------------------------
// Eulerian binning.  The mesh is cut into tiles of tx x ty x tz cells; every step
// the particles are binned by the tile of their base cell (the lower corner of
// their CIC stencil) and, within it, by a 3-bit boundary class: bit d is set when
// the base cell lies on the tile's upper face along axis d, i.e. when the stencil
// reaches into the next tile along d.  Key = 8 tile + class.  Deposit and gather
// then run tile by tile through LDS:
//   bin_count   wavefront-aggregated atomics give each particle its rank among the
//               particles with its key (lanes sharing a key take one atomic);
//   bin_scan    exclusive prefix sum of the key counts (tile t owns the particle
//               range [offset[8t], offset[8t + 8]));
//   bin_scatter idx[offset[key] + rank] = slot;
//   deposit     per tile: its own particles plus the boundary classes of its seven
//               lower neighbours that reach into it, accumulated in an LDS tile of
//               exactly the tile's cells, which are then written with plain stores:
//               every cell has one writer and no halo needs merging;
//   gather      per tile: the three force meshes over the tile's cells read once
//               into LDS; every particle of the tile reads its 8 corners there (the
//               corners past the tile's upper faces through L2).
// ---------------------------------------------------------------------------------
constexpr int kTX = 8, kTY = 8;   // tile cells along x and y; tz (8, 16, 32 or 64) is a template parameter
constexpr int kClasses = 8;

template <int TZ>
struct TileDims {
  static constexpr int EY = kTY, EZ = TZ + 1;               // staged core; rows padded by one word
  static constexpr int EXT = kTX * EY * EZ;
  static constexpr int CORE = kTX * kTY * TZ;
  // threads per tile block: a tile holds 2 TZ particles on average at mesh ratio 2
  static constexpr int TT = TZ >= 64 ? 512 : kPartThreads;
};

// Deposit accumulators: a tile sums its CIC contributions in LDS as 64-bit fixed point
// with 32 fraction bits (two's complement, integer atomics).  Integer adds are exact
// and associative, so the sum does not depend on the order of the adds; each
// contribution is its FP32 value rounded to 2^-32, and the tile value is converted to
// FP32 within one ulp (tile_value).  It is also the faster form on gfx950, whose LDS
// integer atomics run far
// ahead of its LDS float atomics.  The range is enough for any mass deposit (a cell
// holds at most the total mass nm^3 <= 2^30); weighted deposits scale their weights
// into range first (k_deposit_tiles).
constexpr float kFixScale = 4294967296.f;   // 2^32
// |x| < 2^31: round(x 2^32) from the exact split x = h + r, h = floor(x), r in [0, 1),
// as h 2^32 + rint(r 2^32); r 2^32 <= 2^32 - 2^8 for a float r < 1.
__device__ __forceinline__ void tile_add(unsigned long long* p, float x) {
  const float h = floorf(x);
  const unsigned lo = (unsigned)rintf((x - h) * kFixScale);
  atomicAdd(p, ((unsigned long long)(long long)(int)h << 32) | lo);
}
// The cell value v 2^-32 of a sum v = hi 2^32 + lo (hi signed, lo unsigned) as
// hi + lo 2^-32 in one fused multiply-add: lo converts exactly below 2^24 and with a
// relative error of 2^-24 above, hi exactly below 2^24, so the result is within one
// ulp of the correctly rounded value (exact when hi = 0), in three instructions where
// a correctly rounded conversion of the 64-bit integer takes about fourteen.
__device__ __forceinline__ float tile_value(unsigned long long v) {
  return fmaf((float)(unsigned)v, 1.f / kFixScale, (float)(int)(v >> 32));
}

// Base cell (wrapped) and CIC fraction along one axis.  t = s nm / L - 1/2 with nm / L
// carried as the float pair inv_dx + inv_dx_lo: a single float nm / L is off by up to
// 2^-24 relative, which would shift every particle by that fraction of its displacement
// in cells -- a bias, not noise, for particles that moved far -- so only t's own final
// rounding remains.
__device__ __forceinline__ int base_cell(int lag, int ratio, float s, float inv_dx, float inv_dx_lo, int nm,
                                         float& frac) {
  const float t = fmaf(s, inv_dx, fmaf(s, inv_dx_lo, -0.5f));
  const float ft = floorf(t);
  frac = t - ft;
  const int c = ratio * lag + (int)ft;
  return ((unsigned)c < (unsigned)nm) ? c : wrap(c, nm);
}

__device__ __forceinline__ unsigned div_np(const Lattice& lat, unsigned x) {
  return (unsigned)(((unsigned long long)x * lat.np_magic) >> (31 + lat.np_shift));
}
__device__ __forceinline__ void lag_index(const Lattice& lat, unsigned p, int li[3]) {
  const unsigned n = (unsigned)lat.np;
  const unsigned q = div_np(lat, p);
  const unsigned r = div_np(lat, q);
  li[2] = (int)(p - q * n);
  li[1] = (int)(q - r * n);
  li[0] = (int)r;
}

struct Stencil {
  int c[3];     // wrapped base cell
  float f[3];   // fraction towards cell + 1
};

__device__ __forceinline__ Stencil stencil_of(const Lattice& lat, unsigned p, const float sv[3]) {
  int li[3];
  lag_index(lat, p, li);
  Stencil st;
#pragma unroll
  for (int d = 0; d < 3; ++d)
    st.c[d] = base_cell(li[d], lat.ratio, sv[d], lat.inv_dx, lat.inv_dx_lo, lat.nm, st.f[d]);
  return st;
}

template <int TZ>
__device__ __forceinline__ int key_of(const Bins& b, const int c[3]) {
  // base cells are wrapped (non-negative): unsigned shifts and masks
  const unsigned x = (unsigned)c[0], y = (unsigned)c[1], z = (unsigned)c[2];
  const int tile = (int)(((x / kTX) * b.nby + y / kTY) * b.nbz + z / TZ);
  const int cls = ((x % kTX) == kTX - 1) | (((y % kTY) == kTY - 1) << 1) | (((z % TZ) == TZ - 1) << 2);
  return tile * kClasses + cls;
}

// Rank of each active lane among the lanes of its wave with the same bin, plus one
// atomic per distinct bin that reserves the ranks.  Called by every lane of the wave.
// The ballot loop only groups the lanes; the group leaders then issue their atomics
// together, so a wave waits for one atomic round trip whatever its number of bins.
__device__ __forceinline__ int wave_rank(bool active, int bin, int* __restrict__ count) {
  const int lane = __lane_id();
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  unsigned long long pending = __ballot(active);
  int leader = lane, below = 0, members = 0;
  while (pending) {
    const int first = __ffsll((long long)pending) - 1;
    const int lb = __shfl(bin, first);
    const unsigned long long m = __ballot(active && bin == lb);
    if (active && bin == lb) {
      leader = first;
      below = __popcll(m & lt);
      members = __popcll(m);
    }
    pending &= ~m;
  }
  int base = 0;
  if (active && lane == leader) base = atomicAdd(count + bin, members);
  base = __shfl(base, leader);
  return base + below;
}

template <int TZ>
__global__ __launch_bounds__(kPartThreads) void k_bin_count(Lattice lat, Bins bins, const float* __restrict__ s,
                                                            int2* __restrict__ key_rank, int* __restrict__ count) {
  const unsigned p = blockIdx.x * kPartThreads + threadIdx.x;
  const bool ok = p < (unsigned)lat.npart;
  int bin = 0;
  if (ok) {
    const float sv[3] = {s[p], s[lat.npart + p], s[2 * lat.npart + p]};
    const Stencil st = stencil_of(lat, p, sv);
    bin = key_of<TZ>(bins, st.c);
  }
  const int rank = wave_rank(ok, bin, count);
  if (ok) key_rank[p] = make_int2(bin, rank);
}

// Exclusive scan of count[0..n) into offset[0..n] (offset[n] = total) in three
// launches: chunk sums, a one-block scan of the chunk sums, and the chunk scans.
// The first launch also clears count_next (the counts the next gather fills).
constexpr int kScanThreads = 1024;
constexpr int kScanChunk = 4 * kScanThreads;

__device__ __forceinline__ int block_sum_1024(int v, int* wsum) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (lane == 0) wsum[wave] = v;
  __syncthreads();
  int t = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) t += wsum[w];
  return t;
}

// Exclusive scan across the block of one value per thread; returns the prefix and
// the block total.
__device__ __forceinline__ int block_scan_1024(int v, int* wsum, int& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(inc, o);
    if (lane >= o) inc += t;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  int carry = 0;
  total = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) {
    carry += (w < wave) ? wsum[w] : 0;
    total += wsum[w];
  }
  return carry + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sums(const int* __restrict__ count, int n,
                                                            int* __restrict__ part, int* __restrict__ count_next,
                                                            int n_pad) {
  __shared__ int wsum[kScanThreads / 64];
  const long base = (long)blockIdx.x * kScanChunk;
  int v = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const long i = base + threadIdx.x + k * kScanThreads;
    if (i < n) v += count[i];
  }
  const int t = block_sum_1024(v, wsum);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
  if (count_next)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const long i = base + threadIdx.x + k * kScanThreads;
      if (i < n_pad) count_next[i] = 0;
    }
}

// One block: exclusive scan of the nb chunk sums in place; total to *tot.
__global__ __launch_bounds__(kScanThreads) void k_scan_top(int* __restrict__ part, int nb, int* __restrict__ tot,
                                                           int* __restrict__ heavy) {
  __shared__ int wsum[kScanThreads / 64];
  if (threadIdx.x == 0) heavy[0] = 0;   // k_heavy_tiles appends after the offsets are final
  int carry = 0;
  for (int c = 0; c < nb; c += kScanThreads) {
    const int i = c + threadIdx.x;
    const int v = i < nb ? part[i] : 0;
    int total;
    const int ex = block_scan_1024(v, wsum, total);
    if (i < nb) part[i] = carry + ex;
    carry += total;
    __syncthreads();   // wsum is reused by the next round
  }
  if (threadIdx.x == 0) *tot = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_chunks(const int* __restrict__ count, int n,
                                                              const int* __restrict__ part,
                                                              int* __restrict__ offset) {
  __shared__ int wsum[kScanThreads / 64];
  const long base = (long)blockIdx.x * kScanChunk + 4 * threadIdx.x;
  int v[4], s4 = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = (base + k < n) ? count[base + k] : 0;
    s4 += v[k];
  }
  int total;
  int run = part[blockIdx.x] + block_scan_1024(s4, wsum, total);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k < n) offset[base + k] = run;
    run += v[k];
  }
}

// Crowded tiles: every tile holding more than heavy_min particles (own classes) is
// appended to heavy[1..] (count in heavy[0]).  With heavy_min = ceil(npart / cap)
// fewer than cap tiles can qualify, so the list never overflows.  The order within the
// list does not matter: each tile's result is independent of when it runs.
__global__ __launch_bounds__(kPartThreads) void k_heavy_tiles(long nbins, const int* __restrict__ offset, int heavy_min,
                                                              int* __restrict__ heavy) {
  const long t = (long)blockIdx.x * kPartThreads + threadIdx.x;
  if (t >= nbins) return;
  if (offset[(t + 1) * kClasses] - offset[t * kClasses] > heavy_min) heavy[1 + atomicAdd(heavy, 1)] = (int)t;
}

__global__ __launch_bounds__(kPartThreads) void k_bin_scatter(long npart, const int2* __restrict__ key_rank,
                                                              const int* __restrict__ offset, int* __restrict__ idx) {
  const long p = (long)blockIdx.x * kPartThreads + threadIdx.x;
  if (p >= npart) return;
  const int2 kr = key_rank[p];
  idx[offset[kr.x] + kr.y] = (int)p;
}

// The scatter of the public step: besides its list entry (the identity: slot j holds the
// particle listed at j), each particle's record is written packed to its tile-sorted slot
// j = offset[key] + rank from the caller's Lagrangian-order arrays, which are read in
// order; a wave's particles share few keys, so its writes land in runs of slots.
__global__ __launch_bounds__(kPartThreads) void k_bin_scatter_pack(long npart, const int2* __restrict__ key_rank,
                                                                   const int* __restrict__ offset,
                                                                   int* __restrict__ idx, SortedState src,
                                                                   SortedState dst) {
  const long p = (long)blockIdx.x * kPartThreads + threadIdx.x;
  if (p >= npart) return;
  const int2 kr = key_rank[p];
  const long j = offset[kr.x] + kr.y;
  float a[12];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    a[d] = src.s[d * npart + p];
    a[3 + d] = src.v[d * npart + p];
    a[6 + d] = src.s1[d * npart + p];
    a[9 + d] = src.s2[d * npart + p];
  }
  float4* q = reinterpret_cast<float4*>(dst.s);
  q[j] = make_float4(a[0], a[1], a[2], a[3]);
  q[npart + j] = make_float4(a[4], a[5], a[6], a[7]);
  q[2 * npart + j] = make_float4(a[8], a[9], a[10], a[11]);
  dst.lag[j] = (int)p;
  idx[j] = (int)j;
}

struct TileGeom {
  int bin;
  int lo[3];
};

// Tile of this block.  The first b.heavy_cap blocks take the crowded tiles listed
// by k_heavy_tiles (blocks past the list's length exit), so the tiles whose blocks
// loop over many particle batches start first instead of trailing the grid.  The
// other blocks (virtual index v = block - heavy_cap, with v % 8 the block's XCD) map
// v to a tile: each XCD takes the slab of tile planes bx in [k nbx/8, (k+1) nbx/8)
// and walks it with bz fastest, then bx, then by, so a tile's z, x and y neighbours
// (whose cells overlap its +1 halo) run within a few dozen blocks of it on the same
// XCD and share its L2.  Meshes with nbx not a multiple of 8 fall back to the plain
// slab order.  `listed` tells the caller whether the tile came from the list; a
// block that was not listed must skip a crowded tile (tile_is_listed), which a
// listed block handles.
template <int TZ>
__device__ __forceinline__ bool tile_geom(const Bins& b, const int* heavy, TileGeom& g, bool& listed) {
  int bx, by, bz;
  const long blk = blockIdx.x;
  listed = blk < b.heavy_cap;
  if (listed) {
    if (blk >= heavy[0]) return false;
    g.bin = heavy[1 + blk];
    bz = g.bin % b.nbz;
    const int r = g.bin / b.nbz;
    bx = r / b.nby;
    by = r % b.nby;
  } else {
    const long v = blk - b.heavy_cap;
    const long nb = (b.nbins + kXcds - 1) / kXcds * kXcds;
    if (b.nbx % kXcds == 0) {
      const long local = v / kXcds;
      const int sx = b.nbx / kXcds;
      if (local >= b.nbins / kXcds) return false;
      bz = (int)(local % b.nbz);
      const long r = local / b.nbz;
      bx = (int)(v % kXcds) * sx + (int)(r % sx);
      by = (int)(r / sx);
      g.bin = (int)(((long)bx * b.nby + by) * b.nbz + bz);
    } else {
      g.bin = (int)xcd_block(nb, v);
      if (g.bin >= b.nbins) return false;
      bz = g.bin % b.nbz;
      const int r = g.bin / b.nbz;
      bx = r / b.nby;
      by = r % b.nby;
    }
  }
  g.lo[0] = bx * kTX;
  g.lo[1] = by * kTY;
  g.lo[2] = bz * TZ;
  return true;
}

// Whether a tile with `own` particles (its own classes) is on the crowded list: the
// same test as k_heavy_tiles.
__device__ __forceinline__ bool tile_is_listed(const Lattice& lat, const Bins& b, int own) {
  return own > heavy_min_of(lat.npart, b.heavy_cap);
}

// Tile-local stencil of the particle in slot `slot` of s with Lagrangian index `lagi`;
// false if its base cell is not in this tile (never the case: binning used the same
// arithmetic).
template <int TZ>
__device__ __forceinline__ bool local_stencil(const Lattice& lat, const TileGeom& g, const float* s, unsigned slot,
                                              unsigned lagi, float sv[3], int lc[3], float fr[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) sv[d] = s[d * lat.npart + slot];
  const Stencil st = stencil_of(lat, lagi, sv);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lc[d] = st.c[d] - g.lo[d];
    fr[d] = st.f[d];
  }
  return (unsigned)lc[0] < (unsigned)kTX && (unsigned)lc[1] < (unsigned)kTY && (unsigned)lc[2] < (unsigned)TZ;
}

// Copies NF mesh fields over the tile's own cells (x < 8, y < 8, z < TZ) into LDS,
// field c at tile + c * EXT, row stride EZ.  Each staged row is one aligned run of TZ
// floats (whole cache lines).  The +1 planes along x, y and z that the CIC stencils
// of the tile's upper-face particles reach are not staged: those corners are read from
// the mesh (corner_value), where the neighbouring tiles, staged around the same time
// on the same XCD, keep them in L2.  Staging only the core keeps the three-field tile
// at 50 KB (three blocks per CU at depth 64) and reads each mesh cell from HBM once.
// Every load of a lane is issued before its first LDS write, so a block has all of
// its tile reads in flight at once.
template <int TZ, int NF>
__device__ __forceinline__ void stage_fields(const TileGeom& t, int nm, const float* const* f, float* tile) {
  using D = TileDims<TZ>;
  constexpr int RQ = TZ / 4;                   // float4 per staged row
  constexpr int NQ = kTX * D::EY * RQ;         // staged float4
  constexpr int IT = (NQ + D::TT - 1) / D::TT;
  float4 v[NF][IT];
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int i = threadIdx.x + k * D::TT;
    const int ii = i < NQ ? i : NQ - 1;
    const int zq = ii % RQ, r = ii / RQ;
    const int y = r % D::EY, x = r / D::EY;
    int gx = t.lo[0] + x, gy = t.lo[1] + y;
    gx -= (gx >= nm) ? nm : 0;
    gy -= (gy >= nm) ? nm : 0;
    const long gi = ((long)gx * nm + gy) * nm + t.lo[2] + 4 * zq;   // 16-byte aligned: nm, lo[2] are multiples of 8
#pragma unroll
    for (int c = 0; c < NF; ++c) v[c][k] = *reinterpret_cast<const float4*>(f[c] + gi);
  }
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int i = threadIdx.x + k * D::TT;
    if (i < NQ) {
      const int zq = i % RQ, r = i / RQ;
      float* row = tile + r * D::EZ + 4 * zq;
#pragma unroll
      for (int c = 0; c < NF; ++c) {
        row[c * D::EXT] = v[c][k].x;
        row[c * D::EXT + 1] = v[c][k].y;
        row[c * D::EXT + 2] = v[c][k].z;
        row[c * D::EXT + 3] = v[c][k].w;
      }
    }
  }
}

// Field value at tile-local cell (x, y, z), x, y <= 8, z <= TZ: LDS offset o inside the
// staged core, else the mesh (wrapped).
template <int TZ>
__device__ __forceinline__ float corner_value(const float* tile_field, const float* mesh, int o, const TileGeom& t,
                                              int x, int y, int z, int nm) {
  if (x < kTX && y < kTY && z < TZ) return tile_field[o];
  int gx = t.lo[0] + x, gy = t.lo[1] + y, gz = t.lo[2] + z;
  gx -= (gx >= nm) ? nm : 0;
  gy -= (gy >= nm) ? nm : 0;
  gz -= (gz >= nm) ? nm : 0;
  return mesh[((long)gx * nm + gy) * nm + gz];
}

// Deposit of one tile.  The particle ranges that reach into tile t are its own (all
// classes) and, for each lower neighbour n = t - (dx, dy, dz) with (dx, dy, dz) in
// {0,1}^3 \ 0, the classes containing every bit of the mask m = dx | 2 dy | 4 dz.
// Those 1 + 19 ranges are flattened so the block's lanes take consecutive particles
// across all of them.  A particle's position relative to tile t along axis d is its
// local coordinate in its own tile, minus the tile extent when it comes from the
// lower neighbour along d; its stencil corners inside tile t are added to the LDS
// tile (accumulator ACC as above) and the tile's cells are then stored.
//   ACC = unsigned long long: fixed-point sums (the only accumulator: mass deposits,
//   and weighted ones scaled by the power of two that wmax gives).
// idx holds slots of s; with lag (optional) s is a packed state (positions in the
// first float4 of each slot) and lag maps a slot to its Lagrangian index; without,
// s is SoA [3][np^3] in Lagrangian order.  weight is indexed by Lagrangian index.
constexpr int kDepRanges = 20;

// NW weight planes (weighted deposits): NW = 1 deposits mass * weight[lag]; NW = 3
// deposits the three planes weight[c n + lag] into rho + c nm^3 in one particle walk.
template <int TZ, class ACC, int NW = 1>
__global__ __launch_bounds__(TileDims<TZ>::TT) void k_deposit_tiles(Lattice lat, Bins bins, const float* __restrict__ s,
                                                                const int* __restrict__ lag,
                                                                const int* __restrict__ idx,
                                                                const int* __restrict__ offset,
                                                                const int* __restrict__ heavy, float* __restrict__ rho,
                                                                float mass, const float* __restrict__ weight,
                                                                const unsigned* __restrict__ wmax) {
  using D = TileDims<TZ>;
  static_assert(NW == 1 || NW == 3, "one or three weight planes");
  __shared__ ACC tile[NW * D::CORE];
  // Weighted fixed-point deposits (wmax = bits of max |weight|): the weights are scaled
  // by a power of two 2^k chosen so that no cell's sum, at most npart mass max|weight|
  // in magnitude, can leave the 31 integer bits of the accumulator, and the cells are
  // scaled back by 2^-k (both exact).  Mass deposits keep k = 0.
  // A non-finite weight (max |weight| inf or NaN) has no such scale: every cell of the
  // output is then NaN, as an FP32 sum would have carried it.
  float wscale = 1.f, winv = 1.f;
  if (wmax) {
    const float wm = __uint_as_float(*wmax);
    if (wm <= __FLT_MAX__) {
      int e = 0;
      (void)frexp((double)mass * (double)wm * (double)lat.npart, &e);
      const int k = min(max(30 - e, -120), 120);
      wscale = ldexpf(1.f, k);
      winv = ldexpf(1.f, -k);
    } else {
      winv = __int_as_float(0x7fc00000);
    }
  }
  __shared__ int rbeg[kDepRanges], rpre[kDepRanges + 1], rmask[kDepRanges];
  TileGeom g;
  bool listed;
  if (!tile_geom<TZ>(bins, heavy, g, listed)) return;
  for (int i = threadIdx.x; i < NW * D::CORE; i += D::TT) tile[i] = 0;
  if (threadIdx.x < 64) {
    // lane r < 20 describes range r: r = 0 own tile, then the (mask, class) pairs
    const int lane = threadIdx.x;
    int beg = 0, len = 0, mask = 0;
    if (lane < kDepRanges) {
      int cls = 0;
      if (lane > 0) {
        // enumerate (mask, class) with (class & mask) == mask, mask != 0
        int k = lane - 1;
        for (int m = 1; m < 8; ++m) {
          const int nc = 8 >> __popc(m);   // classes containing mask m
          if (k < nc) {
            mask = m;
            // k-th class containing m: spread k over the bits not in m
            int c = m, bit = 0;
            for (int q = 0; q < 3; ++q)
              if (!(m & (1 << q))) {
                if (k & (1 << bit)) c |= 1 << q;
                ++bit;
              }
            cls = c;
            break;
          }
          k -= nc;
        }
      }
      const int bx = g.lo[0] / kTX, by = g.lo[1] / kTY, bz = g.lo[2] / TZ;
      const int nx = (mask & 1) ? (bx + bins.nbx - 1) % bins.nbx : bx;
      const int ny = (mask & 2) ? (by + bins.nby - 1) % bins.nby : by;
      const int nz = (mask & 4) ? (bz + bins.nbz - 1) % bins.nbz : bz;
      const long key = (((long)nx * bins.nby + ny) * bins.nbz + nz) * kClasses;
      if (lane == 0) {
        beg = offset[key];
        len = offset[key + kClasses] - beg;
      } else {
        beg = offset[key + cls];
        len = offset[key + cls + 1] - beg;
      }
    }
    int inc = len;
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
      const int t = __shfl_up(inc, o);
      if (lane >= o) inc += t;
    }
    if (lane < kDepRanges) {
      rbeg[lane] = beg;
      rpre[lane + 1] = inc;
      rmask[lane] = mask;
    }
    if (lane == 0) rpre[0] = 0;
  }
  __syncthreads();
  if (!listed && tile_is_listed(lat, bins, rpre[1])) return;   // block-uniform
  const int total = rpre[kDepRanges];
  // particles per lane per batch: a tile's particles plus its neighbours' boundary
  // classes (about 1.3 per tile thread on average) fit one or two batches, and more
  // slots per lane only add predicated-off work.  A crowded tile (listed) walks tens of
  // thousands of particles in one block; four per lane keep four record loads in
  // flight per batch on that block's long serial loop.
  auto walk = [&](auto slots) {
  constexpr int U = decltype(slots)::value;
  for (int base = 0; base < total; base += U * D::TT) {   // block-uniform trip count
    float sv[U][3];
    unsigned lg[U];
    int msk[U];
    bool in[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * D::TT + (int)threadIdx.x;
      in[u] = i < total;
      const int ii = in[u] ? i : 0;
      int r = 0;
      if (ii >= rpre[1]) {   // past the tile's own particles: find the neighbour range
#pragma unroll
        for (int q = 1; q < kDepRanges; ++q) r += (rpre[q] <= ii) ? 1 : 0;
      }
      msk[u] = rmask[r];
      const unsigned slot = in[u] ? (unsigned)idx[rbeg[r] + ii - rpre[r]] : 0u;
      if (lag) {   // packed state: positions in the first float4 of the slot
        lg[u] = (unsigned)lag[slot];
        const float4 a = reinterpret_cast<const float4*>(s)[slot];
        sv[u][0] = a.x;
        sv[u][1] = a.y;
        sv[u][2] = a.z;
      } else {
        lg[u] = slot;
#pragma unroll
        for (int d = 0; d < 3; ++d) sv[u][d] = s[d * lat.npart + slot];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!in[u]) continue;
      const Stencil st = stencil_of(lat, lg[u], sv[u]);
      // base cells are wrapped (non-negative), so the tile-local parts are masks
      const int rx = (int)((unsigned)st.c[0] % kTX) - ((msk[u] & 1) ? kTX : 0);
      const int ry = (int)((unsigned)st.c[1] % kTY) - ((msk[u] & 2) ? kTY : 0);
      const int rz = (int)((unsigned)st.c[2] % TZ) - ((msk[u] & 4) ? TZ : 0);
      float mw[NW];
#pragma unroll
      for (int c = 0; c < NW; ++c) mw[c] = weight ? mass * weight[c * lat.npart + lg[u]] * wscale : mass;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int x = rx + a;
        if ((unsigned)x >= (unsigned)kTX) continue;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int y = ry + b;
          if ((unsigned)y >= (unsigned)kTY) continue;
#pragma unroll
          for (int c = 0; c < NW; ++c) {
            const float wab = mw[c] * (a ? st.f[0] : 1.f - st.f[0]) * (b ? st.f[1] : 1.f - st.f[1]);
            ACC* row = tile + c * D::CORE + (x * kTY + y) * TZ;
            if ((unsigned)rz < (unsigned)TZ) tile_add(row + rz, wab * (1.f - st.f[2]));
            if ((unsigned)(rz + 1) < (unsigned)TZ) tile_add(row + rz + 1, wab * st.f[2]);
          }
        }
      }
    }
  }
  };
  if (listed)   // block-uniform
    walk(std::integral_constant<int, 4>{});
  else
    walk(std::integral_constant<int, 1>{});
  __syncthreads();
  // every cell written once, four consecutive z cells per 16-byte store (lo[2] and
  // nm are multiples of 8, so each run of four is aligned)
  // A thread's runs are 4 TT cells apart, a whole number of x planes of the tile, so its
  // output address advances by a fixed stride.
  static_assert(TZ % 4 == 0, "16-byte row pieces");
  static_assert((4 * D::TT) % (TZ * kTY) == 0, "runs a whole number of x planes apart");
  const long nm = lat.nm;
  const int i0 = 4 * threadIdx.x;
  float* out = rho + ((g.lo[0] + i0 / (TZ * kTY)) * nm + g.lo[1] + (i0 / TZ) % kTY) * nm + g.lo[2] + i0 % TZ;
  const long stride = (long)(4 * D::TT / (TZ * kTY)) * nm * nm;
  for (int i = i0; i < D::CORE; i += 4 * D::TT, out += stride) {
#pragma unroll
    for (int c = 0; c < NW; ++c) {
      const ACC* v = tile + c * D::CORE + i;
      float4 f = make_float4(tile_value(v[0]), tile_value(v[1]), tile_value(v[2]), tile_value(v[3]));
      if (wmax) {   // weighted: undo the power-of-two scale (NaN if no scale existed)
        f.x *= winv;
        f.y *= winv;
        f.z *= winv;
        f.w *= winv;
      }
      *reinterpret_cast<float4*>(out + c * nm * nm * nm) = f;
    }
  }
}

// ---------------------------------------------------------------------------------
// Force gather, tile by tile: the PM force at every particle of the caller's
// Lagrangian-order displacements (cola_pm_force).  The kick and drift gathers are
// k_gather_sorted's.
// ---------------------------------------------------------------------------------
template <int TZ>
__global__ __launch_bounds__(TileDims<TZ>::TT) void k_gather_tiles(Lattice lat, Bins bins, const int* __restrict__ idx,
                                                               const int* __restrict__ offset,
                                                               const int* __restrict__ heavy, GatherArgs g) {
  using D = TileDims<TZ>;
  __shared__ float tile[3 * D::EXT];
  TileGeom t;
  bool listed;
  if (!tile_geom<TZ>(bins, heavy, t, listed)) return;
  const int beg = offset[(long)t.bin * kClasses], end = offset[(long)(t.bin + 1) * kClasses];
  if (!listed && tile_is_listed(lat, bins, end - beg)) return;
  const float* gf[3] = {g.g0, g.g1, g.g2};
  const TileGeom& T_ = t;
  stage_fields<TZ, 3>(t, lat.nm, gf, tile);
  __syncthreads();
  const long n = lat.npart;
  for (int i = beg + threadIdx.x; i < end; i += D::TT) {
    const unsigned p = (unsigned)idx[i];
    float sv[3], fr[3];
    int lc[3];
    if (!local_stencil<TZ>(lat, t, g.s, p, p, sv, lc, fr)) continue;   // cannot happen
    float f[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const float wab = (a ? fr[0] : 1.f - fr[0]) * (b ? fr[1] : 1.f - fr[1]);
        const float w0 = wab * (1.f - fr[2]), w1 = wab * fr[2];
        const int o = ((lc[0] + a) * D::EY + lc[1] + b) * D::EZ + lc[2];
#pragma unroll
        for (int d = 0; d < 3; ++d)
          f[d] += w0 * corner_value<TZ>(tile + d * D::EXT, gf[d], o, T_, lc[0] + a, lc[1] + b, lc[2], lat.nm) +
                  w1 * corner_value<TZ>(tile + d * D::EXT, gf[d], o + 1, T_, lc[0] + a, lc[1] + b, lc[2] + 1, lat.nm);
      }
#pragma unroll
    for (int d = 0; d < 3; ++d) g.out_a[d * n + p] = f[d];
  }
}

// ---------------------------------------------------------------------------------
// Adjoint gather: the derivative of CIC interpolation with respect to the particle
// position.  For a mesh field F and a particle with base cell c and fractions f,
//   dF_interp/du_x = sum_{b,c} wy_b wz_c (F[c+1,b,c] - F[c,b,c])   (likewise y, z),
// and u = x / dx.  Per particle the kernel adds to lam_s
//   f1 * grad(sum_d mu_d g_d) + f2 * grad(rbar)
// (f1, f2 include 1/dx): the force-field term of the force VJP (when g, mu are
// given) and the density term through rbar = dL/drho.
// ---------------------------------------------------------------------------------
template <int TZ>
__global__ __launch_bounds__(TileDims<TZ>::TT) void k_grad_gather(Lattice lat, Bins bins, const int* __restrict__ idx,
                                                              const int* __restrict__ offset,
                                                              const int* __restrict__ heavy,
                                                              const float* __restrict__ s, AdjGatherArgs ga) {
  using D = TileDims<TZ>;
  __shared__ float tile[4 * D::EXT];
  TileGeom t;
  bool listed;
  if (!tile_geom<TZ>(bins, heavy, t, listed)) return;
  const int beg = offset[(long)t.bin * kClasses], end = offset[(long)(t.bin + 1) * kClasses];
  if (!listed && tile_is_listed(lat, bins, end - beg)) return;
  const bool with_g = ga.g0 != nullptr;
  if (with_g) {
    const float* f[4] = {ga.g0, ga.g1, ga.g2, ga.rbar};
    stage_fields<TZ, 4>(t, lat.nm, f, tile);
  } else {
    const float* f[1] = {ga.rbar};
    stage_fields<TZ, 1>(t, lat.nm, f, tile + 3 * D::EXT);
  }
  __syncthreads();
  const long n = lat.npart;
  for (int i = beg + threadIdx.x; i < end; i += D::TT) {
    const unsigned p = (unsigned)idx[i];
    float sv[3], fr[3];
    int lc[3];
    if (!local_stencil<TZ>(lat, t, s, p, p, sv, lc, fr)) continue;   // cannot happen
    float mu[3] = {0.f, 0.f, 0.f};
    if (with_g) {
#pragma unroll
      for (int d = 0; d < 3; ++d) mu[d] = ga.mu[d * n + p];
    }
    // corner values of H = sum_d mu_d g_d and of rbar
    float h[2][2][2], r[2][2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int o = ((lc[0] + a) * D::EY + lc[1] + b) * D::EZ + lc[2] + c;
          const int x = lc[0] + a, y = lc[1] + b, z = lc[2] + c;
          r[a][b][c] = corner_value<TZ>(tile + 3 * D::EXT, ga.rbar, o, t, x, y, z, lat.nm);
          h[a][b][c] = with_g ? mu[0] * corner_value<TZ>(tile, ga.g0, o, t, x, y, z, lat.nm) +
                                    mu[1] * corner_value<TZ>(tile + D::EXT, ga.g1, o, t, x, y, z, lat.nm) +
                                    mu[2] * corner_value<TZ>(tile + 2 * D::EXT, ga.g2, o, t, x, y, z, lat.nm)
                              : 0.f;
        }
    const float w[3][2] = {{1.f - fr[0], fr[0]}, {1.f - fr[1], fr[1]}, {1.f - fr[2], fr[2]}};
    float gh[3] = {0.f, 0.f, 0.f}, gr[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        gh[0] += w[1][a] * w[2][b] * (h[1][a][b] - h[0][a][b]);
        gr[0] += w[1][a] * w[2][b] * (r[1][a][b] - r[0][a][b]);
        gh[1] += w[0][a] * w[2][b] * (h[a][1][b] - h[a][0][b]);
        gr[1] += w[0][a] * w[2][b] * (r[a][1][b] - r[a][0][b]);
        gh[2] += w[0][a] * w[1][b] * (h[a][b][1] - h[a][b][0]);
        gr[2] += w[0][a] * w[1][b] * (r[a][b][1] - r[a][b][0]);
      }
#pragma unroll
    for (int d = 0; d < 3; ++d) ga.lam_s[d * n + p] += ga.f1 * gh[d] + ga.f2 * gr[d];
  }
}

// ---------------------------------------------------------------------------------
// Tile-sorted particle state (used by whole runs).  The state lives in workspace
// buffers ordered by the tiles of the previous step, with each particle's Lagrangian
// index stored beside it.  A step reads it through this step's tile lists (idx: runs
// of mostly consecutive slots, since particles move a few cells per step):
//   deposit       per tile: positions and Lagrangian indices only (k_deposit_tiles);
//   gather_sorted per tile: gather + kick + drift, the whole updated record written
//                 to slot j of the other buffer (ordered by this step's tiles, so
//                 coalesced), and the drifted particle counted into next step's tile.
// ---------------------------------------------------------------------------------
// One particle's state at slot j.  A state without a lag array (the caller's
// arrays, in Lagrangian order) has lag = j.
struct SortedRecord {
  unsigned lag;
  float s[3], v[3], s1[3], s2[3];
};

// A packed state (lag != nullptr) holds slot j as three float4 in s viewed as
// float4[3][n]: (s.x s.y s.z v.x), (v.y v.z s1.x s1.y), (s1.z s2.x s2.y s2.z), so an
// indirect read of one particle touches 4 cache lines rather than 13.  The caller's
// arrays (lag == nullptr) are SoA [3][n] in Lagrangian order.
__device__ __forceinline__ void load_record(const SortedState& st, long n, int j, SortedRecord& r) {
  if (st.lag) {
    const float4* q = reinterpret_cast<const float4*>(st.s);
    const float4 a = q[j], b = q[n + j], c = q[2 * n + j];
    r.lag = (unsigned)st.lag[j];
    r.s[0] = a.x; r.s[1] = a.y; r.s[2] = a.z;
    r.v[0] = a.w; r.v[1] = b.x; r.v[2] = b.y;
    r.s1[0] = b.z; r.s1[1] = b.w; r.s1[2] = c.x;
    r.s2[0] = c.y; r.s2[1] = c.z; r.s2[2] = c.w;
  } else {
    r.lag = (unsigned)j;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      r.s[d] = st.s[d * n + j];
      r.v[d] = st.v[d * n + j];
      r.s1[d] = st.s1[d * n + j];
      r.s2[d] = st.s2[d * n + j];
    }
  }
}

template <int TZ, int MODE>
__global__ __launch_bounds__(TileDims<TZ>::TT) void k_gather_sorted(Lattice lat, Bins bins, SortedState src,
                                                                SortedState dst, const int* __restrict__ idx,
                                                                const int* __restrict__ offset,
                                                                const int* __restrict__ heavy, GatherArgs g,
                                                                KickArgs k, int2* __restrict__ key_rank_next,
                                                                int* __restrict__ count_next) {
  using D = TileDims<TZ>;
  __shared__ float tile[3 * D::EXT];
  TileGeom t;
  bool listed;
  if (!tile_geom<TZ>(bins, heavy, t, listed)) return;
  const long n = lat.npart;
  const int beg = offset[(long)t.bin * kClasses], end = offset[(long)(t.bin + 1) * kClasses];
  if (!listed && tile_is_listed(lat, bins, end - beg)) return;
  // The first batch of particle reads is issued before the force tile is staged,
  // so both are in flight together (most tiles hold one batch or less); in crowded
  // tiles each batch's reads are issued before the previous batch is processed.
  SortedRecord r, rn;
  if (beg < end) load_record(src, n, idx[min(beg + (int)threadIdx.x, end - 1)], r);
  const float* gf[3] = {g.g0, g.g1, g.g2};
  const TileGeom& T_ = t;
  stage_fields<TZ, 3>(t, lat.nm, gf, tile);
  __syncthreads();
  for (int base = beg; base < end; base += D::TT) {   // block-uniform trip count
    const int j = base + threadIdx.x;
    const bool in = j < end;
    const int nbase = base + D::TT;
    if (nbase < end) load_record(src, n, idx[min(nbase + (int)threadIdx.x, end - 1)], rn);
    const Stencil sc = stencil_of(lat, r.lag, r.s);
    const int lc[3] = {sc.c[0] - t.lo[0], sc.c[1] - t.lo[1], sc.c[2] - t.lo[2]};
    // Always true for a listed particle (binning used the same arithmetic); the
    // test only keeps the LDS reads in bounds.
    const bool act =
        in && (unsigned)lc[0] < (unsigned)kTX && (unsigned)lc[1] < (unsigned)kTY && (unsigned)lc[2] < (unsigned)TZ;
    float f[3] = {0.f, 0.f, 0.f};
    if (act) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const float wab = (a ? sc.f[0] : 1.f - sc.f[0]) * (b ? sc.f[1] : 1.f - sc.f[1]);
          const float w0 = wab * (1.f - sc.f[2]), w1 = wab * sc.f[2];
          const int o = ((lc[0] + a) * D::EY + lc[1] + b) * D::EZ + lc[2];
#pragma unroll
          for (int d = 0; d < 3; ++d)
            f[d] += w0 * corner_value<TZ>(tile + d * D::EXT, gf[d], o, T_, lc[0] + a, lc[1] + b, lc[2], lat.nm) +
                    w1 * corner_value<TZ>(tile + d * D::EXT, gf[d], o + 1, T_, lc[0] + a, lc[1] + b, lc[2] + 1, lat.nm);
        }
    }
    float snew[3] = {r.s[0], r.s[1], r.s[2]};
    float vf[3];
    if (in) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float a1 = r.s1[d], a2 = r.s2[d];
        const float v = r.v[d] + k.alpha * (f[d] - k.t2d1 * a1 - k.t2d2 * a2);
        if constexpr (MODE != kGatherFinish) snew[d] = r.s[d] + k.beta * v + k.dd1 * a1 + k.dd2 * a2;
        vf[d] = v;
      }
      if constexpr (MODE == kGatherKickDriftLag) {
        // the caller's Lagrangian-order arrays (when src is the same arrays, each
        // particle is read and written by one lane)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          dst.s[d * n + r.lag] = snew[d];
          dst.v[d * n + r.lag] = vf[d];
        }
      }
      if constexpr (MODE == kGatherKickDriftInv) g.inv[r.lag] = j;
      if constexpr (MODE == kGatherKickDrift || MODE == kGatherKickDriftInv) {
        float4* q = reinterpret_cast<float4*>(dst.s);
        q[j] = make_float4(snew[0], snew[1], snew[2], vf[0]);
        q[n + j] = make_float4(vf[1], vf[2], r.s1[0], r.s1[1]);
        q[2 * n + j] = make_float4(r.s1[2], r.s2[0], r.s2[1], r.s2[2]);
        dst.lag[j] = (int)r.lag;
      }
      if constexpr (MODE == kGatherFinish) {
        // finish: s and the kicked v, in this step's tile order, as a float4 plane
        // (s.x s.y s.z v.x) and a float2 plane (v.y v.z), and the slot of every
        // Lagrangian index in dst.lag, for k_unsort (which forms x and v_phys)
        reinterpret_cast<float4*>(dst.s)[j] = make_float4(r.s[0], r.s[1], r.s[2], vf[0]);
        reinterpret_cast<float2*>(dst.s + 4 * n)[j] = make_float2(vf[1], vf[2]);
        dst.lag[r.lag] = j;
      }
    }
    if constexpr (MODE == kGatherKickDrift || MODE == kGatherKickDriftInv) {
      int bin = 0;
      if (in) bin = key_of<TZ>(bins, stencil_of(lat, r.lag, snew).c);
      const int rank = wave_rank(in, bin, count_next);
      if (in) key_rank_next[j] = make_int2(bin, rank);
    }
    r = rn;
  }
}

// ---------------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al. 2011) white noise with Box-Muller pairs.
// Block g of 4 values: counter (g lo, g hi, 0, 0), key (seed lo, seed hi);
// (r0, r1) -> values 4g, 4g+1; (r2, r3) -> 4g+2, 4g+3;
// u1 = ((r >> 8) + 1) 2^-24, u2 = (r' >> 8) 2^-24, z = sqrt(-2 ln u1) (cos, sin)(2 pi u2).
// ---------------------------------------------------------------------------------
__device__ __forceinline__ void philox_round(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
  const uint32_t hi0 = __umulhi(m0, c[0]), lo0 = m0 * c[0];
  const uint32_t hi1 = __umulhi(m1, c[2]), lo1 = m1 * c[2];
  const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

__global__ __launch_bounds__(kPartThreads) void k_noise(uint64_t seed, float* __restrict__ w, long count) {
  const long g = (long)blockIdx.x * kPartThreads + threadIdx.x;
  if (4 * g >= count) return;
  uint32_t c[4] = {(uint32_t)g, (uint32_t)((uint64_t)g >> 32), 0u, 0u};
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    philox_round(c, k0, k1);
  }
  float z[4];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const float u1 = (float)((c[2 * j] >> 8) + 1u) * 5.9604644775390625e-8f;
    const float u2 = (float)(c[2 * j + 1] >> 8) * 5.9604644775390625e-8f;
    const float rad = sqrtf(-2.0f * logf(u1));
    float sn, cs;
    sincospif(2.0f * u2, &sn, &cs);
    z[2 * j] = rad * cs;
    z[2 * j + 1] = rad * sn;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (4 * g + j < count) w[4 * g + j] = z[j];
}

// ---------------------------------------------------------------------------------
Bins make_bins(int nm, int tz_max) {
  Bins b;
  b.tx = kTX;
  b.ty = kTY;
  b.tz = 8;
  while (b.tz < tz_max && b.tz < 64 && nm % (2 * b.tz) == 0) b.tz *= 2;
  b.nbx = nm / b.tx;
  b.nby = nm / b.ty;
  b.nbz = nm / b.tz;
  b.nbins = (long)b.nbx * b.nby * b.nbz;
  b.nkeys = b.nbins * kClasses;
  b.heavy_cap = (int)((b.nbins + 16 * kXcds - 1) / (16 * kXcds) * kXcds);   // ~nbins / 16, a multiple of 8
  return b;
}

static size_t count_len(const Bins& b) { return (size_t)((b.nkeys + 4) / 4 * 4); }
static size_t scan_chunks(const Bins& b) { return (size_t)((b.nkeys + kScanChunk - 1) / kScanChunk); }

static size_t part_len(const Bins& b) { return (scan_chunks(b) + 4) / 4 * 4; }

size_t bin_workspace_bytes(long npart, const Bins& b) {
  return npart * sizeof(int2) + npart * sizeof(int) + 3 * count_len(b) * sizeof(int) + part_len(b) * sizeof(int) +
         (size_t)(b.heavy_cap + 4) / 4 * 4 * sizeof(int);
}

BinBuffers carve_bins(void* base, long npart, const Bins& b) {
  char* c = static_cast<char*>(base);
  const size_t cnt = count_len(b);
  BinBuffers bb;
  bb.key_rank = reinterpret_cast<int2*>(c);
  c += npart * sizeof(int2);
  bb.idx = reinterpret_cast<int*>(c);
  c += npart * sizeof(int);
  bb.count = reinterpret_cast<int*>(c);
  c += cnt * sizeof(int);
  bb.count_next = reinterpret_cast<int*>(c);
  c += cnt * sizeof(int);
  bb.offset = reinterpret_cast<int*>(c);
  c += cnt * sizeof(int);
  bb.part = reinterpret_cast<int*>(c);
  c += part_len(b) * sizeof(int);
  bb.heavy = reinterpret_cast<int*>(c);
  bb.count_len = (long)cnt;
  bb.npart = npart;
  return bb;
}

hipError_t launch_fill(float* p, long n, float value, hipStream_t st) {
  if (n % 4) return hipErrorInvalidValue;
  const long n4 = n / 4;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n4 + kPartThreads - 1) / kPartThreads)), dim3(kPartThreads), 0, st,
                     reinterpret_cast<float4*>(p), n4, value);
  return hipGetLastError();
}

static unsigned part_blocks(long npart) { return (unsigned)((npart + kPartThreads - 1) / kPartThreads); }
// Listed crowded tiles first, then every tile in XCD order (tile_geom).
static unsigned tile_blocks(const Bins& b) {
  return (unsigned)(b.heavy_cap + (b.nbins + kXcds - 1) / kXcds * kXcds);
}

#define COLA_TZ_DISPATCH(tz, CALL) \
  switch (tz) {                    \
    case 8: { constexpr int TZ = 8; CALL; break; }   \
    case 16: { constexpr int TZ = 16; CALL; break; } \
    case 32: { constexpr int TZ = 32; CALL; break; } \
    case 64: { constexpr int TZ = 64; CALL; break; } \
    default: return hipErrorInvalidValue;            \
  }

hipError_t launch_bin_count(Lattice lat, Bins b, const float* s, BinBuffers bb, hipStream_t st) {
  hipError_t e = launch_fill(reinterpret_cast<float*>(bb.count), bb.count_len, 0.0f, st);
  if (e != hipSuccess) return e;
  COLA_TZ_DISPATCH(b.tz, hipLaunchKernelGGL(k_bin_count<TZ>, dim3(part_blocks(lat.npart)), dim3(kPartThreads), 0, st,
                                            lat, b, s, bb.key_rank, bb.count));
  return hipGetLastError();
}

hipError_t launch_bin_scan(Bins b, BinBuffers bb, bool clear_next, hipStream_t st) {
  const int n = (int)b.nkeys;
  const unsigned nb = (unsigned)scan_chunks(b);
  hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(kScanThreads), 0, st, bb.count, n, bb.part,
                     clear_next ? bb.count_next : nullptr, (int)bb.count_len);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, st, bb.part, (int)nb, bb.offset + n, bb.heavy);
  hipLaunchKernelGGL(k_scan_chunks, dim3(nb), dim3(kScanThreads), 0, st, bb.count, n, bb.part, bb.offset);
  hipLaunchKernelGGL(k_heavy_tiles, dim3((unsigned)((b.nbins + kPartThreads - 1) / kPartThreads)), dim3(kPartThreads), 0,
                     st, b.nbins, bb.offset, heavy_min_of(bb.npart, b.heavy_cap), bb.heavy);
  return hipGetLastError();
}

hipError_t launch_bin_scatter_pack(Lattice lat, BinBuffers bb, SortedState src, SortedState dst, hipStream_t st) {
  if (src.lag || !dst.s || !dst.lag || reinterpret_cast<uintptr_t>(dst.s) % 16 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_bin_scatter_pack, dim3(part_blocks(lat.npart)), dim3(kPartThreads), 0, st, lat.npart,
                     bb.key_rank, bb.offset, bb.idx, src, dst);
  return hipGetLastError();
}

hipError_t launch_bin_scatter(Lattice lat, BinBuffers bb, hipStream_t st) {
  hipLaunchKernelGGL(k_bin_scatter, dim3(part_blocks(lat.npart)), dim3(kPartThreads), 0, st, lat.npart, bb.key_rank,
                     bb.offset, bb.idx);
  return hipGetLastError();
}

// max |x| over count floats into *out (which the caller clears), as the bits of a
// non-negative float, whose unsigned order is the numeric order with +inf above every
// finite value and NaN above +inf: a non-finite entry gives a non-finite maximum.
// One atomic per block: atomics on a single address serialise in L2, so the waves of a
// block combine their maxima in LDS first.  Each thread keeps four loads in flight.
constexpr int kAbsmaxBlocks = 1024;
__global__ __launch_bounds__(kPartThreads) void k_absmax(const float* __restrict__ x, long count,
                                                         unsigned* __restrict__ out) {
  __shared__ unsigned wave_max[kPartThreads / 64];
  unsigned m = 0;
  const long step = (long)gridDim.x * kPartThreads;
  long i = (long)blockIdx.x * kPartThreads + threadIdx.x;
  for (; i + 3 * step < count; i += 4 * step) {
    const unsigned a = __float_as_uint(x[i]), b = __float_as_uint(x[i + step]);
    const unsigned c = __float_as_uint(x[i + 2 * step]), d = __float_as_uint(x[i + 3 * step]);
    m = max(max(m, a & 0x7fffffffu), max(max(b & 0x7fffffffu, c & 0x7fffffffu), d & 0x7fffffffu));
  }
  for (; i < count; i += step) m = max(m, __float_as_uint(x[i]) & 0x7fffffffu);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, o));
  if (__lane_id() == 0) wave_max[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kPartThreads / 64; ++k) m = max(m, wave_max[k]);   // m: wave 0's maximum
    atomicMax(out, m);
  }
}

hipError_t launch_deposit3(Lattice lat, Bins b, const float* s, BinBuffers bb, float* rho, float mass,
                           const float* weight, unsigned* wmax, hipStream_t st) {
  if (!weight || !wmax) return hipErrorInvalidValue;
  // the scale of the fixed-point sums: max |weight| over the three components
  const hipError_t e = launch_fill(reinterpret_cast<float*>(wmax), 4, 0.0f, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_absmax, dim3(kAbsmaxBlocks), dim3(kPartThreads), 0, st, weight, 3 * lat.npart, wmax);
  COLA_TZ_DISPATCH(b.tz, hipLaunchKernelGGL((k_deposit_tiles<TZ, unsigned long long, 3>), dim3(tile_blocks(b)),
                                            dim3(TileDims<TZ>::TT), 0, st, lat, b, s, nullptr, bb.idx, bb.offset,
                                            bb.heavy, rho, mass, weight, wmax))
  return hipGetLastError();
}

hipError_t launch_deposit(Lattice lat, Bins b, const float* s, BinBuffers bb, float* rho, float mass,
                          hipStream_t st, const int* lag) {
  COLA_TZ_DISPATCH(b.tz, hipLaunchKernelGGL((k_deposit_tiles<TZ, unsigned long long>), dim3(tile_blocks(b)),
                                            dim3(TileDims<TZ>::TT), 0, st, lat, b, s, lag, bb.idx, bb.offset, bb.heavy, rho,
                                            mass, nullptr, nullptr))
  return hipGetLastError();
}

hipError_t launch_gather_force(Lattice lat, Bins b, BinBuffers bb, GatherArgs a, hipStream_t st) {
  COLA_TZ_DISPATCH(b.tz, hipLaunchKernelGGL(k_gather_tiles<TZ>, dim3(tile_blocks(b)), dim3(TileDims<TZ>::TT), 0, st,
                                            lat, b, bb.idx, bb.offset, bb.heavy, a));
  return hipGetLastError();
}

template <int TZ>
static void gather_sorted_tz(Lattice lat, Bins b, SortedState src, SortedState dst, BinBuffers bb, int mode,
                             GatherArgs a, KickArgs k, hipStream_t st) {
  const dim3 grid(tile_blocks(b)), block(TileDims<TZ>::TT);
  if (mode == kGatherKickDrift)
    hipLaunchKernelGGL((k_gather_sorted<TZ, kGatherKickDrift>), grid, block, 0, st, lat, b, src, dst, bb.idx,
                       bb.offset, bb.heavy, a, k, bb.key_rank, bb.count_next);
  else if (mode == kGatherKickDriftInv)
    hipLaunchKernelGGL((k_gather_sorted<TZ, kGatherKickDriftInv>), grid, block, 0, st, lat, b, src, dst, bb.idx,
                       bb.offset, bb.heavy, a, k, bb.key_rank, bb.count_next);
  else if (mode == kGatherKickDriftLag)
    hipLaunchKernelGGL((k_gather_sorted<TZ, kGatherKickDriftLag>), grid, block, 0, st, lat, b, src, dst, bb.idx,
                       bb.offset, bb.heavy, a, k, bb.key_rank, bb.count_next);
  else
    hipLaunchKernelGGL((k_gather_sorted<TZ, kGatherFinish>), grid, block, 0, st, lat, b, src, dst, bb.idx, bb.offset, bb.heavy,
                       a, k, bb.key_rank, bb.count_next);
}

hipError_t launch_gather_sorted(Lattice lat, Bins b, SortedState src, SortedState dst, BinBuffers bb, int mode,
                                GatherArgs a, KickArgs k, hipStream_t st) {
  if (mode != kGatherKickDrift && mode != kGatherFinish && mode != kGatherKickDriftLag &&
      mode != kGatherKickDriftInv)
    return hipErrorInvalidValue;
  if (mode == kGatherKickDriftInv && !a.inv) return hipErrorInvalidValue;
  if (mode == kGatherKickDriftLag) {
    // dst is the caller's SoA arrays (s, v) in Lagrangian order
    if (!dst.s || !dst.v || dst.lag) return hipErrorInvalidValue;
  } else if (!dst.s || !dst.lag || reinterpret_cast<uintptr_t>(dst.s) % 16 != 0) {
    // dst is packed: 12 n floats from dst.s, 16-byte aligned, and n ints of lag
    return hipErrorInvalidValue;
  }
  if (src.lag && reinterpret_cast<uintptr_t>(src.s) % 16 != 0) return hipErrorInvalidValue;
  COLA_TZ_DISPATCH(b.tz, gather_sorted_tz<TZ>(lat, b, src, dst, bb, mode, a, k, st));
  return hipGetLastError();
}

// Lagrangian order from the finish output: particle p takes s and v from slot inv[p]
// of the tile-ordered finish copy, then L+(a_n) (eq. Lops): v_phys = v + T[D1] s1 +
// T[D2] s2 (k.td1, k.td2; s1, s2 from the caller's arrays, read in order) and
// x = (q + s) mod L.  Only 24 bytes per particle are read out of order.  A block
// covers a 4 x 4 x 16 block of the Lagrangian grid (when np allows), whose particles
// sit in a few neighbouring tiles, so its scattered reads stay local; its writes are
// runs of 16 consecutive elements.
// Lagrangian index of this thread in the unsort-order walks: a block takes a 4 x 4 x 16
// block of the Lagrangian grid (when np allows), whose particles sit in a few
// neighbouring tiles, so its out-of-order reads stay local and its writes are runs of
// 16 consecutive elements.
__device__ __forceinline__ long unsort_index(const Lattice& lat) {
  const int np = lat.np;
  if (np % 16 == 0) {
    const int nbk = np / 16, nbj = np / 4;
    const int b = blockIdx.x;
    const int bk = b % nbk, bj = (b / nbk) % nbj, bi = b / (nbk * nbj);
    const int t = threadIdx.x;
    return ((long)(4 * bi + t / 64) * np + 4 * bj + (t / 16) % 4) * np + 16 * bk + t % 16;
  }
  return (long)blockIdx.x * kPartThreads + threadIdx.x;
}

__global__ __launch_bounds__(kPartThreads) void k_writeback(Lattice lat, const float4* __restrict__ w,
                                                            const int* __restrict__ inv, float* __restrict__ s,
                                                            float* __restrict__ v) {
  const long n = lat.npart;
  const long p = unsort_index(lat);
  if (p >= n) return;
  const long j = inv[p];
  const float4 a = w[j], b = w[n + j];   // (s.x s.y s.z v.x), (v.y v.z s1.x s1.y)
  s[p] = a.x;
  s[n + p] = a.y;
  s[2 * n + p] = a.z;
  v[p] = a.w;
  v[n + p] = b.x;
  v[2 * n + p] = b.y;
}

hipError_t launch_writeback(Lattice lat, SortedState w, const int* inv, float* s, float* v, hipStream_t st) {
  if (!w.s || !inv || !s || !v || reinterpret_cast<uintptr_t>(w.s) % 16 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_writeback, dim3(part_blocks(lat.npart)), dim3(kPartThreads), 0, st, lat,
                     reinterpret_cast<const float4*>(w.s), inv, s, v);
  return hipGetLastError();
}

__global__ __launch_bounds__(kPartThreads) void k_unsort(Lattice lat, SortedState w, GatherArgs g, KickArgs k) {
  const int np = lat.np;
  const long n = lat.npart;
  const long p = unsort_index(lat);
  if (p >= n) return;
  const long j = w.lag[p];
  const float4 a = reinterpret_cast<const float4*>(w.s)[j];
  const float2 b = reinterpret_cast<const float2*>(w.s + 4 * n)[j];
  const float sv[3] = {a.x, a.y, a.z}, vv[3] = {a.w, b.x, b.y};
  int li[3];
  lag_index(lat, (unsigned)p, li);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    g.s[d * n + p] = sv[d];
    g.v[d * n + p] = vv[d];
    g.out_b[d * n + p] = vv[d] + k.td1 * g.s1[d * n + p] + k.td2 * g.s2[d * n + p];
    float x = (float)li[d] * (k.box / (float)np) + sv[d];
    x = x - k.box * floorf(x / k.box);
    if (x >= k.box) x -= k.box;
    g.out_a[d * n + p] = x;
  }
}

hipError_t launch_unsort(Lattice lat, SortedState w, GatherArgs a, KickArgs k, hipStream_t st) {
  hipLaunchKernelGGL(k_unsort, dim3(part_blocks(lat.npart)), dim3(kPartThreads), 0, st, lat, w, a, k);
  return hipGetLastError();
}

hipError_t launch_grad_gather(Lattice lat, Bins b, BinBuffers bb, const float* s, AdjGatherArgs ga, hipStream_t st) {
  COLA_TZ_DISPATCH(b.tz, hipLaunchKernelGGL(k_grad_gather<TZ>, dim3(tile_blocks(b)), dim3(TileDims<TZ>::TT), 0, st, lat, b,
                                            bb.idx, bb.offset, bb.heavy, s, ga));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Elementwise adjoint updates over [3][n] particle arrays.
// ---------------------------------------------------------------------------------
// Reverse of v' = v + alpha (F - c1 s1 - c2 s2), s' = s + beta v' + d1 s1 + d2 s2:
//   mu = lam_v + beta lam_s;  lam_s1 += d1 lam_s - alpha c1 mu;
//   lam_s2 += d2 lam_s - alpha c2 mu;  lam_v = mu  (lam_s is updated by the gather).
__global__ __launch_bounds__(kPartThreads) void k_adj_kick_drift(long n3, AdjStepArgs a, float* __restrict__ lam_s,
                                                                 float* __restrict__ lam_v, float* __restrict__ lam_s1,
                                                                 float* __restrict__ lam_s2) {
  const long i = (long)blockIdx.x * kPartThreads + threadIdx.x;
  if (i >= n3) return;
  const float ls = lam_s[i];
  const float mu = lam_v[i] + a.beta * ls;
  lam_s1[i] += a.dd1 * ls - a.alpha * a.t2d1 * mu;
  lam_s2[i] += a.dd2 * ls - a.alpha * a.t2d2 * mu;
  lam_v[i] = mu;
}

hipError_t launch_adj_kick_drift(long n3, AdjStepArgs a, float* lam_s, float* lam_v, float* lam_s1, float* lam_s2,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_adj_kick_drift, dim3((unsigned)((n3 + kPartThreads - 1) / kPartThreads)), dim3(kPartThreads),
                     0, st, n3, a, lam_s, lam_v, lam_s1, lam_s2);
  return hipGetLastError();
}

// y += a x over n floats
__global__ __launch_bounds__(kPartThreads) void k_axpy(long n, float a, const float* __restrict__ x,
                                                       float* __restrict__ y) {
  const long i = (long)blockIdx.x * kPartThreads + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

hipError_t launch_axpy(long n, float a, const float* x, float* y, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3((unsigned)((n + kPartThreads - 1) / kPartThreads)), dim3(kPartThreads), 0, st, n, a,
                     x, y);
  return hipGetLastError();
}

// Adjoint of S = sum_{i<j} (phi_ii phi_jj - phi_ij^2) with cotangent sigma, in place:
// phi_aa <- sigma (tr phi - phi_aa), phi_ab <- -2 sigma phi_ab.  phi order xx yy zz xy yz zx.
__global__ __launch_bounds__(kPartThreads) void k_hessian_adjoint(long n, const float* __restrict__ sigma,
                                                                  HessPtrs h) {
  const long i = (long)blockIdx.x * kPartThreads + threadIdx.x;
  if (i >= n) return;
  const float sg = sigma[i];
  const float xx = h.p[0][i], yy = h.p[1][i], zz = h.p[2][i];
  const float tr = xx + yy + zz;
  h.p[0][i] = sg * (tr - xx);
  h.p[1][i] = sg * (tr - yy);
  h.p[2][i] = sg * (tr - zz);
  h.p[3][i] = -2.f * sg * h.p[3][i];
  h.p[4][i] = -2.f * sg * h.p[4][i];
  h.p[5][i] = -2.f * sg * h.p[5][i];
}

hipError_t launch_hessian_adjoint(long n, const float* sigma, HessPtrs h, hipStream_t st) {
  hipLaunchKernelGGL(k_hessian_adjoint, dim3((unsigned)((n + kPartThreads - 1) / kPartThreads)), dim3(kPartThreads), 0,
                     st, n, sigma, h);
  return hipGetLastError();
}

hipError_t launch_noise(uint64_t seed, float* w, long count, hipStream_t st) {
  const long ng = (count + 3) / 4;
  hipLaunchKernelGGL(k_noise, dim3((unsigned)((ng + kPartThreads - 1) / kPartThreads)), dim3(kPartThreads), 0, st,
                     seed, w, count);
  return hipGetLastError();
}

}  // namespace cola
