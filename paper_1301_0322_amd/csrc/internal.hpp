// Internal declarations shared by the host code and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

struct cola_plan_s;

namespace cola {

constexpr int kMaxFields = 9;

struct FieldPtrs {
  float2* p[kMaxFields];
};

// k-space multiplier applied between the forward and inverse x transforms.
enum MulMode : int {
  kMulGrad = 0,      // out_j = c * i n_j / n^2 * X            (3 outputs)
  kMulLpt1 = 1,      // s1_j = i n_j tab[n^2] X, phi_ij = kf n_i n_j tab[n^2] X  (9 outputs)
  kMulGradPair = 2,  // out_0 = c * i n_x / n^2 * X, out_1 = c / n^2 * X  (2 outputs): the y and z
                     // components follow from out_1 in the y and z passes (i n_y, i n_z there)
};

struct MulArgs {
  float c;            // kMulGrad scale
  float kf;           // fundamental wavenumber, kMulLpt1 phi scale
  const float* tab;   // kMulLpt1 table indexed by n^2
};

// Epilogue of the inverse z (complex-to-real) pass.
enum ZinvEpi : int {
  kEpiStore = 0,      // out = scale * x
  kEpiLptFinal = 1,   // out = s2_d; s_d = d1 s1_d + d2 s2_d; v_d = v1 s1_d + v2 s2_d
};

struct EpiArgs {
  float scale;
  float d1, d2;
  float v1, v2;
  const float* s1;    // component base pointers, advanced by comp_stride per field
  float* s;
  float* v;
  long comp_stride;
  int reverse;        // rows from the last block to the first (memory-side cache reuse)
  int deriv;          // bit f: field f's mode k is multiplied by i k before the transform (z derivative)
  int nfields;        // set by launch_zinv
};

bool fft_size_supported(int n);

// Forward real-to-complex z pass: rows of n reals -> rows of n/2 complex
// (modes 0..n/2-1; the n/2 mode is dropped).  in and out may alias.
hipError_t launch_zfwd(int n, const float* in, float2* out, long nrows, const float2* tw,
                       hipStream_t st);
// Inverse complex-to-real z pass for nfields fields; field f reads in.p[f], writes
// out.p[f] (as float rows).  May alias.
hipError_t launch_zinv(int n, FieldPtrs in, FieldPtrs out, int nfields, long nrows,
                       const float2* tw, int epi, EpiArgs epi_args, hipStream_t st);
// Inverse z pass over the six Hessian fields (xx, yy, zz, xy, yz, zx) writing the
// second-order source S = sum_{i<j} (phi_ii phi_jj - phi_ij^2) as real rows.
hipError_t launch_zinv_hessian(int n, FieldPtrs in, float* out, long nrows, const float2* tw,
                               float scale, hipStream_t st);
// Strided column pass (length n along inner_stride) over tiles of contiguous columns.
// Tiles: outer index o in [0, n_outer) at outer_stride; columns [0, ncols) contiguous.
// width: columns per tile (4, 8 or 16; 0 picks the default for n).
// rot (0 <= rot < n): for y passes (o = x plane, inner_stride = one row), the k-space
// side (output of dir < 0, input of dir > 0) is a rotated half spectrum: row y of plane
// x at row (y + rot x) mod n.  0 for the plain layout and for passes along x.
// reverse: blocks take the tiles from the last to the first.
hipError_t launch_col(int n, int dir, FieldPtrs in, FieldPtrs out, int nfields, int n_outer,
                      long outer_stride, long inner_stride, int ncols, const float2* tw, int width, int rot,
                      hipStream_t st, int reverse = 0);
// Shell statistics of one or two half spectra (b may be null) into out[6][n/2]
// (doubles, row r, shell s = round(|n|) for 1 <= s < n/2; s = 0 stays zero): mode
// count, P_aa, P_bb, P_ab (sums / count * norm), rho and n_max.  part holds
// part_doubles doubles of per-block partial sums (at least 2 n).
hipError_t launch_shell_stats(int n, const float2* a, const float2* b, double* part, long part_doubles, double norm,
                              double* out, hipStream_t st);
// Inverse column pass of one field with two outputs: out_d = inverse transform of
// i n X (n the signed mode number along the column) and out_p = inverse transform of
// X.  The three buffers are distinct.  in is rotated by rot as the input of an
// inverse y pass of launch_col; the outputs are plain.
hipError_t launch_col_pair(int n, const float2* in, float2* out_p, float2* out_d, int n_outer, long outer_stride,
                           long inner_stride, int ncols, const float2* tw, int width, int rot, hipStream_t st,
                           int reverse = 0);
// x pass with the k-space multiplier: forward x transform of `in`, multiply, inverse
// x transform into each of nout outputs.  Layout [x][y][kz] with n/2 kz per row, the
// rows of every x plane rotated by rot (input and outputs alike), rot a multiple of
// fft_rot_rows(n).  kMulGrad requires nout = 3, kMulGradPair 2, kMulLpt1 1..9.
hipError_t launch_xmul(int n, int mode, const float2* in, FieldPtrs out, int nout, MulArgs m,
                       const float2* tw, int width, int rot, hipStream_t st);
// Rows per plane by which a rotated half spectrum of transform length n is rotated
// (the x passes' R2, so that a thread's rows share one stride), and whether plans
// rotate by default at length n.
int fft_rot_rows(int n);
bool fft_rot_default_on(int n);
// Whether `width` columns per tile is a valid strided-pass shape for length n.
bool fft_width_supported(int n, int width);

// Particle kernels.
struct Lattice {
  int np;           // particles per side
  int nm;           // mesh cells per side
  int ratio;        // nm / np
  float inv_dx;     // nm / L rounded to float
  float inv_dx_lo;  // nm / L - inv_dx (the rounding remainder, as a float)
  long npart;       // np^3
  // x / np for x < 2^31 as (x * np_magic) >> (31 + np_shift): np_shift = ceil(log2 np),
  // np_magic = floor(2^(31 + np_shift) / np) + 1 (Granlund and Montgomery 1994, the
  // round-up method; exact because np_magic * np lies in (2^(31+l), 2^(31+l) + np]).
  unsigned np_magic;
  int np_shift;
};
inline void set_lattice_divisor(Lattice& l) {
  int s = 0;
  while ((1L << s) < l.np) ++s;
  l.np_shift = s;
  l.np_magic = (unsigned)((1ULL << (31 + s)) / (unsigned long long)l.np + 1);
}

hipError_t launch_fill(float* p, long n, float value, hipStream_t st);

// Eulerian tiles of tx x ty x tz cells used to bin particles every step.  Within a
// tile, particles are further keyed by a 3-bit boundary class (bit d: the base cell
// is on the tile's upper face along d); key = 8 tile + class.
struct Bins {
  int tx, ty, tz;
  int nbx, nby, nbz;
  long nbins;
  long nkeys;        // 8 nbins
  int heavy_cap;     // crowded-tile list capacity (a multiple of 8, about nbins / 16)
};
struct BinBuffers {
  int2* key_rank;    // [npart] (key, rank within key)
  int* idx;          // [npart] particle slots grouped by key
  int* count;        // [count_len] particles per key
  int* count_next;   // [count_len] counts for the next step, filled by a binning gather
  int* offset;       // [count_len] exclusive prefix sum, offset[nkeys] = npart
  int* part;         // scan chunk sums
  int* heavy;        // [1 + heavy_cap] number of crowded tiles, then their indices
  long count_len;
  long npart;
};
// A tile is crowded when its own classes hold more than ceil(npart / heavy_cap)
// particles; fewer than heavy_cap tiles can be.  The scan lists them and the tile
// kernels run them first.
__host__ __device__ inline int heavy_min_of(long npart, int heavy_cap) {
  return (int)((npart + heavy_cap - 1) / heavy_cap);
}
// Tile depth: the largest of 8, 16, 32, 64 (<= tz_max) dividing nm.  32 by default:
// with the force tiles staged without halo, 8 x 8 x 32 tiles (25 KB of LDS, 256
// threads) keep more blocks resident than 8 x 8 x 64 and measure as fast or faster at
// every mesh size benchmarked; the autotuner can pick any depth per plan.
Bins make_bins(int nm, int tz_max = 32);
size_t bin_workspace_bytes(long npart, const Bins& b);
BinBuffers carve_bins(void* base, long npart, const Bins& b);

hipError_t launch_bin_count(Lattice lat, Bins b, const float* s, BinBuffers bb, hipStream_t st);
// clear_next also zeroes count_next for a binning gather later in the step.
// Also lists the crowded tiles (bb.heavy) for the tile kernels.
hipError_t launch_bin_scan(Bins b, BinBuffers bb, bool clear_next, hipStream_t st);
hipError_t launch_bin_scatter(Lattice lat, BinBuffers bb, hipStream_t st);
// Tile deposit: each tile accumulates its own particles and the boundary classes of
// its lower neighbours that reach into it, then writes its cells with plain stores.
// rho needs no clearing.  bb.idx lists slots of s by key.  With lag, s is a packed
// state (SortedState) and lag gives a slot's Lagrangian index; without, s is SoA
// [3][np^3] in Lagrangian order.  weight (optional, [np^3] by Lagrangian index): the
// particle carries mass * weight.
hipError_t launch_deposit(Lattice lat, Bins b, const float* s, BinBuffers bb, float* rho, float mass,
                          hipStream_t st, const int* lag = nullptr);
// Three weighted deposits in one particle walk: rho + c nm^3 receives the CIC deposit
// of mass * weight[c n + Lagrangian index], c = 0..2 (s SoA in Lagrangian order), summed
// in 64-bit fixed point after scaling by a power of two from max |weight| (computed into
// wmax, four words of device scratch).  Deterministic: independent of particle order.
hipError_t launch_deposit3(Lattice lat, Bins b, const float* s, BinBuffers bb, float* rho, float mass,
                           const float* weight, unsigned* wmax, hipStream_t st);

struct KickArgs {
  float alpha;                 // kick factor
  float t2d1, t2d2;            // T^2[D1](a_c), T^2[D2](a_c)
  float beta;                  // drift factor (do_drift)
  float dd1, dd2;              // D1, D2 increments (do_drift)
  float td1, td2;              // T[D1](a_n), T[D2](a_n) for L+ (finish)
  float box;
};
// Modes of launch_gather_sorted (the force-only gather is launch_gather_force).
enum GatherMode : int {
  kGatherKickDrift = 1,     // v += alpha (F - t2d1 s1 - t2d2 s2); s += beta v + dd1 s1 + dd2 s2, written
                            // packed in this step's tile order and binned for the next step
  kGatherFinish = 2,        // the kick only, written packed for launch_unsort (x, L+)
  kGatherKickDriftLag = 3,  // kick and drift, s and v written to the caller's Lagrangian-order arrays
                            // (dst SoA, by each record's Lagrangian index; no binning)
  kGatherKickDriftInv = 4,  // kGatherKickDrift, and a.inv[Lagrangian index] = dst slot (for
                            // launch_writeback)
};
struct GatherArgs {
  const float* g0;
  const float* g1;
  const float* g2;
  float* s;
  float* v;
  const float* s1;
  const float* s2;
  float* out_a;     // force gather: acc; launch_unsort: x
  float* out_b;     // launch_unsort: v_phys
  int* inv;         // kGatherKickDriftInv: slot of every Lagrangian index ([n])
};
// Force gather (cola_pm_force): a.out_a[d n + p] = F_d of particle p of the SoA
// displacements a.s, through the tile lists of bb.
hipError_t launch_gather_force(Lattice lat, Bins b, BinBuffers bb, GatherArgs a, hipStream_t st);

// Particle state ordered by tile (slot j), with each particle's Lagrangian index.
// lag == nullptr: the caller's SoA arrays s, v, s1, s2 ([3][n], slot = Lagrangian
// index).  lag != nullptr: a packed state, s pointing at 12 n floats (16-byte
// aligned) read as float4[3][n] = (s.x s.y s.z v.x), (v.y v.z s1.x s1.y),
// (s1.z s2.x s2.y s2.z); v, s1, s2 are unused.
struct SortedState {
  float* s;
  float* v;
  float* s1;
  float* s2;
  int* lag;
};
// The scatter of the public step: idx becomes the identity and dst (packed) receives, at
// each particle's tile-sorted slot, its record from the caller's Lagrangian-order SoA
// arrays src (src.lag == nullptr).
hipError_t launch_bin_scatter_pack(Lattice lat, BinBuffers bb, SortedState src, SortedState dst, hipStream_t st);
// Gather + kick over the tile lists bb.idx (slots of src).  kGatherKickDrift writes
// the kicked and drifted record of list position j to slot j of the packed dst
// (ordered by this step's tiles) and bins it for the next step (bb.count_next,
// bb.key_rank by dst slot); kGatherFinish writes s and the kicked v of list position
// j as float4 j of dst.s (s.x s.y s.z v.x) and float2 j of dst.s + 4n (v.y v.z), and
// sets dst.lag[Lagrangian index] = j, for launch_unsort.  kGatherKickDriftInv does
// what kGatherKickDrift does and also records each record's dst slot in a.inv at its
// Lagrangian index.
hipError_t launch_gather_sorted(Lattice lat, Bins b, SortedState src, SortedState dst, BinBuffers bb, int mode,
                                GatherArgs a, KickArgs k, hipStream_t st);
// The caller's Lagrangian-order s and v ([3][n]) from the packed state w (a
// kGatherKickDriftInv dst) and its inverse permutation inv.
hipError_t launch_writeback(Lattice lat, SortedState w, const int* inv, float* s, float* v, hipStream_t st);
// Lagrangian order from a kGatherFinish output w: a.s, a.v take s and v; a.out_a
// x = (q + s) mod L (k.box); a.out_b v_phys = v + k.td1 a.s1 + k.td2 a.s2, the L+ of
// the closing step (a.s1, a.s2 the caller's arrays).
hipError_t launch_unsort(Lattice lat, SortedState w, GatherArgs a, KickArgs k, hipStream_t st);

// Adjoint kernels.
struct AdjGatherArgs {
  const float* g0;    // force meshes (nullptr: density term only)
  const float* g1;
  const float* g2;
  const float* mu;    // [3][np^3] cotangent of the force (with g)
  const float* rbar;  // dL/drho mesh
  float* lam_s;       // [3][np^3] accumulated dL/ds
  float f1, f2;       // scales of the force-field and density terms (include 1/dx)
};
hipError_t launch_grad_gather(Lattice lat, Bins b, BinBuffers bb, const float* s, AdjGatherArgs ga, hipStream_t st);
struct AdjStepArgs {
  float alpha, beta, t2d1, t2d2, dd1, dd2;
};
hipError_t launch_adj_kick_drift(long n3, AdjStepArgs a, float* lam_s, float* lam_v, float* lam_s1, float* lam_s2,
                                 hipStream_t st);
hipError_t launch_axpy(long n, float a, const float* x, float* y, hipStream_t st);
struct HessPtrs {
  float* p[6];
};
hipError_t launch_hessian_adjoint(long n, const float* sigma, HessPtrs h, hipStream_t st);
// Transposed x pass: forward x transform of each of nin inputs, multiply by the
// complex conjugate of the mode's multiplier for that input, sum, inverse x
// transform into out.  kMulGrad: nin = 3 (conj of c i n_j / n^2); kMulLpt1: nin = 9
// (conj of the s1_j and phi_ab multipliers).  Inputs and output rotated by rot.
hipError_t launch_xmul_adj(int n, int mode, FieldPtrs in, int nin, float2* out, MulArgs m, const float2* tw,
                           int rot, hipStream_t st);

hipError_t launch_noise(uint64_t seed, float* w, long count, hipStream_t st);

// Entry points of the allocation-free density (defined with the plan in cola_api.cpp).
// record_hip: COLA status of a HIP error, kept for cola_last_hip_error().
// plan_bin_bytes: bytes of the binning buffers of the plan's particle and tile counts.
// density_with_bins: the mean-1 CIC density of particles at q + s into rho, with the
// binning buffers carved from bin_base (plan_bin_bytes(p) bytes, 256-byte aligned);
// enqueues kernels only (no allocation, no plan-table upload); COLA_ERR_INVALID when
// the plan traces (its events are created on demand).
int record_hip(hipError_t e);
size_t plan_bin_bytes(cola_plan_s* p);
int density_with_bins(cola_plan_s* p, const float* s, float* rho, void* bin_base, hipStream_t st);

}  // namespace cola
