// Per-particle kernels on gfx950: cloud-in-cell deposit, the fused CIC gather +
// COLA kick + drift, Philox white noise and a fill kernel.
//
// Particles are in Lagrangian order p = (i np + j) np + k (k fastest) with SoA
// components [3][np^3]; the Lagrangian position q = (i, j, k) L / np is implicit.
// Cell-centred mesh: the mesh coordinate of a particle is
//   u = ratio * (i, j, k) + (s / dx - 1/2),
// evaluated as an exact integer plus a small FP32 remainder so the CIC weights keep
// full FP32 precision on large meshes.
//
// Blocks are remapped so that each of the 8 XCDs (which receive blocks round-robin)
// works on one contiguous, spatially coherent slab of particles and shares its L2.
#include "internal.hpp"

namespace cola {

constexpr int kPartThreads = 256;
constexpr int kXcds = 8;

__device__ __forceinline__ long xcd_block(long nblocks_padded) {
  const long b = blockIdx.x;
  return (b % kXcds) * (nblocks_padded / kXcds) + b / kXcds;
}

struct Stencil {
  int c0[3], c1[3];
  float w1[3];
};

__device__ __forceinline__ int wrap(int c, int n) {
  c %= n;
  return c < 0 ? c + n : c;
}

__device__ __forceinline__ Stencil make_stencil(const Lattice& lat, long p, float sx, float sy, float sz) {
  const long np2 = (long)lat.np * lat.np;
  const int li[3] = {(int)(p / np2), (int)((p / lat.np) % lat.np), (int)(p % lat.np)};
  const float sd[3] = {sx, sy, sz};
  Stencil st;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float t = sd[d] * lat.inv_dx - 0.5f;
    const float ft = floorf(t);
    st.w1[d] = t - ft;
    const int c = wrap(lat.ratio * li[d] + (int)ft, lat.nm);
    st.c0[d] = c;
    st.c1[d] = (c + 1 == lat.nm) ? 0 : c + 1;
  }
  return st;
}

// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(kPartThreads) void k_fill(float4* p, long n4, float value) {
  const long i = (long)blockIdx.x * kPartThreads + threadIdx.x;
  if (i < n4) p[i] = make_float4(value, value, value, value);
}

// ---------------------------------------------------------------------------------
// Deposit: rho[c] += mass * prod_d w_d for the 8 cells of each particle.
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(kPartThreads) void k_deposit(Lattice lat, const float* __restrict__ s,
                                                          float* __restrict__ rho, float mass, long nbp) {
  const long p = xcd_block(nbp) * kPartThreads + threadIdx.x;
  if (p >= lat.npart) return;
  const float sx = s[p], sy = s[lat.npart + p], sz = s[2 * lat.npart + p];
  const Stencil st = make_stencil(lat, p, sx, sy, sz);
  const long nm = lat.nm;
  const float wx[2] = {1.f - st.w1[0], st.w1[0]};
  const float wy[2] = {1.f - st.w1[1], st.w1[1]};
  const float wz[2] = {1.f - st.w1[2], st.w1[2]};
  const int cx[2] = {st.c0[0], st.c1[0]};
  const int cy[2] = {st.c0[1], st.c1[1]};
  const int cz[2] = {st.c0[2], st.c1[2]};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const long row = ((long)cx[a] * nm + cy[b]) * nm;
      const float wab = mass * wx[a] * wy[b];
#pragma unroll
      for (int c = 0; c < 2; ++c) unsafeAtomicAdd(rho + row + cz[c], wab * wz[c]);
    }
}

// ---------------------------------------------------------------------------------
// Gather + kick (+ drift | + finish).
// ---------------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(kPartThreads) void k_gather(Lattice lat, GatherArgs g, KickArgs k, long nbp) {
  const long p = xcd_block(nbp) * kPartThreads + threadIdx.x;
  if (p >= lat.npart) return;
  const long n = lat.npart;
  float s3[3] = {g.s[p], g.s[n + p], g.s[2 * n + p]};
  const Stencil st = make_stencil(lat, p, s3[0], s3[1], s3[2]);
  const long nm = lat.nm;
  const float wx[2] = {1.f - st.w1[0], st.w1[0]};
  const float wy[2] = {1.f - st.w1[1], st.w1[1]};
  const float wz[2] = {1.f - st.w1[2], st.w1[2]};
  const int cx[2] = {st.c0[0], st.c1[0]};
  const int cy[2] = {st.c0[1], st.c1[1]};
  const int cz[2] = {st.c0[2], st.c1[2]};
  float f[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const long row = ((long)cx[a] * nm + cy[b]) * nm;
      const float wab = wx[a] * wy[b];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const long idx = row + cz[c];
        const float w = wab * wz[c];
        f[0] += w * g.g0[idx];
        f[1] += w * g.g1[idx];
        f[2] += w * g.g2[idx];
      }
    }
  if constexpr (MODE == kGatherForce) {
#pragma unroll
    for (int d = 0; d < 3; ++d) g.out_a[d * n + p] = f[d];
    return;
  } else {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float a1 = g.s1[d * n + p];
      const float a2 = g.s2[d * n + p];
      float v = g.v[d * n + p];
      v += k.alpha * (f[d] - k.t2d1 * a1 - k.t2d2 * a2);
      if constexpr (MODE == kGatherKickDrift) {
        g.v[d * n + p] = v;
        g.s[d * n + p] = s3[d] + k.beta * v + k.dd1 * a1 + k.dd2 * a2;
      } else {
        g.v[d * n + p] = v;
        g.out_b[d * n + p] = v + k.td1 * a1 + k.td2 * a2;
        const long li = (d == 0) ? p / ((long)lat.np * lat.np) : (d == 1) ? (p / lat.np) % lat.np : p % lat.np;
        float x = (float)li * (k.box / (float)lat.np) + s3[d];
        x = x - k.box * floorf(x / k.box);
        if (x >= k.box) x -= k.box;
        g.out_a[d * n + p] = x;
      }
    }
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
static long padded_blocks(long npart) {
  long nb = (npart + kPartThreads - 1) / kPartThreads;
  return (nb + kXcds - 1) / kXcds * kXcds;
}

hipError_t launch_fill(float* p, long n, float value, hipStream_t st) {
  if (n % 4) return hipErrorInvalidValue;
  const long n4 = n / 4;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n4 + kPartThreads - 1) / kPartThreads)), dim3(kPartThreads), 0, st,
                     reinterpret_cast<float4*>(p), n4, value);
  return hipGetLastError();
}

hipError_t launch_deposit(Lattice lat, const float* s, float* rho, float mass, hipStream_t st) {
  const long nb = padded_blocks(lat.npart);
  hipLaunchKernelGGL(k_deposit, dim3((unsigned)nb), dim3(kPartThreads), 0, st, lat, s, rho, mass, nb);
  return hipGetLastError();
}

hipError_t launch_gather(Lattice lat, int mode, GatherArgs a, KickArgs k, hipStream_t st) {
  const long nb = padded_blocks(lat.npart);
  switch (mode) {
    case kGatherForce:
      hipLaunchKernelGGL(k_gather<kGatherForce>, dim3((unsigned)nb), dim3(kPartThreads), 0, st, lat, a, k, nb);
      break;
    case kGatherKickDrift:
      hipLaunchKernelGGL(k_gather<kGatherKickDrift>, dim3((unsigned)nb), dim3(kPartThreads), 0, st, lat, a, k, nb);
      break;
    case kGatherFinish:
      hipLaunchKernelGGL(k_gather<kGatherFinish>, dim3((unsigned)nb), dim3(kPartThreads), 0, st, lat, a, k, nb);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_noise(uint64_t seed, float* w, long count, hipStream_t st) {
  const long ng = (count + 3) / 4;
  hipLaunchKernelGGL(k_noise, dim3((unsigned)((ng + kPartThreads - 1) / kPartThreads)), dim3(kPartThreads), 0, st,
                     seed, w, count);
  return hipGetLastError();
}

}  // namespace cola
