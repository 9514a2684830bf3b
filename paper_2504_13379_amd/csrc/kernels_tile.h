// Tile order of a problem's nodes.
//
// The fused split kernel evaluates the normalised kernel
// u = exp2(-t) + kappa exp2(-rho t) of a Gaussian Mexican hat (rho < 1: the
// excitatory exponential is the steeper one).  Where (1 - rho) t exceeds
// 25 - log2|kappa| the first term is below half a unit in the last place of
// the second, so the FP32 sum equals the second term alone and the first
// exponential need not be evaluated.  Whether a whole block of entries lies
// in that range follows from bounding spheres of its target and source
// nodes, which is useful only when consecutive nodes are close in space.
// The tile order is a permutation of the nodes that makes them so: the
// Morton (Z-order) index of the FP32 coordinates quantised to 2^10 cells per
// axis of the bounding cube, ties by node index.  Problems keep their own
// node order at the boundary; the fused form gathers states into the tile
// order at the start of a call and scatters them back at the end.
#pragma once

#include "common.h"

namespace nfr {

constexpr int kTileRowBlock = 32;   // target rows per wave of the fused kernel
constexpr int kTileColBlock = 16;   // source columns per MFMA step of the fused kernel

inline int64_t tile_pow2(int64_t npad) {
  int64_t p = 1;
  while (p < npad) p <<= 1;
  return p;
}

// box[0..2] = min, box[3..5] = max of the n FP32 coordinates (one workgroup).
__global__ __launch_bounds__(kWG) void k_tile_box(const float4* __restrict__ src, int64_t n, double* __restrict__ box) {
  __shared__ double red[6][kWG];
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = threadIdx.x; i < n; i += kWG) {
    const float4 p = src[i];
    const double c[3] = {p.x, p.y, p.z};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], c[d]);
      hi[d] = fmax(hi[d], c[d]);
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    red[d][threadIdx.x] = lo[d];
    red[3 + d][threadIdx.x] = hi[d];
  }
  __syncthreads();
  for (int s = kWG / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        red[d][threadIdx.x] = fmin(red[d][threadIdx.x], red[d][threadIdx.x + s]);
        red[3 + d][threadIdx.x] = fmax(red[3 + d][threadIdx.x], red[3 + d][threadIdx.x + s]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) box[threadIdx.x] = red[threadIdx.x][0];
}

// 10 bits of v spread to every third bit.
__device__ inline uint32_t spread3(uint32_t v) {
  v &= 0x3ff;
  v = (v | (v << 16)) & 0x030000ff;
  v = (v | (v << 8)) & 0x0300f00f;
  v = (v | (v << 4)) & 0x030c30c3;
  v = (v | (v << 2)) & 0x09249249;
  return v;
}

// keys[i] = (Morton index << 32) | i for i < n; all-ones for n <= i < np2.
__global__ __launch_bounds__(kWG) void k_tile_keys(const float4* __restrict__ src, int64_t n, int64_t np2,
                                                   const double* __restrict__ box, uint64_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= np2) return;
  if (i >= n) {
    keys[i] = ~0ull;
    return;
  }
  const double ext = fmax(fmax(box[3] - box[0], box[4] - box[1]), fmax(box[5] - box[2], 1e-300));
  const float4 p = src[i];
  const double c[3] = {p.x, p.y, p.z};
  uint32_t q[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double f = (c[d] - box[d]) / ext * 1024.0;
    q[d] = (uint32_t)fmin(fmax(f, 0.0), 1023.0);
  }
  const uint32_t code = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
  keys[i] = ((uint64_t)code << 32) | (uint64_t)i;
}

// One compare-exchange pass (k, j) of a bitonic sort of np2 keys (ascending).
__global__ __launch_bounds__(kWG) void k_bitonic(uint64_t* __restrict__ keys, int64_t np2, int64_t k, int64_t j) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= np2) return;
  const int64_t l = i ^ j;
  if (l <= i) return;
  const uint64_t a = keys[i], b = keys[l];
  const bool up = (i & k) == 0;
  if (up ? (a > b) : (a < b)) {
    keys[i] = b;
    keys[l] = a;
  }
}

// perm[s] = node in slot s of the tile order (padding slots keep their index),
// with the slot's packed coordinates and weight.
__global__ __launch_bounds__(kWG) void k_tile_build(const uint64_t* __restrict__ keys, int64_t n, int64_t npad,
                                                    const float4* __restrict__ src, const double* __restrict__ q,
                                                    int* __restrict__ perm, float4* __restrict__ src_t,
                                                    double* __restrict__ q_t) {
  const int64_t s = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (s >= npad) return;
  const int64_t i = s < n ? (int64_t)(keys[s] & 0xffffffffull) : s;
  perm[s] = (int)i;
  src_t[s] = src[i];
  q_t[s] = q[i];
}

// Bounding sphere of each block of BS slots of the tile order: centre (mean of
// its nodes) and a radius rounded up past every node's FP32 distance from the
// FP32 centre; blocks holding no node get radius -1.
template <int BS>
__global__ __launch_bounds__(kWG) void k_tile_bounds(const float4* __restrict__ src_t, int64_t n, int64_t nblocks,
                                                     float4* __restrict__ bnd) {
  const int64_t b = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (b >= nblocks) return;
  const int64_t s0 = b * BS;
  int64_t s1 = s0 + BS;
  if (s1 > n) s1 = n;
  if (s1 <= s0) {
    bnd[b] = make_float4(0.0f, 0.0f, 0.0f, -1.0f);
    return;
  }
  double cx = 0.0, cy = 0.0, cz = 0.0;
  for (int64_t s = s0; s < s1; ++s) {
    const float4 p = src_t[s];
    cx += p.x;
    cy += p.y;
    cz += p.z;
  }
  const double inv = 1.0 / (double)(s1 - s0);
  const float fx = (float)(cx * inv), fy = (float)(cy * inv), fz = (float)(cz * inv);
  double r2 = 0.0;
  for (int64_t s = s0; s < s1; ++s) {
    const float4 p = src_t[s];
    const double dx = (double)p.x - fx, dy = (double)p.y - fy, dz = (double)p.z - fz;
    r2 = fmax(r2, dx * dx + dy * dy + dz * dz);
  }
  // relative margin covers the FP32 rounding of the centre and of the test's
  // own arithmetic
  const double r = sqrt(r2) * (1.0 + 1e-6) + 1e-6 * (1.0 + fabs((double)fx) + fabs((double)fy) + fabs((double)fz));
  bnd[b] = make_float4(fx, fy, fz, (float)r * (1.0f + 1e-6f));
}

// ut[b n + s] = u[b n + perm[s]] (states into the tile order).
__global__ __launch_bounds__(kWG) void k_tile_gather(const double* __restrict__ u, const int* __restrict__ perm,
                                                     int64_t n, int64_t total, double* __restrict__ ut) {
  const int64_t idx = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (idx >= total) return;
  const int64_t b = idx / n, s = idx - b * n;
  ut[idx] = u[b * n + perm[s]];
}

// u[b n + perm[s]] = ut[b n + s] (states back into the problem's order).
__global__ __launch_bounds__(kWG) void k_tile_scatter(const double* __restrict__ ut, const int* __restrict__ perm,
                                                      int64_t n, int64_t total, double* __restrict__ u) {
  const int64_t idx = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (idx >= total) return;
  const int64_t b = idx / n, s = idx - b * n;
  u[b * n + perm[s]] = ut[idx];
}

// Far test of the fused kernel for a target block (centre, radius) and a
// source block: every pair at distance^2 > d2far, or the source block empty.
__device__ inline bool tile_far(float4 rb, float4 cb, float d2far) {
  if (cb.w < 0.0f || rb.w < 0.0f) return true;
  const float dx = rb.x - cb.x, dy = rb.y - cb.y, dz = rb.z - cb.z;
  const float d = __builtin_amdgcn_sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx))) - rb.w - cb.w;
  return d > 0.0f && d * d > d2far;
}

// Count of (target block of kTileRowBlock, source block of kTileColBlock)
// pairs that the far test passes, over all npad / 32 x npad / 16 pairs; one
// thread per target block, counts[target block] (exact integers).
__global__ __launch_bounds__(kWG) void k_tile_far_count(const float4* __restrict__ bnd32,
                                                        const float4* __restrict__ bnd16, int64_t nrow, int64_t ncol,
                                                        float d2far, int64_t* __restrict__ counts) {
  const int64_t r = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (r >= nrow) return;
  const float4 rb = bnd32[r];
  int64_t c = 0;
  for (int64_t j = 0; j < ncol; ++j) c += tile_far(rb, bnd16[j], d2far) ? 1 : 0;
  counts[r] = c;
}

}  // namespace nfr
