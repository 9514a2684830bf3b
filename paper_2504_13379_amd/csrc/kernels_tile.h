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
// The tile order is a permutation of the nodes that makes them so (a k-d
// tree, below).  Problems keep their own node order at the boundary; the
// fused form gathers states into the tile order at the start of a call and
// scatters them back at the end.
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

// The order is built by recursive bisection (a k-d tree): level l cuts the
// slots into 2^l segments of whole 16-slot blocks, segment s holding blocks
// [floor(s nb / 2^l), floor((s + 1) nb / 2^l)) of the nb = ceil(n / 16) blocks
// (the last one may be partial); each segment is sorted along the longest
// axis of its nodes' bounding box, so that its halves at the next level are
// the nodes below and above its median.  After the last level every segment
// is one block of 16 nodes, and blocks of 32 are two sibling leaves.  Sort
// keys: segment (18 bits) | coordinate along the axis quantised to 24 bits
// over the segment's extent | node index (22 bits), so keys are unique and the
// order is deterministic.  On the ellipsoid of 65536 nodes 75 % of the
// 32 x 16 blocks of one application are far with this order (a Morton order
// gave 69 %, a Hilbert order 72 %).
constexpr int kTileLeaf = 16;
constexpr int kTileSegBits = 18, kTileNodeBits = 22, kTileCoordBits = 24;
static_assert(kTileSegBits + kTileCoordBits + kTileNodeBits == 64, "one 64-bit key");

inline int tile_levels(int64_t n) {
  const int64_t nb = ceil_div(n, kTileLeaf);
  int L = 0;
  while ((int64_t(1) << L) < nb) ++L;
  return L;
}

// Segment of 16-slot block k at level l (nb blocks): the largest s with
// floor(s nb / 2^l) <= k.
__device__ inline int64_t tile_segment(int64_t k, int l, int64_t nb) { return (((k + 1) << l) - 1) / nb; }

// perm[s] = s for s < n (the nodes in their own order before the first level).
__global__ __launch_bounds__(kWG) void k_tile_init(int64_t n, int* __restrict__ perm) {
  const int64_t s = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (s < n) perm[s] = (int)s;
}

// box[6 seg + 0..2] = min, [6 seg + 3..5] = max of the FP32 coordinates of the
// nodes in segment `seg` (one workgroup per segment) at level l.
__global__ __launch_bounds__(kWG) void k_tile_seg_box(const float4* __restrict__ src, const int* __restrict__ perm,
                                                      int64_t n, int l, double* __restrict__ box) {
  __shared__ double red[6][kWG];
  const int64_t nb = ceil_div(n, kTileLeaf);
  const int64_t seg = blockIdx.x;
  const int64_t s0 = ((seg * nb) >> l) * kTileLeaf;
  int64_t s1 = (((seg + 1) * nb) >> l) * kTileLeaf;
  if (s1 > n) s1 = n;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t s = s0 + threadIdx.x; s < s1; s += kWG) {
    const float4 p = src[perm[s]];
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
  for (int h = kWG / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        red[d][threadIdx.x] = fmin(red[d][threadIdx.x], red[d][threadIdx.x + h]);
        red[3 + d][threadIdx.x] = fmax(red[3 + d][threadIdx.x], red[3 + d][threadIdx.x + h]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) box[6 * seg + threadIdx.x] = red[threadIdx.x][0];
}

// Sort keys of level l for the np2 slots (all-ones beyond n).
__global__ __launch_bounds__(kWG) void k_tile_seg_keys(const float4* __restrict__ src, const int* __restrict__ perm,
                                                       int64_t n, int64_t np2, int l, const double* __restrict__ box,
                                                       uint64_t* __restrict__ keys) {
  const int64_t s = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (s >= np2) return;
  if (s >= n) {
    keys[s] = ~0ull;
    return;
  }
  const int64_t nb = ceil_div(n, kTileLeaf);
  const int64_t seg = tile_segment(s / kTileLeaf, l, nb);
  const double* b = box + 6 * seg;
  int ax = 0;
  double ext = b[3] - b[0];
  if (b[4] - b[1] > ext) {
    ax = 1;
    ext = b[4] - b[1];
  }
  if (b[5] - b[2] > ext) {
    ax = 2;
    ext = b[5] - b[2];
  }
  const int node = perm[s];
  const float4 p = src[node];
  const double c = ax == 0 ? p.x : (ax == 1 ? p.y : p.z);
  const double qmax = (double)((1u << kTileCoordBits) - 1);
  const uint64_t q = ext > 0.0 ? (uint64_t)fmin(fmax((c - b[ax]) / ext * qmax, 0.0), qmax) : 0;
  keys[s] = ((uint64_t)seg << (kTileCoordBits + kTileNodeBits)) | (q << kTileNodeBits) | (uint64_t)node;
}

// perm[s] = node of sorted key s, for s < n.
__global__ __launch_bounds__(kWG) void k_tile_take(const uint64_t* __restrict__ keys, int64_t n, int* __restrict__ perm) {
  const int64_t s = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (s < n) perm[s] = (int)(keys[s] & ((1ull << kTileNodeBits) - 1));
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

// The slots' packed coordinates and weights (padding slots keep their index).
__global__ __launch_bounds__(kWG) void k_tile_build(int64_t n, int64_t npad, const float4* __restrict__ src,
                                                    const double* __restrict__ q, int* __restrict__ perm,
                                                    float4* __restrict__ src_t, double* __restrict__ q_t) {
  const int64_t s = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (s >= npad) return;
  int64_t i = s;
  if (s < n)
    i = perm[s];
  else
    perm[s] = (int)s;
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
