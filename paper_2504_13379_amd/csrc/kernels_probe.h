// Roofline microbenchmarks: issue rates of FP32 FMA (two- and three-operand
// encodings), exp2, sqrt and an exp2 + FMA mix; BF16 and FP32 MFMA rates,
// alone and next to independent FMAs; HBM read and copy bandwidth.  Every kernel touches only `out[gid]` (one float
// per thread) or the caller's [src, src + n) / [dst, dst + n) ranges.
#pragma once

#include "common.h"

namespace nfr {

constexpr int kProbeChains = 8;

// Eight independent FMA chains per thread, `iters` iterations each; register
// operands only (compact accumulate encoding).
__global__ __launch_bounds__(kWG) void k_probe_fma(int64_t iters, float* __restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * kWG + threadIdx.x;
  float a[kProbeChains], b[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) {
    a[c] = 1.0f + 1e-7f * (float)(threadIdx.x + c);
    b[c] = 1e-9f * (float)((threadIdx.x + 3 * c) & 7);
  }
  const float m = 1.0f - 1e-6f * (float)(threadIdx.x & 1);
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) a[c] = fmaf(b[c], m, a[c]);
  }
  float r = 0.0f;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) r += a[c];
  out[gid] = r;
}

// As k_probe_fma, but x <- x * m + b: the destination is not the addend, so
// the three-operand (VOP3) encoding is needed, which the hardware does not
// dual-issue.
__global__ __launch_bounds__(kWG) void k_probe_fma_vop3(int64_t iters, float* __restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * kWG + threadIdx.x;
  float a[kProbeChains], b[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) {
    a[c] = 1.0f + 1e-7f * (float)(threadIdx.x + c);
    b[c] = 1e-9f * (float)((threadIdx.x + 3 * c) & 7);
  }
  const float m = 1.0f - 1e-6f * (float)(threadIdx.x & 1);
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) a[c] = fmaf(a[c], m, b[c]);
  }
  float r = 0.0f;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) r += a[c];
  out[gid] = r;
}

// The pair kernels' kind of mix: per chain and iteration one exp2 and three
// accumulating FMAs (4 lane-operations); x stays in (0, 1].
__global__ __launch_bounds__(kWG) void k_probe_fma_exp(int64_t iters, float* __restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * kWG + threadIdx.x;
  float a[kProbeChains], z[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) {
    a[c] = 0.5f + 1e-3f * (float)((threadIdx.x + c) & 63);
    z[c] = 0.0f;
  }
  const float m = -1.0f + 1e-6f * (float)(threadIdx.x & 1);
  const float k = 1e-3f;
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) {
      const float e = __builtin_amdgcn_exp2f(a[c]);
      a[c] = fmaf(e, m, a[c]);
      z[c] = fmaf(e, k, z[c]);
      z[c] = fmaf(a[c], k, z[c]);
    }
  }
  float r = 0.0f;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) r += a[c] + z[c];
  out[gid] = r;
}

// Eight independent exp2 chains per thread: x <- exp2(-x) stays in (0, 1].
__global__ __launch_bounds__(kWG) void k_probe_exp(int64_t iters, float* __restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * kWG + threadIdx.x;
  float a[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) a[c] = 0.5f + 1e-3f * (float)((threadIdx.x + c) & 63);
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) a[c] = __builtin_amdgcn_exp2f(-a[c]);
  }
  float r = 0.0f;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) r += a[c];
  out[gid] = r;
}

// Eight independent sqrt chains per thread: x <- sqrt(x) + 0.5 stays in [0.5, 2].
__global__ __launch_bounds__(kWG) void k_probe_sqrt(int64_t iters, float* __restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * kWG + threadIdx.x;
  float a[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) a[c] = 1.0f + 1e-3f * (float)((threadIdx.x + c) & 63);
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) a[c] = __builtin_amdgcn_sqrtf(a[c]) + 0.5f;
  }
  float r = 0.0f;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) r += a[c];
  out[gid] = r;
}

// Reads n floats (n a multiple of 4) with a grid-stride float4 loop; one partial per thread.
__global__ __launch_bounds__(kWG) void k_probe_read(const float* __restrict__ src, int64_t n, float* __restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * kWG + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kWG;
  const f32x4* s4 = reinterpret_cast<const f32x4*>(src);
  const int64_t n4 = n / 4;
  float acc = 0.0f;
  for (int64_t i = gid; i < n4; i += stride) {
    const f32x4 v = __builtin_nontemporal_load(&s4[i]);
    acc += (v.x + v.y) + (v.z + v.w);
  }
  out[gid] = acc;
}

// Plain copy of n floats (n a multiple of 4): the reference for HBM byte counters.
__global__ __launch_bounds__(kWG) void k_probe_copy(const float* __restrict__ src, float* __restrict__ dst, int64_t n) {
  const int64_t gid = (int64_t)blockIdx.x * kWG + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kWG;
  const f32x4* s4 = reinterpret_cast<const f32x4*>(src);
  f32x4* d4 = reinterpret_cast<f32x4*>(dst);
  for (int64_t i = gid; i < n / 4; i += stride) d4[i] = s4[i];
}

typedef __attribute__((ext_vector_type(8))) __bf16 probe_bf16x8;
typedef __attribute__((ext_vector_type(16))) float probe_f32x16;

// Four independent 32x32x16 BF16 MFMA accumulation chains per wave.
__global__ __launch_bounds__(kWG) void k_probe_mfma(int64_t iters, float* __restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * kWG + threadIdx.x;
  probe_bf16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(1e-3f * (float)((threadIdx.x + e) & 7));
    b[e] = (__bf16)(1e-3f * (float)((threadIdx.x * 3 + e) & 7));
  }
  probe_f32x16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
  for (int64_t it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c3, 0, 0, 0);
  }
  float r = 0.0f;
#pragma unroll
  for (int e = 0; e < 16; ++e) r += c0[e] + c1[e] + c2[e] + c3[e];
  out[gid] = r;
}

// Four independent 32x32x2 FP32 MFMA accumulation chains per wave.
__global__ __launch_bounds__(kWG) void k_probe_mfma_f32(int64_t iters, float* __restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * kWG + threadIdx.x;
  const float a = 1e-3f * (float)(threadIdx.x & 7), b = 1e-3f * (float)((threadIdx.x * 3) & 7);
  probe_f32x16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
  for (int64_t it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c3, 0, 0, 0);
  }
  float r = 0.0f;
#pragma unroll
  for (int e = 0; e < 16; ++e) r += c0[e] + c1[e] + c2[e] + c3[e];
  out[gid] = r;
}

// Co-issue probes: per iteration two independent MFMA chains (FP32: two
// 32x32x2, 64 clocks each; BF16: four 32x32x16, 32 clocks each, so 128 clocks
// of matrix-core work either way) and eight independent FMA chains of four
// FMAs (32 wave instructions, 128 clocks at one per four clocks), no data
// shared between the two.  Their rate next to the pure probes shows whether
// the vector units run while the matrix cores do.
__global__ __launch_bounds__(kWG) void k_probe_mfma_f32_fma(int64_t iters, float* __restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * kWG + threadIdx.x;
  const float a = 1e-3f * (float)(threadIdx.x & 7), b = 1e-3f * (float)((threadIdx.x * 3) & 7);
  probe_f32x16 c0 = {}, c1 = {};
  float x[kProbeChains], y[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) {
    x[c] = 1.0f + 1e-7f * (float)(threadIdx.x + c);
    y[c] = 1e-9f * (float)((threadIdx.x + 3 * c) & 7);
  }
  const float m = 1.0f - 1e-6f * (float)(threadIdx.x & 1);
  for (int64_t it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c1, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < kProbeChains; ++c) x[c] = fmaf(y[c], m, x[c]);
  }
  float r = 0.0f;
#pragma unroll
  for (int e = 0; e < 16; ++e) r += c0[e] + c1[e];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) r += x[c];
  out[gid] = r;
}

__global__ __launch_bounds__(kWG) void k_probe_mfma_bf16_fma(int64_t iters, float* __restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * kWG + threadIdx.x;
  probe_bf16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(1e-3f * (float)((threadIdx.x + e) & 7));
    b[e] = (__bf16)(1e-3f * (float)((threadIdx.x * 3 + e) & 7));
  }
  probe_f32x16 c0 = {}, c1 = {};
  float x[kProbeChains], y[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) {
    x[c] = 1.0f + 1e-7f * (float)(threadIdx.x + c);
    y[c] = 1e-9f * (float)((threadIdx.x + 3 * c) & 7);
  }
  const float m = 1.0f - 1e-6f * (float)(threadIdx.x & 1);
  for (int64_t it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c1, 0, 0, 0);
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c1, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < kProbeChains; ++c) x[c] = fmaf(y[c], m, x[c]);
  }
  float r = 0.0f;
#pragma unroll
  for (int e = 0; e < 16; ++e) r += c0[e] + c1[e];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) r += x[c];
  out[gid] = r;
}

// The same four BF16 MFMAs per iteration beside 32 other vector instructions
// in eight independent chains: OP 0 v_dot2c_f32_bf16 (x <- x + pair . k, the
// one-instruction remainder of a BF16 split), OP 1 a mask and a multiply-add
// (x <- x - 2^-30 (x & 0xffff0000), the shape of the shift-and-subtract
// remainder).
template <int OP>
__global__ __launch_bounds__(kWG) void k_probe_mfma_bf16_vop(int64_t iters, float* __restrict__ out) {
  typedef __attribute__((ext_vector_type(2))) __bf16 probe_bf16x2;
  const int64_t gid = (int64_t)blockIdx.x * kWG + threadIdx.x;
  probe_bf16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(1e-3f * (float)((threadIdx.x + e) & 7));
    b[e] = (__bf16)(1e-3f * (float)((threadIdx.x * 3 + e) & 7));
  }
  probe_f32x16 c0 = {}, c1 = {};
  float x[kProbeChains];
  probe_bf16x2 p[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) {
    x[c] = 1.0f + 1e-7f * (float)(threadIdx.x + c);
    p[c][0] = (__bf16)(1e-6f * (float)((threadIdx.x + c) & 7));
    p[c][1] = (__bf16)(1e-6f * (float)((threadIdx.x + 5 * c) & 7));
  }
  const probe_bf16x2 k = {(__bf16)0.5f, (__bf16)-0.25f};
  for (int64_t it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c1, 0, 0, 0);
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c1, 0, 0, 0);
    if constexpr (OP == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < kProbeChains; ++c) x[c] = __builtin_amdgcn_fdot2_f32_bf16(p[c], k, x[c], false);
    } else {
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < kProbeChains; ++c) {
          const float hi = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, x[c]) & 0xffff0000u);
          x[c] = fmaf(-0x1p-30f, hi, x[c]);
        }
    }
  }
  float r = 0.0f;
#pragma unroll
  for (int e = 0; e < 16; ++e) r += c0[e] + c1[e];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) r += x[c];
  out[gid] = r;
}

}  // namespace nfr
