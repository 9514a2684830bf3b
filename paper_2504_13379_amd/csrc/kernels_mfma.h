// Split-precision W form on the matrix cores (BF16 or FP16, hi + lo).
//
//   W_ij = w(|x_i - x_j|) q_j  (targets i, sources j; paper eq. NFODETilde),
//   W' = 2^sW W = Whi + 2^-c Wlo,   G = f(U) = Ghi + 2^-c Glo   (c = 0 BF16, 11 FP16),
//   Y = 2^-sW [ Whi Ghi + 2^-c (Whi Glo + Wlo Ghi) ]     (the lo*lo product is dropped).
//
// The two FP32 accumulators (main, correction) are kept apart and only combined
// in the epilogue.  sW lifts W into FP16's normal range (0 for BF16), and the
// FP16 remainders are lifted by 2^c for the same reason; BF16 has FP32's
// exponent range, so its remainders need no lift (c = 0).
//
// Buffers: W = [header 256 B | tiles]: Whi and Wlo, each npad x npad (rows =
// targets, zero beyond n), cut into 32 x 16 tiles, each tile 64 lanes x 8
// halves in the A-operand order of a 32x32x16 MFMA (lane m + 32 h holds row
// m, columns 8 h .. 8 h + 7).  Tile order: for row block group g (four 32-row
// blocks, the rows of one workgroup), column block kb, then hi / lo, then the
// four row blocks: tile index ((g * (npad/16) + kb) * 2 + hl) * 4 + r.  A wave
// reads one contiguous 1 KB tile per load instruction, and the four waves of
// a workgroup together read 8 KB of consecutive memory per column block, so a
// workgroup streams one contiguous region (measured: 74 % of HBM peak against
// 71 % for separate hi and lo matrices read by each wave; a column-major tile
// order that keeps all workgroups in a few dense bands was slower, 66 %).
// G = [Ghi Bp x npad | Glo Bp x npad] state-major with states padded to Bp
// (a multiple of 64) with zeros.
#pragma once

#include <utility>

#include "common.h"
#include "kernels_core.h"
#include "kernels_tile.h"

namespace nfr {

constexpr bool kMfmaAvailable = true;
#ifndef NFR_MFMA_SPLITS
#define NFR_MFMA_SPLITS 8
#endif
constexpr int kMfmaSplits = NFR_MFMA_SPLITS;   // one source chunk per XCD (workgroup id % 8 picks the XCD)
// The BF16 split-W kernel streams W in half as many, longer chunks: at
// N = 65536, B = 64 2.68 against 2.90 ms per application with 8 (2 chunks:
// 2.59 ms), and the combine reads half the partial sums.  Each chunk is
// summed in FP32 on the matrix cores, so longer chunks cost accuracy: FP16,
// the accurate split (2e-6 of the absolute sum per application), keeps 8
// (with 4 its full-size error reached 2.3e-6); the on-the-fly kernels, 1-2 %
// slower with 4, keep 8 too.
#ifndef NFR_MFMA_APPLY_SPLITS_BF16
#define NFR_MFMA_APPLY_SPLITS_BF16 4
#endif
constexpr int kMfmaRowsPerWG = 128;   // 4 waves x 32 rows
constexpr int kMfmaHeader = 256;

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8_t;
typedef __attribute__((ext_vector_type(16))) float f32x16_t;
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4_t;

template <typename T> struct MfmaTraits;
template <> struct MfmaTraits<__bf16> {
  typedef bf16x8_t vec;
  static constexpr int c = 0;
  static constexpr bool fp16 = false;
  static __device__ inline f32x16_t mma(vec a, vec b, f32x16_t acc) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
};
template <> struct MfmaTraits<_Float16> {
  typedef f16x8_t vec;
  static constexpr int c = 11;
  static constexpr bool fp16 = true;
  static __device__ inline f32x16_t mma(vec a, vec b, f32x16_t acc) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc, 0, 0, 0);
  }
};

// Forms 2 / 3: W matrix in BF16 / FP16; 4 / 5: the same products with W
// evaluated on the fly (no W matrix).
inline bool is_mfma_form(int form) { return form >= 2 && form <= 5; }
inline bool mfma_has_w(int form) { return form == 2 || form == 3; }
inline bool mfma_is_bf16(int form) { return form == 2 || form == 4; }
inline int64_t mfma_bp(int B) { return round_up(B, 64); }
inline size_t mfma_g_bytes(int64_t npad, int B) { return size_t(2) * mfma_bp(B) * npad * 2; }
// Source chunks of the split-W kernel for element type T (see above).
template <typename T>
__host__ __device__ constexpr int apply_splits() {
  return MfmaTraits<T>::fp16 ? kMfmaSplits : NFR_MFMA_APPLY_SPLITS_BF16;
}
inline int mfma_nsplit(int form) { return form == 2 ? NFR_MFMA_APPLY_SPLITS_BF16 : kMfmaSplits; }   // 2: W_BF16X3
inline size_t mfma_w_bytes(int64_t, int64_t npad) { return kMfmaHeader + size_t(2) * npad * npad * 2; }

// Round-to-nearest-even conversions of a double through float.
template <typename T> __device__ inline T to_half_type(double x) { return (T)(float)x; }

// hi/lo split of a double: hi = T(x), lo = T((x - hi) * 2^c).
template <typename T>
__device__ inline void split_hi_lo(double x, T& hi, T& lo) {
  hi = to_half_type<T>(x);
  const double r = x - (double)(float)hi;
  lo = to_half_type<T>(r * (double)(1 << MfmaTraits<T>::c));
}

// One workgroup: header[0] = sW, header[1] = 2^-sW, header[2] = 2^-(sW + c).
// FP16: sW = 14 - ceil(log2((|A_e| + |A_i|) max_j |q_j|)) puts the largest
// possible |W| just below 2^14.  BF16: sW = 0.
template <typename T>
__global__ __launch_bounds__(kWG) void k_mfma_scale(const double* __restrict__ qd, int64_t npad, double amp,
                                                    int is_fp16, float* __restrict__ header) {
  __shared__ double red[kWG];
  double m = 0.0;
  for (int64_t j = threadIdx.x; j < npad; j += kWG) m = fmax(m, fabs(qd[j]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = kWG / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int sW = 0;
    const double bound = amp * red[0];
    if (is_fp16 && bound > 0.0) sW = 14 - (int)ceil(log2(bound));
    header[0] = (float)sW;
    header[1] = (float)ldexp(1.0, -sW);
    header[2] = (float)ldexp(1.0, -(sW + MfmaTraits<T>::c));
    header[3] = 0.0f;
  }
}

// Whi/Wlo in fragment order; zero for rows i >= n or q_j = 0.  A thread
// builds the 8 entries W_i,8g .. W_i,8g+7 (one lane's share of one tile) and
// stores them as one 16-byte chunk per matrix.
// Grid: x = rows (npad), y = blocks of kWG column groups (npad / 8 groups).
template <typename T>
__global__ __launch_bounds__(kWG) void k_mfma_w_build(const double* __restrict__ xyz64, const double* __restrict__ qd,
                                                      int64_t n, int64_t npad, KernelF64 kp,
                                                      const float* __restrict__ header, T* __restrict__ Wt) {
  const int64_t i = blockIdx.x;
  const int64_t g = (int64_t)blockIdx.y * kWG + threadIdx.x;
  if (i >= npad || g >= npad / 8) return;
  const double scale = ldexp(1.0, (int)header[0]);
  T hi[8], lo[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t j = 8 * g + e;
    double wq = 0.0;
    if (i < n && qd[j] != 0.0) {
      const double r2 = pair_r2_64(kp, xyz64[3 * i] - xyz64[3 * j], xyz64[3 * i + 1] - xyz64[3 * j + 1],
                                   xyz64[3 * i + 2] - xyz64[3 * j + 2]);
      wq = kernel_w64(kp, r2) * qd[j] * scale;
    }
    split_hi_lo<T>(wq, hi[e], lo[e]);
  }
  const int64_t rb = i >> 5, m = i & 31, kb = g >> 1, h = g & 1;
  const int64_t tile_hi = (((rb >> 2) * (npad / 16) + kb) * 2) * 4 + (rb & 3);
  const int64_t off = tile_hi * 512 + (m + 32 * h) * 8;
  u32x4_t vh, vl;
  __builtin_memcpy(&vh, hi, 16);
  __builtin_memcpy(&vl, lo, 16);
  *reinterpret_cast<u32x4_t*>(Wt + off) = vh;
  *reinterpret_cast<u32x4_t*>(Wt + off + 4 * 512) = vl;
}

// 14 - ceil(log2(bound)) for FP16 (puts |x| <= bound just below 2^14), else 0;
// bound = f 2^e with f in [0.5, 1).
__device__ inline int mfma_scale_exp(double bound, bool fp16) {
  if (!fp16 || !(bound > 0.0)) return 0;
  int e;
  const double f = frexp(bound, &e);
  return 14 - (f == 0.5 ? e - 1 : e);
}

// Factor of source j in G: 1 for the W forms (q sits in W); q_j 2^sG for the
// fused forms (qd non-null), whose kernel values carry no weight, with sG from
// max |q| (FP16 only).
template <typename T>
__device__ inline double source_factor(const double* __restrict__ qd, const double* __restrict__ qmax, int64_t j) {
  if (!qd) return 1.0;
  return ldexp(qd[j], mfma_scale_exp(qmax[0], MfmaTraits<T>::fp16));
}

// Ghi/Glo[b*npad + j] from f_b(u[b*n + j]) (times source_factor) for b < Bp,
// j < npad (zero outside b < B, j < n); optionally copies u into v.
template <typename T>
__global__ __launch_bounds__(kWG) void k_mfma_prep(const double* __restrict__ u, int64_t n, int64_t npad, int B,
                                                   int64_t Bp, Firing fr, const double* __restrict__ qd,
                                                   const double* __restrict__ qmax, T* __restrict__ Ghi,
                                                   T* __restrict__ Glo, double* __restrict__ v_copy) {
  const int64_t idx = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (idx >= npad * Bp) return;
  const int b = (int)(idx / npad);
  const int64_t j = idx - (int64_t)b * npad;
  double g = 0.0;
  if (b < B && j < n) {
    const double uj = u[(int64_t)b * n + j];
    g = sigmoid(uj, fr.beta, state_theta(fr, b)) * source_factor<T>(qd, qmax, j);
    if (v_copy) v_copy[(int64_t)b * n + j] = uj;
  }
  T hi, lo;
  split_hi_lo<T>(g, hi, lo);
  Ghi[idx] = hi;
  Glo[idx] = lo;
}

// Y partials on the matrix cores.
// Workgroup w: source chunk split = w % S, row block w / S, S =
// apply_splits<T>() (kMfmaRowsPerWG rows, 32 per wave); grid.y = state
// groups of 32*NB states.
// Each wave runs over its source chunk kMfmaStep columns at a time.
//
// Operand placement: for MFMA step kb of a pipeline step, lane l = m + 32 h
// holds the 8 consecutive columns 16 kb + 8 h .. +7 of its row (A operand: W,
// read as one contiguous fragment) or of its state (B operand: G, from LDS).
// Output element r of lane l sits at row 8 (r / 4) + 4 h + r % 4 of the
// wave's 32 rows, state m of the 32-state block.
//
// Pipeline: W streams from HBM straight into registers through a ring of
// kMfmaDepth register stages (kMfmaDepth - 1 steps in flight while the matrix
// cores work on the current one); the G tile of the next step is fetched into
// registers, then stored into the other half of a double-buffered LDS tile
// that the four waves share.  32 rows per wave keep a wave under 256
// registers, so two workgroups fit on a compute unit.
#ifndef NFR_MFMA_STEP
#define NFR_MFMA_STEP 64
#endif
#ifndef NFR_MFMA_DEPTH
#define NFR_MFMA_DEPTH 3
#endif
constexpr int kMfmaStep = NFR_MFMA_STEP;         // source columns per pipeline step
constexpr int kMfmaDepth = NFR_MFMA_DEPTH;       // W register stages
constexpr int kMfmaKb = kMfmaStep / 16;          // 32x32x16 MFMA steps per pipeline step
constexpr int kMfmaLdsStride = kMfmaStep + 8;    // halves per LDS row (padding against bank conflicts)

// LDS buffers of the staged G tile: two (one step's tile written while the
// other is read).  One buffer with a second barrier per step, which helped
// the on-the-fly kernels, measured slower here: 3.01 against 2.90 ms (BF16)
// at N = 65536, B = 64.
#ifndef NFR_MFMA_APPLY_LDS_BUFS
#define NFR_MFMA_APPLY_LDS_BUFS 2
#endif
constexpr int kApplyBufs = NFR_MFMA_APPLY_LDS_BUFS;
template <typename T, int NB>
__global__ __launch_bounds__(kWG, 2) void k_mfma_apply(const T* __restrict__ Wt, const T* __restrict__ Ghi, const T* __restrict__ Glo,
                                                       int64_t npad, int B, int64_t kchunk,
                                                       const float* __restrict__ header, double* __restrict__ part) {
  typedef typename MfmaTraits<T>::vec V;
  constexpr int NS = 32 * NB;                                  // states per group
  constexpr int ROWCH = kMfmaStep / 8;                         // 16-byte chunks per LDS row
  constexpr int CHUNKS = NS * 2 * ROWCH / kWG;                 // G chunks per thread per step
  __shared__ __attribute__((aligned(16))) T sG[kApplyBufs][2][NS][kMfmaLdsStride];

  const int64_t wg = blockIdx.x;
  const int split = (int)(wg % apply_splits<T>());
  const int64_t rb = wg / apply_splits<T>();
  const int sg = blockIdx.y;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int m = lane & 31;
  const int h = lane >> 5;
  const int64_t row0 = rb * kMfmaRowsPerWG + wave * 32;
  const int64_t k_begin = (int64_t)split * kchunk;
  int64_t k_end = k_begin + kchunk;
  if (k_end > npad) k_end = npad;
  const int nsteps = (int)((k_end - k_begin) / kMfmaStep);

  const int64_t frag0 = ((rb * (npad / 16) + k_begin / 16) * 8 + wave) * 512 + (int64_t)lane * 8;
  const T* wph = Wt + frag0;
  const T* wpl = Wt + frag0 + 4 * 512;

  const T* gsrc[CHUNKS];
  int g_hl[CHUNKS], g_st[CHUNKS], g_col[CHUNKS];
#pragma unroll
  for (int q = 0; q < CHUNKS; ++q) {
    const int c = tid + kWG * q;
    const int row = c / ROWCH;
    g_hl[q] = row / NS;
    g_st[q] = row % NS;
    g_col[q] = 8 * (c % ROWCH);
    gsrc[q] = (g_hl[q] ? Glo : Ghi) + ((int64_t)sg * NS + g_st[q]) * npad + k_begin + g_col[q];
  }

  f32x16_t accM[NB], accC[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int r = 0; r < 16; ++r) accM[nb][r] = accC[nb][r] = 0.0f;

  struct WSet {
    V hi[kMfmaKb], lo[kMfmaKb];
  };
  // Loads past the last step re-read the last step (their data is never used):
  // no branches around loads, so the compiler's load counters stay exact and
  // the W prefetch is not drained at every step.
  auto load_w = [&](WSet& w, int t) {
    const int64_t base = (int64_t)(t < nsteps ? t : nsteps - 1) * kMfmaKb * 8 * 512;
#pragma unroll
    for (int kb = 0; kb < kMfmaKb; ++kb) {
      const int64_t off = base + kb * 8 * 512;
      w.hi[kb] = __builtin_bit_cast(V, __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(wph + off)));
      w.lo[kb] = __builtin_bit_cast(V, __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(wpl + off)));
    }
  };
  u32x4_t gn[CHUNKS];
  auto load_g = [&](int t) {
    const int64_t tc = t < nsteps ? t : nsteps - 1;
#pragma unroll
    for (int q = 0; q < CHUNKS; ++q) gn[q] = *reinterpret_cast<const u32x4_t*>(gsrc[q] + tc * kMfmaStep);
  };
  auto store_g = [&](int t) {
#pragma unroll
    for (int q = 0; q < CHUNKS; ++q) *reinterpret_cast<u32x4_t*>(&sG[t % kApplyBufs][g_hl[q]][g_st[q]][g_col[q]]) = gn[q];
  };
  auto compute = [&](const WSet& w, int t) {
    const int buf = t % kApplyBufs;
#pragma unroll
    for (int kb = 0; kb < kMfmaKb; ++kb) {
      const int col = 16 * kb + 8 * h;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const V bh = *reinterpret_cast<const V*>(&sG[buf][0][nb * 32 + m][col]);
        const V bl = *reinterpret_cast<const V*>(&sG[buf][1][nb * 32 + m][col]);
        accM[nb] = MfmaTraits<T>::mma(w.hi[kb], bh, accM[nb]);
        accC[nb] = MfmaTraits<T>::mma(w.hi[kb], bl, accC[nb]);
        accC[nb] = MfmaTraits<T>::mma(w.lo[kb], bh, accC[nb]);
      }
    }
  };
  // step t (ring slot t mod kMfmaDepth): issue the G loads of t + 1, then the
  // W loads of step t + kMfmaDepth - 1, compute t from LDS half t % kApplyBufs, store
  // G of t + 1 into the other half, barrier.  The G loads go first: loads
  // complete in issue order, so waiting for G does not wait for the W
  // prefetch, which stays in flight across the barrier.
  WSet ring[kMfmaDepth];
  if (nsteps > 0) {
#pragma unroll
    for (int d = 0; d + 1 < kMfmaDepth; ++d) load_w(ring[d], d);
    load_g(0);
    store_g(0);
    __syncthreads();
    int t0 = 0;
    for (; t0 + kMfmaDepth <= nsteps; t0 += kMfmaDepth) {
#pragma unroll
      for (int d = 0; d < kMfmaDepth; ++d) {
        const int t = t0 + d;
        load_g(t + 1);
        load_w(ring[(d + kMfmaDepth - 1) % kMfmaDepth], t + kMfmaDepth - 1);
        compute(ring[d], t);
        if (kApplyBufs == 1) __syncthreads();
        store_g(t + 1);
        __syncthreads();
      }
    }
#pragma unroll
    for (int d = 0; d < kMfmaDepth; ++d) {   // the last nsteps mod kMfmaDepth steps
      const int t = t0 + d;
      if (t < nsteps) {
        load_g(t + 1);
        load_w(ring[(d + kMfmaDepth - 1) % kMfmaDepth], t + kMfmaDepth - 1);
        compute(ring[d], t);
        if (kApplyBufs == 1) __syncthreads();
        store_g(t + 1);
        __syncthreads();
      }
    }
  }

  const double sm = header[1];
  const double sc = header[2];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int b = sg * NS + nb * 32 + m;
    if (b >= B) continue;
    double* dst = part + ((int64_t)split * B + b) * npad;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t i = row0 + 8 * (r / 4) + 4 * h + (r % 4);
      dst[i] = (double)accM[nb][r] * sm + (double)accC[nb][r] * sc;
    }
  }
}

// Fused on-the-fly split form: the same product on the matrix cores, but
// every W tile is evaluated by the vector units straight into the A-operand
// layout, so no W matrix exists and nothing but G and the coordinates is read.
//
// The weights move into G (G_bj = q_j 2^sG f_b(u_bj), see source_factor), so
// the tile entries are the bare radial kernel normalised by its excitatory
// amplitude (pair_u: u = exp2(-t) + kappa exp2(-rho t)), and amp 2^-sG is
// applied in the epilogue.  This keeps the evaluation at 3 subtractions, 3
// multiply-adds for r^2 (plus the square root of the exponential kernel),
// 1 multiply for rho t, 2 exp2 (or one exp2 and 1-3 multiplies for a length
// ratio 1/m) and 1 multiply-add per entry.
// Lane l = m + 32 h evaluates, for MFMA step kb, the 8 entries of row m and
// columns 16 kb + 8 h .. +7 in FP32 and splits each into hi + 2^-c lo; each
// entry serves all 32 NB states of the workgroup (3 NB products per 8
// entries; BF16 keeps the main and correction products in one accumulator,
// as its remainders are not lifted).  The column coordinates of a pipeline
// step sit in a double-buffered LDS tile read by broadcast (the 32 lanes of
// a half-wave read the same address).  Within a step the entries of MFMA
// step kb + 1 are evaluated before the products of step kb are issued, so
// the vector units work while the matrix cores run.
struct MfmaOtfParams {
  float sig, rho, per;
  float kappa;         // -A_i / A_e (PairParams)
  double amp;          // A_e
  const double* qmax;  // [0] max_j |q_j| (FP16 source lift sG), [1] max_j |x_j|^2 (norm expansion)
  // far blocks (BF16, norm expansion, nodes in the tile order of
  // kernels_tile.h): bounding spheres of the 32-row and 16-column blocks and
  // the squared distance beyond which the steep exponential drops out of the
  // FP32 sum; bnd16 null: every block takes both exponentials
  const float4* bnd32;
  const float4* bnd16;
  float d2far;
};

#ifndef NFR_MFMA_OTF_MIN_WGS
#define NFR_MFMA_OTF_MIN_WGS 2
#endif
// BF16: four workgroups per compute unit (128 registers, 4 waves per SIMD);
// with t from the matrix cores the compiler would take 148 registers (3 waves)
// and the kernel ran 1.5 % slower (1.788 against 1.762 ms per application at
// N = 65536, B = 64); at 128 it spills a few values held across the loop only.
#ifndef NFR_MFMA_OTF_BF16_MIN_WGS
#define NFR_MFMA_OTF_BF16_MIN_WGS 4
#endif
// BF16 far form in eight-wave workgroups whose wave pairs take turns on the
// vector units and the matrix cores (the ping-pong loop in k_mfma_otf): 1.676
// -> 1.659 ms per application at N = 65536, B = 64, measured alternately.  The
// second launch-bounds argument is a minimum of waves per SIMD: 4 keeps the
// eight-wave kernel at 128 registers, two workgroups per compute unit.
#ifndef NFR_MFMA_OTF_PINGPONG
#define NFR_MFMA_OTF_PINGPONG 1
#endif
constexpr bool kMfmaOtfPingPong = NFR_MFMA_OTF_PINGPONG;
// LDS buffers of the staged G tile.  FP16 keeps two (one step's tile is
// written while the other is read; one barrier per step).  BF16 uses one
// (a second barrier per step) and halves its LDS: 2.29 -> 2.22-2.24 ms per
// application at N = 65536, B = 64, the same 114 registers and 4 waves per
// SIMD; FP16, whose two accumulator sets need 152 registers, gained nothing.
#ifndef NFR_MFMA_OTF_BF16_LDS_BUFS
#define NFR_MFMA_OTF_BF16_LDS_BUFS 1
#endif
#ifndef NFR_MFMA_OTF_FP16_LDS_BUFS
#define NFR_MFMA_OTF_FP16_LDS_BUFS 2
#endif
// Gaussian kernels on non-periodic surfaces (BF16) evaluate t = sig^2 r^2 by
// the norm expansion sig^2 (|x_i|^2 + |x_j|^2 - 2 x_i . x_j): three
// multiply-adds against staged column values (-2 sig^2 x_j, sig^2 |x_j|^2),
// the row's sig^2 |x_i|^2 folded into a row factor, instead of three
// subtractions and three multiply-adds (13 -> 10 vector instructions per
// entry).  Its
// partial sums reach sig^2 (|x_i| + |x_j|)^2, so its rounding error in t is
// absolute, a few units in the last place of that size rather than of t:
// the expansion is taken only while sig^2 max_j |x_j|^2 <= kNormMaxT (for
// the steeper of the kernel's two exponentials).  There,
// for the entries that matter (t up to a few tens), the column values' and
// norms' roundings (at most 1.1e-5 and 1.1e-5 in t) and the three
// multiply-adds' (partial sums near sig^2 |x|^2: 1.1e-5) keep t within 4e-5,
// i.e. an entry within 3e-5 of itself; larger coordinates (relative to the
// kernel's width) take the differences.
#ifndef NFR_MFMA_OTF_NORM
#define NFR_MFMA_OTF_NORM 1
#endif
// BF16 remainders by a dot-product instruction (see the split in k_mfma_otf).
#ifndef NFR_MFMA_OTF_DOT2
#define NFR_MFMA_OTF_DOT2 1
#endif
constexpr double kNormMaxT = 96.0;
// Column values of the norm expansion reach each lane by a DPP row broadcast
// fused into the multiply-add (row_newbcast: every lane of a 16-lane row reads
// lane 16 r + E of the operand) instead of an LDS read per entry: each wave
// holds a step's column values in 8 registers (per pair of MFMA steps and
// coordinate), loaded by 8 four-byte LDS reads per step, against 32 128-bit
// LDS reads before, which kept the LDS at 80 % of its 128 B/clock.
#ifndef NFR_MFMA_OTF_DPP
#define NFR_MFMA_OTF_DPP 1
#endif
// Norm expansion with t from the FP32 matrix cores: per 32 columns two
// 32x32x2 FP32 MFMAs take the four products of every entry off the vector
// units (which then only evaluate the exponentials and split): 1.85 -> 1.76 ms
// per application at N = 65536, B = 64 (same GPU session), against the
// broadcast multiply-adds below.
#ifndef NFR_MFMA_OTF_TMMA
#define NFR_MFMA_OTF_TMMA 1
#endif

template <int... I, typename F>
__device__ __forceinline__ void static_for_impl(std::integer_sequence<int, I...>, F&& f) {
  (f(std::integral_constant<int, I>{}), ...);
}
// f(std::integral_constant<int, i>) for i = 0 .. N - 1, in order.
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(std::make_integer_sequence<int, N>{}, f);
}

// Lane 16 r + E of v, in every lane of row r.
template <int E>
__device__ __forceinline__ float row_bcast(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x150 + E, 0xf, 0xf, true));
}
// acc += row_bcast<E>(v) * x in one instruction (the broadcast is the DPP
// source operand of the multiply-add; v is written by LDS loads only).
template <int E>
__device__ __forceinline__ void fmac_row_bcast(float& acc, float v, float x) {
  asm volatile("v_fmac_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf bound_ctrl:1"
      : "+v"(acc)
      : "v"(v), "v"(x), "n"(E));
}
template <typename T, int KIND, int NB, int WAVES = 4>
__global__ __launch_bounds__(64 * WAVES, WAVES == 8 ? 4 : (MfmaTraits<T>::fp16 ? NFR_MFMA_OTF_MIN_WGS : NFR_MFMA_OTF_BF16_MIN_WGS)) void k_mfma_otf(const float4* __restrict__ src, const T* __restrict__ Ghi,
                                                     const T* __restrict__ Glo, int64_t npad, int B, int64_t kchunk,
                                                     MfmaOtfParams op, float* __restrict__ part) {
  typedef typename MfmaTraits<T>::vec V;
  constexpr int c = MfmaTraits<T>::c;
  constexpr bool kTwoAcc = MfmaTraits<T>::fp16;
  constexpr int NS = 32 * NB;
  constexpr int ROWCH = kMfmaStep / 8;
  // WAVES = 8 (BF16, far form): 256 rows per workgroup, waves w and w + 4 on
  // one SIMD taking turns on the vector units and the matrix cores (see the
  // ping-pong loop below); the G tile, double-buffered, serves all eight
  static_assert(WAVES == 4 || (WAVES == 8 && !MfmaTraits<T>::fp16), "eight waves: BF16 only");
  constexpr bool kPP = WAVES == 8;
  constexpr int kThreads = 64 * WAVES;
  constexpr int CHUNKS = NS * 2 * ROWCH / kThreads;
  constexpr int kOtfBufs = kPP ? 2 : (kTwoAcc ? NFR_MFMA_OTF_FP16_LDS_BUFS : NFR_MFMA_OTF_BF16_LDS_BUFS);
  constexpr bool kNormCapable = (KIND & 3) == 0 && !kTwoAcc && NFR_MFMA_OTF_NORM;
  __shared__ __attribute__((aligned(16))) T sG[kOtfBufs][2][NS][kMfmaLdsStride];
  // column values: rows 0-2 the coordinates scaled by sig (norm expansion:
  // by -2 sig^2), row 3 unused (norm expansion: sig^2 |x_j|^2); wave w loads
  // and stores row w, so no load sits behind a branch
  __shared__ __attribute__((aligned(16))) float sS[kOtfBufs][4][kMfmaStep];
  // norm expansion: row factors of the wave's 32 rows, applied in the epilogue
  __shared__ double sR[WAVES][32];
  static_assert(kWG == 4 * 64, "one wave per coordinate row");

  const int64_t wg = blockIdx.x;
  const int split = (int)(wg % kMfmaSplits);
  const int64_t rb = wg / kMfmaSplits;
  const int sg = blockIdx.y;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int m = lane & 31;
  const int h = lane >> 5;
  const int64_t row0 = rb * (32 * WAVES) + wave * 32;
  const int64_t k_begin = (int64_t)split * kchunk;
  int64_t k_end = k_begin + kchunk;
  if (k_end > npad) k_end = npad;
  const int nsteps = (int)((k_end - k_begin) / kMfmaStep);

  // (-1, 0) and (0, -1) as packed BF16 pairs (low half first), in scalar registers
  int m10i = 0, m01i = 0;
  if constexpr (!kTwoAcc && NFR_MFMA_OTF_DOT2) {
    asm volatile("s_mov_b32 %0, 0xbf80" : "=s"(m10i));
    asm volatile("s_mov_b32 %0, 0xbf800000" : "=s"(m01i));
  }
  // FP16 entries are lifted by 2^sU so that |u| <= 1 + |kappa| sits below 2^14.
  const int sU = mfma_scale_exp(1.0 + fabs((double)op.kappa), kTwoAcc);
  const float lift = (float)ldexp(1.0, sU);
  const float4 pr = src[row0 + m];
  const double s2d = (double)op.sig * op.sig;

  const T* gsrc[CHUNKS];
  int g_hl[CHUNKS], g_st[CHUNKS], g_col[CHUNKS];
#pragma unroll
  for (int q = 0; q < CHUNKS; ++q) {
    const int cc = tid + kThreads * q;
    const int row = cc / ROWCH;
    g_hl[q] = row / NS;
    g_st[q] = row % NS;
    g_col[q] = 8 * (cc % ROWCH);
    gsrc[q] = (g_hl[q] ? Glo : Ghi) + ((int64_t)sg * NS + g_st[q]) * npad + k_begin + g_col[q];
  }

  f32x16_t accM[NB], accC[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int r = 0; r < 16; ++r) accM[nb][r] = accC[nb][r] = 0.0f;

  // Wave w loads component w of the column coordinates of a step (lane =
  // column).  Loads past the last step re-read the last step.
  u32x4_t gn[CHUNKS];
  float sn;
  auto load_next = [&](int t) {
    const int64_t tc = t < nsteps ? t : nsteps - 1;
#pragma unroll
    for (int q = 0; q < CHUNKS; ++q) gn[q] = *reinterpret_cast<const u32x4_t*>(gsrc[q] + tc * kMfmaStep);
    sn = reinterpret_cast<const float*>(src + k_begin + tc * kMfmaStep + lane)[wave & 3];
  };
  auto mma = [&](int buf, int kb, const V& whi, const V& wlo) {
    const int col = 16 * kb + 8 * h;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const V bh = *reinterpret_cast<const V*>(&sG[buf][0][nb * 32 + m][col]);
      const V bl = *reinterpret_cast<const V*>(&sG[buf][1][nb * 32 + m][col]);
      accM[nb] = MfmaTraits<T>::mma(whi, bh, accM[nb]);
      if (kTwoAcc) {
        accC[nb] = MfmaTraits<T>::mma(whi, bl, accC[nb]);
        accC[nb] = MfmaTraits<T>::mma(wlo, bh, accC[nb]);
      } else {
        accM[nb] = MfmaTraits<T>::mma(whi, bl, accM[nb]);
        accM[nb] = MfmaTraits<T>::mma(wlo, bh, accM[nb]);
      }
    }
  };
  // The whole pipeline for one way of evaluating t (kNorm: norm expansion;
  // kFar: blocks of entries far apart skip the steep exponential).
  auto run = [&](auto norm_tag, auto far_tag) {
    constexpr bool kNorm = decltype(norm_tag)::value;
    constexpr bool kFar = decltype(far_tag)::value;
    static_assert(!kFar || (kNorm && sym_pow<KIND>() == 0), "far blocks need the norm expansion and two exponentials");
    static_assert(!kFar || kMfmaKb == 4, "far masks hold 4 MFMA steps per pipeline step");
    const float xi = kNorm ? pr.x : pr.x * op.sig, yi = kNorm ? pr.y : pr.y * op.sig,
                zi = kNorm ? pr.z : pr.z * op.sig;
    // norm expansion: the row's sig^2 |x_i|^2 and the column values rounded
    // once from FP64 (wave-uniform scale: -2 sig^2 for rows 0-2, sig^2 for 3)
    // norm expansion: t = n_i + a with n_i = sig^2 |x_i|^2 and a the sum of the
    // three multiply-adds.  The row's n_i is folded into a row factor: with
    // e = exp2(-t) = 2^-n_i exp2(-a), u = R_i u'(a), where u' is u with kappa
    // replaced by kappa_i (R_i = 2^-n_i, kappa_i = kappa 2^((1 - rho) n_i);
    // length ratio 1/m: R_i = 2^-m n_i, kappa_i = kappa 2^((m - 1) n_i)), so
    // an entry needs no add for n_i.  u' stays below (1 + |kappa|) 2^96 (the
    // bound on the steeper exponent's n_i), inside FP32 and BF16 range.
    const double ni = s2d * ((double)pr.x * pr.x + (double)pr.y * pr.y + (double)pr.z * pr.z);
    float kap = op.kappa;
    if constexpr (kFar) {
      // u = R_i kappa_i (e1' / kappa_i + e2'): the row factor R_i kappa_i =
      // kappa 2^(-rho n_i) goes to the epilogue, kap = 1 / kappa_i multiplies
      // e1' (so an entry of a far block is e2' alone)
      kap = (float)(exp2(-(1.0 - (double)op.rho) * ni) / (double)op.kappa);
      if (h == 0) sR[wave][m] = (double)op.kappa * exp2(-(double)op.rho * ni);
    } else if (kNorm) {
      constexpr int M = sym_pow<KIND>();
      kap = (float)((double)op.kappa * (M ? exp2((M - 1) * ni) : exp2((1.0 - (double)op.rho) * ni)));
      if (h == 0) sR[wave][m] = M ? exp2(-M * ni) : exp2(-ni);
    }
    // far blocks: bit 4 (t % 16) + kb of fmask is set when the wave's 32 rows
    // and the 16 columns of MFMA step kb of pipeline step t are far apart;
    // lane l tests column block 64 g + l of the chunk for the group g = t / 16
    // of 16 pipeline steps.  The row block's bounds sit in scalar registers
    // (wave-uniform address) and a group's column bounds are live only while
    // its mask is made, so the far path adds no vector registers to the loop.
    uint64_t fmask = 0;
    float4 rbnd = make_float4(0.0f, 0.0f, 0.0f, -1.0f);
    if constexpr (kFar) {
      const int64_t rblk = (int64_t)__builtin_amdgcn_readfirstlane((int)(row0 / kTileRowBlock));
      rbnd = op.bnd32[rblk];
    }
    auto make_mask = [&](int g) {
      const int64_t cb = k_begin / kTileColBlock + 64 * (int64_t)g + lane, cend = k_end / kTileColBlock;
      const bool ok = cb < cend;
      const float4 bn = op.bnd16[ok ? cb : cend - 1];
      fmask = __ballot(ok && tile_far(rbnd, bn, op.d2far));
    };
    // t from the matrix cores (below); in the far form the column values carry
    // rho, so that the matrix product is rho a, the broad exponential's argument
    constexpr bool kTmma = kNorm && NFR_MFMA_OTF_TMMA;
    constexpr bool kFarT = kFar && kTmma && !kTwoAcc && c == 0;
    const double wsd = ((wave & 3) < 3 ? -2.0 * s2d : s2d) * (kFarT ? (double)op.rho : 1.0);
    const float irho = kFarT ? (float)(1.0 / (double)op.rho) : 0.0f;
    auto store_next = [&](int t) {
      const int buf = t % kOtfBufs;
#pragma unroll
      for (int q = 0; q < CHUNKS; ++q) *reinterpret_cast<u32x4_t*>(&sG[buf][g_hl[q]][g_st[q]][g_col[q]]) = gn[q];
      if (wave < 4) sS[buf][wave][lane] = kNorm ? (float)((double)sn * wsd) : sn * op.sig;
    };
    // norm expansion with broadcasts: X[p][r] holds coordinate row r of the
    // step's columns for MFMA steps 2p and 2p + 1, lane 16 R + 8 s + e holding
    // column 16 (2p + s) + 8 (R / 2) + e (R = row of 16 lanes, h = R / 2), so
    // that row_newbcast:(8 s + e) hands lane m + 32 h the column 16 kb + 8 h + e
    // of MFMA step kb = 2p + s (the A operand's column of its entry e)
    constexpr bool kDpp = kNorm && !kTmma && NFR_MFMA_OTF_DPP;
    static_assert(kMfmaKb % 2 == 0, "column registers hold MFMA steps in pairs");
    // t by matrix cores: for the 32 columns of MFMA steps 2p and 2p + 1, the
    // product of the columns' (-2 sig^2 x, -2 sig^2 y, -2 sig^2 z, sig^2 |x|^2)
    // (A operand, 32 x 4) and the rows' (x, y, z, 1) (B operand, 4 x 32) is
    // the transposed block of t - n_i: lane m + 32 h holds row m and output
    // rows 8 (v / 4) + 4 h + v % 4.  Lane j reads column j with bits 2 and 3
    // swapped, so output v = 8 s + e of lane m + 32 h is column 16 s + 8 h + e:
    // entry e of MFMA step 2p + s in the layout of the split's A operand.
    // Both blocks of a pipeline step are multiplied at its start (TT[p]).
    const float tb0 = h ? yi : xi, tb1 = h ? 1.0f : zi;
    const int tcol = (m & 0x13) | ((m & 4) << 1) | ((m & 8) >> 1);
    f32x16_t TT[kMfmaKb / 2];
    auto tmma = [&](int buf, int p) {
      const float a0 = sS[buf][h][32 * p + tcol], a1 = sS[buf][2 + h][32 * p + tcol];
      const f32x16_t zero = {};
      TT[p] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, tb0, zero, 0, 0, 0);
      TT[p] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, tb1, TT[p], 0, 0, 0);
    };
    float X[kMfmaKb / 2][4];
    const int jl = 16 * ((lane & 15) >> 3) + 8 * (lane >> 5) + (lane & 7);
    auto load_cols = [&](int buf) {
#pragma unroll
      for (int p = 0; p < kMfmaKb / 2; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) X[p][r] = sS[buf][r][32 * p + jl];
    };
    int tstep = 0;
    // split pairwise: one conversion instruction rounds two entries
    auto split = [&](const float (&w)[8], V& whi, V& wlo, auto dot2_tag) {
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        typedef __attribute__((ext_vector_type(2))) float f2_t;
        typedef __attribute__((ext_vector_type(2))) T h2_t;
        const f2_t wv = {w[e], w[e + 1]};
        const h2_t hv = __builtin_convertvector(wv, h2_t);
        f2_t rv;
        if constexpr (decltype(dot2_tag)::value) {
          // remainders w - hi in one instruction per entry: the packed pair's
          // dot product with (-1, 0) or (0, -1), plus w (exact: the BF16
          // products are exact in FP32 and w - hi is representable).  The
          // constant pairs come from registers: as an inline constant the
          // compiler encodes (-1, 0) as -1.0, which this instruction reads as
          // the FP32 pattern, i.e. the pair (0, -1) (checked on the device)
          rv[0] = __builtin_amdgcn_fdot2_f32_bf16(hv, __builtin_bit_cast(h2_t, m10i), w[e], false);
          rv[1] = __builtin_amdgcn_fdot2_f32_bf16(hv, __builtin_bit_cast(h2_t, m01i), w[e + 1], false);
        } else {
          const f2_t hf = __builtin_convertvector(hv, f2_t);
          rv = wv - hf;
        }
        if (c) rv *= (float)(1 << c);
        const h2_t lv = __builtin_convertvector(rv, h2_t);
        whi[e] = hv[0];
        whi[e + 1] = hv[1];
        wlo[e] = lv[0];
        wlo[e + 1] = lv[1];
      }
    };
    auto eval = [&](int buf, auto kbc, V& whi, V& wlo) {
      constexpr int kb = decltype(kbc)::value;
      const int col = 16 * kb + 8 * h;
      float w[8];
      float tb[8];
      if constexpr (kTmma) {
        static_for<8>([&](auto ec) { tb[ec] = TT[kb / 2][8 * (kb % 2) + decltype(ec)::value]; });
      } else if constexpr (kDpp) {
        // the same fused multiply-adds in the same order as from LDS, the 8
        // entries interleaved (a broadcast multiply-add must not read an
        // accumulator written by the instruction just before it)
        constexpr int p = kb / 2, E0 = 8 * (kb % 2);
        static_for<8>([&](auto ec) { tb[ec] = row_bcast<E0 + decltype(ec)::value>(X[p][3]); });
        static_for<8>([&](auto ec) { fmac_row_bcast<E0 + decltype(ec)::value>(tb[ec], X[p][2], zi); });
        static_for<8>([&](auto ec) { fmac_row_bcast<E0 + decltype(ec)::value>(tb[ec], X[p][1], yi); });
        static_for<8>([&](auto ec) { fmac_row_bcast<E0 + decltype(ec)::value>(tb[ec], X[p][0], xi); });
      } else if constexpr (kNorm) {
        static_for<8>([&](auto ec) {
          constexpr int e = decltype(ec)::value;
          tb[e] = fmaf(xi, sS[buf][0][col + e], fmaf(yi, sS[buf][1][col + e], fmaf(zi, sS[buf][2][col + e], sS[buf][3][col + e])));
        });
      }
      // far blocks are decided per 16-column block; deciding per pipeline step
      // instead (two branch-free variants of the interleaved schedule) needed 160
      // registers and measured 2.00 against 1.87 ms at N = 65536, B = 64
      bool far = false;
      if constexpr (kFar) far = (fmask >> (4 * (tstep & 15) + kb)) & 1;
      if (far) {
        // (1 - rho) t beyond 27 - log2|kappa| in every entry: the steep term is
        // below half an ulp of the broad one, whose value the sum takes
        static_for<8>([&](auto ec) { w[ec] = __builtin_amdgcn_exp2f(-(tb[ec] * op.rho)); });
      } else static_for<8>([&](auto ec) {
        constexpr int e = decltype(ec)::value;
        float tt;
        if constexpr (kNorm) {
          tt = tb[e];
        } else {
          const float r2 = pair_r2<KIND>(xi - sS[buf][0][col + e], yi - sS[buf][1][col + e],
                                         zi - sS[buf][2][col + e], op.per);
          tt = ((KIND & 1) == 0) ? r2 : __builtin_amdgcn_sqrtf(r2);
        }
        if constexpr (kFar)
          w[e] = fmaf(kap, __builtin_amdgcn_exp2f(-tt), __builtin_amdgcn_exp2f(-(tt * op.rho)));
        else
          w[e] = pair_u<KIND>(tt, op.rho, kap);
        if (kTwoAcc) w[e] *= lift;
      });
      split(w, whi, wlo, std::bool_constant<!kTwoAcc && NFR_MFMA_OTF_DOT2>{});
    };
    // far form with t from the matrix cores (TT = rho a): every entry's broad
    // exponential (pre) is split from the near blocks' steep term and the
    // split (fin), so that the products of MFMA step kb share a basic block
    // with the broad exponentials of step kb + 1.  The remainders take a
    // shift and a subtraction instead of the dot-product instruction, which
    // does not run beside the matrix cores (a probe: 24 of them took their
    // full time on top of 6 MFMAs, where conversions, shifts and FP32 adds or
    // multiply-adds were 93-100 % hidden): 1.74 -> 1.72 ms per application.
    auto pre = [&](auto kbc, float (&w)[8]) {
      constexpr int kb = decltype(kbc)::value;
      static_for<8>([&](auto ec) { w[ec] = __builtin_amdgcn_exp2f(-TT[kb / 2][8 * (kb % 2) + decltype(ec)::value]); });
    };
    auto fin = [&](auto kbc, float (&w)[8], V& whi, V& wlo) {
      constexpr int kb = decltype(kbc)::value;
      // (1 - rho) t beyond 27 - log2|kappa| in every entry of a far block: the
      // steep term is below half an ulp of the broad one, whose value the sum takes
      const bool far = (fmask >> (4 * (tstep & 15) + kb)) & 1;
      if (!far)
        static_for<8>([&](auto ec) {
          constexpr int e = decltype(ec)::value;
          w[e] = fmaf(kap, __builtin_amdgcn_exp2f(-(TT[kb / 2][8 * (kb % 2) + e] * irho)), w[e]);
        });
      split(w, whi, wlo, std::false_type{});
    };
    auto compute = [&](int t) {
      const int buf = t % kOtfBufs;
      tstep = t;
      if constexpr (kDpp) load_cols(buf);
      if constexpr (kTmma) static_for<kMfmaKb / 2>([&](auto pc) { tmma(buf, decltype(pc)::value); });
      if constexpr (kFarT) {
        using K0 = std::integral_constant<int, 0>;
        using K1 = std::integral_constant<int, 1>;
        using K2 = std::integral_constant<int, 2>;
        using K3 = std::integral_constant<int, 3>;
        V h0, l0, h1, l1;
        float wa[8], wb[8];
        pre(K0{}, wa);
        fin(K0{}, wa, h0, l0);
        pre(K1{}, wb);
        mma(buf, 0, h0, l0);
        fin(K1{}, wb, h1, l1);
        pre(K2{}, wa);
        mma(buf, 1, h1, l1);
        fin(K2{}, wa, h0, l0);
        pre(K3{}, wb);
        mma(buf, 2, h0, l0);
        fin(K3{}, wb, h1, l1);
        mma(buf, 3, h1, l1);
      } else {
        V h0, l0, h1, l1;
        eval(buf, std::integral_constant<int, 0>{}, h0, l0);
        static_for<kMfmaKb / 2>([&](auto pc) {
          constexpr int kb = 2 * decltype(pc)::value;
          eval(buf, std::integral_constant<int, kb + 1>{}, h1, l1);
          mma(buf, kb, h0, l0);
          if constexpr (kb + 2 < kMfmaKb) eval(buf, std::integral_constant<int, kb + 2>{}, h0, l0);
          mma(buf, kb + 1, h1, l1);
        });
      }
    };
    // Ping-pong (eight waves, far form): waves w and w + 4 share a SIMD, and
    // the step runs in four phases separated by barriers, in which one of the
    // two evaluates (vector units) while the other multiplies (matrix cores):
    //   phase  waves 0-3 (group A)        waves 4-7 (group B)
    //   0      evaluate t, steps 0-1      multiply t - 1, steps 2-3
    //   1      multiply t, steps 0-1      evaluate t, steps 0-1
    //   2      evaluate t, steps 2-3      multiply t, steps 0-1    (+ store t + 1)
    //   3      multiply t, steps 2-3      evaluate t, steps 2-3
    // so the SIMD always has a vector stream and a matrix stream that do not
    // wait for each other.  Buffer (t + 1) % 2 is stored in phase 2: its last
    // readers (group B's products of step t - 1) finished in phase 0.
    if constexpr (kPP && kFarT) {
      const bool grpB = wave >= 4;
      V h0, l0, h1, l1;
      float wa[8], wb[8];
      auto valu = [&](int t, auto hfc) {
        constexpr int hf = decltype(hfc)::value;
        const int buf = t % kOtfBufs;
        tstep = t;
        if constexpr (hf == 0) static_for<kMfmaKb / 2>([&](auto pc) { tmma(buf, decltype(pc)::value); });
        using KA = std::integral_constant<int, 2 * hf>;
        using KB = std::integral_constant<int, 2 * hf + 1>;
        pre(KA{}, wa);
        fin(KA{}, wa, h0, l0);
        pre(KB{}, wb);
        fin(KB{}, wb, h1, l1);
      };
      auto mmah = [&](int t, int hf) {
        const int buf = t % kOtfBufs;
        mma(buf, 2 * hf, h0, l0);
        mma(buf, 2 * hf + 1, h1, l1);
      };
      using H0 = std::integral_constant<int, 0>;
      using H1 = std::integral_constant<int, 1>;
      if (nsteps > 0) {
        load_next(0);
        store_next(0);
        __syncthreads();
        for (int t = 0; t < nsteps; ++t) {
          if ((t & 15) == 0) make_mask(t / 16);
          load_next(t + 1);
          __builtin_amdgcn_sched_barrier(0);
          if (!grpB) valu(t, H0{});
          else if (t > 0) mmah(t - 1, 1);
          __syncthreads();
          if (!grpB) mmah(t, 0);
          else valu(t, H0{});
          __syncthreads();
          if (!grpB) valu(t, H1{});
          else mmah(t, 0);
          store_next(t + 1);
          __syncthreads();
          if (!grpB) mmah(t, 1);
          else valu(t, H1{});
          __syncthreads();
        }
        if (grpB) mmah(nsteps - 1, 1);
      }
      return;
    }
    // step t: issue the loads of step t + 1, evaluate and multiply step t from
    // LDS buffer t % kOtfBufs, (one buffer: barrier), store step t + 1 into the
    // next buffer, barrier.
    if (nsteps > 0) {
      load_next(0);
      store_next(0);
      __syncthreads();
      for (int t = 0; t < nsteps; ++t) {
        if constexpr (kFar) {
          if ((t & 15) == 0) make_mask(t / 16);
        }
        load_next(t + 1);
        // keep the prefetch at the top: left to itself the scheduler sinks it
        // to just before its LDS store, exposing its latency every step
        __builtin_amdgcn_sched_barrier(0);
        compute(t);
        if (kOtfBufs == 1) __syncthreads();
        store_next(t + 1);
        __syncthreads();
      }
    }
  };
  bool norm = false;
  if constexpr (kNormCapable) {
    // qmax[1] = max_j |x_j|^2 of the problem's FP32 coordinates; the bound
    // holds for the steeper exponent, m t (kernels with a length ratio 1/m)
    // or max(1, rho) t
    constexpr int M = sym_pow<KIND>();
    const double steep = M ? (double)M : fmax(1.0, (double)op.rho);
    norm = s2d * steep * op.qmax[1] <= kNormMaxT;
    if constexpr (M == 0) {
      if (norm && op.bnd16)
        run(std::true_type{}, std::true_type{});
      else if (norm)
        run(std::true_type{}, std::false_type{});
      else
        run(std::false_type{}, std::false_type{});
    } else {
      if (norm)
        run(std::true_type{}, std::false_type{});
      else
        run(std::false_type{}, std::false_type{});
    }
    __syncthreads();   // the row factors in sR
  } else {
    run(std::false_type{}, std::false_type{});
  }

  const int sG_ = mfma_scale_exp(op.qmax[0], kTwoAcc);
  const double sm = op.amp * ldexp(1.0, -(sG_ + sU));
  const double sc = op.amp * ldexp(1.0, -(sG_ + sU + c));
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int b = sg * NS + nb * 32 + m;
    if (b >= B) continue;
    float* dst = part + ((int64_t)split * B + b) * npad;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int ir = 8 * (r / 4) + 4 * h + (r % 4);
      const int64_t i = row0 + ir;
      const double y = kTwoAcc ? (double)accM[nb][r] * sm + (double)accC[nb][r] * sc : (double)accM[nb][r] * sm;
      dst[i] = (float)(norm ? y * sR[wave][ir] : y);
    }
  }
}

// On-the-fly FP32 form with the products on the FP32 matrix cores
// (32x32x2 FP32 MFMA): the same arithmetic class as the vector-unit sum
// (FP32 kernel values, FP32 products and sums over 256 sources folded into
// FP64), for blocks of 32 NB states.  The sources are g = q f(u) in FP32, as
// for the vector-unit form, so its source preparation and RK4 combination
// are shared.
//
// MFMA step ks of a pipeline step covers sources ks and 32 + ks: lane
// l = m + 32 h evaluates u(row m, source 32 h + ks) (A operand, one value)
// and holds g(source 32 h + ks, state m) (B operand); outputs as in the split
// kernels (rows 8 (r / 4) + 4 h + r % 4, state m).  The vector units only
// evaluate the kernel (one value per lane per MFMA step), so the matrix
// cores bound the kernel.  Coordinates and g of a pipeline step are staged
// through double-buffered LDS tiles; states beyond B read state B - 1 (their
// outputs are never written).
constexpr int kF32FoldSteps = 4;     // pipeline steps (of 64 sources) per FP64 fold
// One LDS buffer for the staged sources and a second barrier per step: 5.19
// -> 5.10 ms per application at N = 65536, B = 64 (measured alternately
// against two buffers), same registers and occupancy.
#ifndef NFR_MFMA_F32_LDS_BUFS
#define NFR_MFMA_F32_LDS_BUFS 1
#endif
constexpr int kF32Bufs = NFR_MFMA_F32_LDS_BUFS;

template <int KIND, int NB>
__global__ __launch_bounds__(kWG, 2) void k_mfma_otf_f32(const float4* __restrict__ src, const float* __restrict__ g,
                                                         int64_t npad, int B, int64_t kchunk, PairParams pp,
                                                         double* __restrict__ part) {
  constexpr int NS = 32 * NB;
  constexpr int STRIDE = kMfmaStep + 4;          // floats per LDS row of sG
  constexpr int ROWCH = kMfmaStep / 4;           // 16-byte chunks per row
  constexpr int CHUNKS = NS * ROWCH / kWG;       // chunks per thread per step
  typedef __attribute__((ext_vector_type(4))) float f4_t;
  __shared__ __attribute__((aligned(16))) float sG[kF32Bufs][NS][STRIDE];
  // column coordinates x, y, z (row 3: the packed zero component); wave w
  // loads and stores row w, so no load sits behind a branch
  __shared__ __attribute__((aligned(16))) float sS[kF32Bufs][4][kMfmaStep];
  static_assert(kWG == 4 * 64, "one wave per coordinate row");

  const int64_t wg = blockIdx.x;
  const int split = (int)(wg % kMfmaSplits);
  const int64_t rb = wg / kMfmaSplits;
  const int sg = blockIdx.y;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int m = lane & 31;
  const int h = lane >> 5;
  const int64_t row0 = rb * kMfmaRowsPerWG + wave * 32;
  const int64_t k_begin = (int64_t)split * kchunk;
  int64_t k_end = k_begin + kchunk;
  if (k_end > npad) k_end = npad;
  const int nsteps = (int)((k_end - k_begin) / kMfmaStep);

  const float4 pr = src[row0 + m];
  const float xi = pr.x * pp.sig, yi = pr.y * pp.sig, zi = pr.z * pp.sig;

  const float* gsrc[CHUNKS];
  int g_row[CHUNKS], g_col[CHUNKS];
#pragma unroll
  for (int q = 0; q < CHUNKS; ++q) {
    const int cc = tid + kWG * q;
    g_row[q] = cc / ROWCH;
    g_col[q] = 4 * (cc % ROWCH);
    int b = sg * NS + g_row[q];
    if (b > B - 1) b = B - 1;
    gsrc[q] = g + (int64_t)b * npad + k_begin + g_col[q];
  }

  f32x16_t acc[NB];
  double facc[NB][16];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      acc[nb][r] = 0.0f;
      facc[nb][r] = 0.0;
    }

  f4_t gn[CHUNKS];
  float sn;
  auto load_next = [&](int t) {
    const int64_t tc = t < nsteps ? t : nsteps - 1;
#pragma unroll
    for (int q = 0; q < CHUNKS; ++q) gn[q] = *reinterpret_cast<const f4_t*>(gsrc[q] + tc * kMfmaStep);
    sn = reinterpret_cast<const float*>(src + k_begin + tc * kMfmaStep + lane)[wave];
  };
  auto store_next = [&](int t) {
    const int buf = t % kF32Bufs;
#pragma unroll
    for (int q = 0; q < CHUNKS; ++q) *reinterpret_cast<f4_t*>(&sG[buf][g_row[q]][g_col[q]]) = gn[q];
    sS[buf][wave][lane] = sn * pp.sig;
  };
  auto compute = [&](int t) {
    const int buf = t % kF32Bufs;
#pragma unroll
    for (int k4 = 0; k4 < kMfmaStep / 8; ++k4) {
      const int c0 = 32 * h + 4 * k4;
      const f4_t cx = *reinterpret_cast<const f4_t*>(&sS[buf][0][c0]);
      const f4_t cy = *reinterpret_cast<const f4_t*>(&sS[buf][1][c0]);
      const f4_t cz = *reinterpret_cast<const f4_t*>(&sS[buf][2][c0]);
      f4_t gv[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) gv[nb] = *reinterpret_cast<const f4_t*>(&sG[buf][nb * 32 + m][c0]);
      float u[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float r2 = pair_r2<KIND>(xi - cx[e], yi - cy[e], zi - cz[e], pp.per);
        const float tt = ((KIND & 1) == 0) ? r2 : __builtin_amdgcn_sqrtf(r2);
        u[e] = pair_u<KIND>(tt, pp.rho, pp.kappa);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(u[e], gv[nb][e], acc[nb], 0, 0, 0);
    }
  };
  auto fold = [&]() {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        facc[nb][r] += (double)acc[nb][r];
        acc[nb][r] = 0.0f;
      }
  };
  if (nsteps > 0) {
    load_next(0);
    store_next(0);
    __syncthreads();
    for (int t = 0; t < nsteps; ++t) {
      load_next(t + 1);
      // keep the prefetch at the top: left to itself the scheduler sinks it
      // to just before its LDS store, exposing its latency every step
      __builtin_amdgcn_sched_barrier(0);
      compute(t);
      if ((t + 1) % kF32FoldSteps == 0) fold();
      if (kF32Bufs == 1) __syncthreads();
      store_next(t + 1);
      __syncthreads();
    }
    fold();
  }

#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int b = sg * NS + nb * 32 + m;
    if (b >= B) continue;
    double* dst = part + ((int64_t)split * B + b) * npad;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t i = row0 + 8 * (r / 4) + 4 * h + (r % 4);
      dst[i] = pp.amp * facc[nb][r];
    }
  }
}

// RK4 stage combination for the split forms: as k_rk4_combine, but the next
// stage's sources are written as Ghi/Glo (no q: it sits inside W).
template <typename T, typename PT>
__global__ __launch_bounds__(kWG) void k_mfma_combine(const PT* __restrict__ part, int nsplit, int64_t n,
                                                      int64_t npad, int B, int stage, double dt,
                                                      double* __restrict__ u, double* __restrict__ v,
                                                      double* __restrict__ ksum, Firing fr, const double* __restrict__ qd,
                                                      const double* __restrict__ qmax, T* __restrict__ Ghi,
                                                      T* __restrict__ Glo, double* __restrict__ k1_out,
                                                      const double* __restrict__ gamma) {
  const int64_t idx = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (idx >= n * (int64_t)B) return;
  const int b = (int)(idx / n);
  const int64_t i = idx - (int64_t)b * n;
  double y = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) y += (double)part[((int64_t)sp * B + b) * npad + i];
  const double k = -v[idx] + y + (gamma ? gamma[idx] : 0.0);
  double ui = u[idx];
  double vn;
  if (stage == 1) {
    if (k1_out) k1_out[idx] = k;
    ksum[idx] = k;
    vn = ui + 0.5 * dt * k;
  } else if (stage == 2) {
    ksum[idx] += 2.0 * k;
    vn = ui + 0.5 * dt * k;
  } else if (stage == 3) {
    ksum[idx] += 2.0 * k;
    vn = ui + dt * k;
  } else {
    ui = ui + (dt / 6.0) * (ksum[idx] + k);
    u[idx] = ui;
    vn = ui;
  }
  v[idx] = vn;
  T hi, lo;
  split_hi_lo<T>(sigmoid(vn, fr.beta, state_theta(fr, b)) * source_factor<T>(qd, qmax, i), hi, lo);
  Ghi[(int64_t)b * npad + i] = hi;
  Glo[(int64_t)b * npad + i] = lo;
}

// One Adams-Bashforth 5 step for the split forms (see k_ab5_combine); the next
// sources are written as Ghi/Glo.
template <typename T, typename PT>
__global__ __launch_bounds__(kWG) void k_mfma_ab5_combine(const PT* __restrict__ part, int nsplit, int64_t n,
                                                          int64_t npad, int B, double dt, Ab5Weights wt,
                                                          int4 slots03, int slot4, double* __restrict__ u,
                                                          double* __restrict__ hist, Firing fr,
                                                          const double* __restrict__ qd, const double* __restrict__ qmax,
                                                          T* __restrict__ Ghi, T* __restrict__ Glo) {
  const int64_t idx = (int64_t)blockIdx.x * kWG + threadIdx.x;
  const int64_t nb = n * (int64_t)B;
  if (idx >= nb) return;
  const int b = (int)(idx / n);
  const int64_t i = idx - (int64_t)b * n;
  double y = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) y += (double)part[((int64_t)sp * B + b) * npad + i];
  const double ui = u[idx];
  const double F = -ui + y;
  hist[slots03.x * nb + idx] = F;
  const double incr = wt.a[0] * F + wt.a[1] * hist[slots03.y * nb + idx] + wt.a[2] * hist[slots03.z * nb + idx] +
                      wt.a[3] * hist[slots03.w * nb + idx] + wt.a[4] * hist[(int64_t)slot4 * nb + idx];
  const double un = ui + dt * incr;
  u[idx] = un;
  T hi, lo;
  split_hi_lo<T>(sigmoid(un, fr.beta, state_theta(fr, b)) * source_factor<T>(qd, qmax, i), hi, lo);
  Ghi[(int64_t)b * npad + i] = hi;
  Glo[(int64_t)b * npad + i] = lo;
}

// ---------------------------------------------------------------- launchers

struct MfmaBufs {
  const float* header;
  void* tiles;
};

inline MfmaBufs mfma_bufs(const void* W, int64_t) {
  char* base = static_cast<char*>(const_cast<void*>(W));
  MfmaBufs m;
  m.header = reinterpret_cast<const float*>(base);
  m.tiles = base + kMfmaHeader;
  return m;
}

inline void mfma_g_split(void* g, int64_t npad, int B, void** ghi, void** glo) {
  char* base = static_cast<char*>(g);
  *ghi = base;
  *glo = base + size_t(mfma_bp(B)) * npad * 2;
}

template <typename T>
inline void launch_mfma_w_build_t(const ProblemView& pv, const KernelF64& kp, void* W, hipStream_t s) {
  MfmaBufs m = mfma_bufs(W, pv.npad);
  const double amp = fabs(kp.Ae) + fabs(kp.Ai);
  hipLaunchKernelGGL(k_mfma_scale<T>, dim3(1), dim3(kWG), 0, s, pv.q, pv.npad, amp,
                     (int)MfmaTraits<T>::fp16, const_cast<float*>(m.header));
  hipLaunchKernelGGL(k_mfma_w_build<T>, dim3((unsigned)pv.npad, (unsigned)ceil_div(pv.npad / 8, kWG)), dim3(kWG), 0, s,
                     pv.xyz, pv.q, pv.n, pv.npad, kp, m.header, static_cast<T*>(m.tiles));
}

inline void launch_mfma_w_build(const ProblemView& pv, int form, const KernelF64& kp, void* W, hipStream_t s) {
  if (mfma_is_bf16(form))
    launch_mfma_w_build_t<__bf16>(pv, kp, W, s);
  else
    launch_mfma_w_build_t<_Float16>(pv, kp, W, s);
}

template <typename T>
inline void launch_mfma_prep_t(const ProblemView& pv, int B, const double* u, const Firing& fr, const double* qd,
                               void* g, double* v, hipStream_t s) {
  void *ghi, *glo;
  mfma_g_split(g, pv.npad, B, &ghi, &glo);
  const int64_t Bp = mfma_bp(B);
  hipLaunchKernelGGL(k_mfma_prep<T>, dim3((unsigned)ceil_div(pv.npad * Bp, kWG)), dim3(kWG), 0, s, u, pv.n, pv.npad,
                     B, Bp, fr, qd, pv.qmax, static_cast<T*>(ghi), static_cast<T*>(glo), v);
}

// Weights in G for the fused forms (their kernel values carry none), not for the W forms.
inline const double* mfma_source_q(const ProblemView& pv, int form) { return mfma_has_w(form) ? nullptr : pv.q; }

inline void launch_mfma_prep(const ProblemView& pv, int form, int B, const double* u, const Firing& fr, float* g,
                             double* v, hipStream_t s) {
  if (mfma_is_bf16(form))
    launch_mfma_prep_t<__bf16>(pv, B, u, fr, mfma_source_q(pv, form), g, v, s);
  else
    launch_mfma_prep_t<_Float16>(pv, B, u, fr, mfma_source_q(pv, form), g, v, s);
}

template <typename T>
inline void launch_mfma_apply_t(const ProblemView& pv, int B, const void* W, const void* g, double* part,
                                hipStream_t s) {
  MfmaBufs m = mfma_bufs(W, pv.npad);
  void *ghi, *glo;
  mfma_g_split(const_cast<void*>(g), pv.npad, B, &ghi, &glo);
  const int64_t kchunk = round_up(ceil_div(pv.npad, apply_splits<T>()), kMfmaStep);
  const unsigned grid_x = (unsigned)(pv.npad / kMfmaRowsPerWG * apply_splits<T>());
  if (B <= 32) {
    hipLaunchKernelGGL((k_mfma_apply<T, 1>), dim3(grid_x, 1), dim3(kWG), 0, s, static_cast<const T*>(m.tiles),
                       static_cast<const T*>(ghi), static_cast<const T*>(glo), pv.npad, B, kchunk, m.header, part);
  } else {
    hipLaunchKernelGGL((k_mfma_apply<T, 2>), dim3(grid_x, (unsigned)(mfma_bp(B) / 64)), dim3(kWG), 0, s,
                       static_cast<const T*>(m.tiles), static_cast<const T*>(ghi), static_cast<const T*>(glo),
                       pv.npad, B, kchunk, m.header, part);
  }
}

inline void launch_mfma_apply(const ProblemView& pv, int form, int B, const void* W, const float* g, double* part,
                              hipStream_t s) {
  if (mfma_is_bf16(form))
    launch_mfma_apply_t<__bf16>(pv, B, W, g, part, s);
  else
    launch_mfma_apply_t<_Float16>(pv, B, W, g, part, s);
}

template <typename T, int KIND>
inline void launch_mfma_otf_t(const ProblemView& pv, const MfmaOtfParams& op, int B, const void* g, float* part,
                              hipStream_t s) {
  void *ghi, *glo;
  mfma_g_split(const_cast<void*>(g), pv.npad, B, &ghi, &glo);
  const int64_t kchunk = round_up(ceil_div(pv.npad, kMfmaSplits), kMfmaStep);
  const unsigned grid_x = (unsigned)(pv.npad / kMfmaRowsPerWG * kMfmaSplits);
  if (B <= 32) {
    hipLaunchKernelGGL((k_mfma_otf<T, KIND, 1>), dim3(grid_x, 1), dim3(kWG), 0, s, pv.src,
                       static_cast<const T*>(ghi), static_cast<const T*>(glo), pv.npad, B, kchunk, op, part);
  } else {
    if constexpr (kMfmaOtfPingPong && !MfmaTraits<T>::fp16 && KIND == 0) {
      if (op.bnd16) {
        // far form: eight waves per workgroup (npad is a multiple of 256)
        hipLaunchKernelGGL((k_mfma_otf<T, KIND, 2, 8>), dim3(grid_x / 2, (unsigned)(mfma_bp(B) / 64)), dim3(2 * kWG),
                           0, s, pv.src, static_cast<const T*>(ghi), static_cast<const T*>(glo), pv.npad, B, kchunk,
                           op, part);
        return;
      }
    }
    hipLaunchKernelGGL((k_mfma_otf<T, KIND, 2>), dim3(grid_x, (unsigned)(mfma_bp(B) / 64)), dim3(kWG), 0, s, pv.src,
                       static_cast<const T*>(ghi), static_cast<const T*>(glo), pv.npad, B, kchunk, op, part);
  }
}

// Forms 4 / 5 for template code KIND (see k_mfma_otf).
template <int KIND>
inline void launch_mfma_otf(const ProblemView& pv, int form, const MfmaOtfParams& op, int B, const float* g,
                            double* part, hipStream_t s) {
  // the fused forms write FP32 partial sums (each source chunk's FP32 matrix-core
  // sum rounded once more; the combine adds them in FP64): half the bytes of
  // FP64 slots, written here and read by every combine
  float* pf = reinterpret_cast<float*>(part);
  if (mfma_is_bf16(form))
    launch_mfma_otf_t<__bf16, KIND>(pv, op, B, g, pf, s);
  else
    launch_mfma_otf_t<_Float16, KIND>(pv, op, B, g, pf, s);
}

// On-the-fly FP32 form on the FP32 matrix cores for template code KIND; g is
// the FP32 source array of the on-the-fly forms (npad x B, q included).
template <int KIND>
inline void launch_mfma_otf_f32(const ProblemView& pv, const PairParams& pp, int B, const float* g, double* part,
                                hipStream_t s) {
  const int64_t kchunk = round_up(ceil_div(pv.npad, kMfmaSplits), kMfmaStep);
  const unsigned grid_x = (unsigned)(pv.npad / kMfmaRowsPerWG * kMfmaSplits);
  if (B <= 32)
    hipLaunchKernelGGL((k_mfma_otf_f32<KIND, 1>), dim3(grid_x, 1), dim3(kWG), 0, s, pv.src, g, pv.npad, B, kchunk, pp,
                       part);
  else
    hipLaunchKernelGGL((k_mfma_otf_f32<KIND, 2>), dim3(grid_x, (unsigned)ceil_div(B, 64)), dim3(kWG), 0, s, pv.src, g,
                       pv.npad, B, kchunk, pp, part);
}

template <typename T, typename PT>
inline void launch_mfma_combine_t(const ProblemView& pv, int B, int stage, double dt, double* u, double* v,
                                  double* ksum, const PT* part, int nsplit, const Firing& fr, const double* qd,
                                  void* g, double* k1_out, const double* gamma, hipStream_t s) {
  void *ghi, *glo;
  mfma_g_split(g, pv.npad, B, &ghi, &glo);
  const int64_t total = pv.n * (int64_t)B;
  hipLaunchKernelGGL((k_mfma_combine<T, PT>), dim3((unsigned)ceil_div(total, kWG)), dim3(kWG), 0, s, part, nsplit,
                     pv.n, pv.npad, B, stage, dt, u, v, ksum, fr, qd, pv.qmax, static_cast<T*>(ghi),
                     static_cast<T*>(glo), k1_out, gamma);
}

inline void launch_mfma_combine(const ProblemView& pv, int form, int B, int stage, double dt, double* u, double* v,
                                double* ksum, const double* part, int nsplit, const Firing& fr, float* g,
                                double* k1_out, const double* gamma, hipStream_t s) {
  const double* qd = mfma_source_q(pv, form);
  const float* pf = reinterpret_cast<const float*>(part);
  switch (form) {
    case 2: launch_mfma_combine_t<__bf16>(pv, B, stage, dt, u, v, ksum, part, nsplit, fr, qd, g, k1_out, gamma, s); break;
    case 3: launch_mfma_combine_t<_Float16>(pv, B, stage, dt, u, v, ksum, part, nsplit, fr, qd, g, k1_out, gamma, s); break;
    case 4: launch_mfma_combine_t<__bf16>(pv, B, stage, dt, u, v, ksum, pf, nsplit, fr, qd, g, k1_out, gamma, s); break;
    default: launch_mfma_combine_t<_Float16>(pv, B, stage, dt, u, v, ksum, pf, nsplit, fr, qd, g, k1_out, gamma, s); break;
  }
}

template <typename T, typename PT>
inline void launch_mfma_ab5_t(const ProblemView& pv, int B, double dt, const Ab5Weights& wt, int4 s03, int s4,
                              double* u, double* hist, const PT* part, int nsplit, const Firing& fr,
                              const double* qd, void* g, hipStream_t s) {
  void *ghi, *glo;
  mfma_g_split(g, pv.npad, B, &ghi, &glo);
  const int64_t total = pv.n * (int64_t)B;
  hipLaunchKernelGGL((k_mfma_ab5_combine<T, PT>), dim3((unsigned)ceil_div(total, kWG)), dim3(kWG), 0, s, part, nsplit,
                     pv.n, pv.npad, B, dt, wt, s03, s4, u, hist, fr, qd, pv.qmax, static_cast<T*>(ghi),
                     static_cast<T*>(glo));
}

inline void launch_mfma_ab5(const ProblemView& pv, int form, int B, double dt, const Ab5Weights& wt, int4 s03, int s4,
                            double* u, double* hist, const double* part, int nsplit, const Firing& fr, float* g,
                            hipStream_t s) {
  const double* qd = mfma_source_q(pv, form);
  const float* pf = reinterpret_cast<const float*>(part);
  switch (form) {
    case 2: launch_mfma_ab5_t<__bf16>(pv, B, dt, wt, s03, s4, u, hist, part, nsplit, fr, qd, g, s); break;
    case 3: launch_mfma_ab5_t<_Float16>(pv, B, dt, wt, s03, s4, u, hist, part, nsplit, fr, qd, g, s); break;
    case 4: launch_mfma_ab5_t<__bf16>(pv, B, dt, wt, s03, s4, u, hist, pf, nsplit, fr, qd, g, s); break;
    default: launch_mfma_ab5_t<_Float16>(pv, B, dt, wt, s03, s4, u, hist, pf, nsplit, fr, qd, g, s); break;
  }
}

inline void launch_mfma_reduce(const ProblemView& pv, int form, int B, const double* part, int nsplit, double* y,
                               hipStream_t s) {
  const int64_t total = pv.n * (int64_t)B;
  if (mfma_has_w(form))
    hipLaunchKernelGGL((k_reduce_partials<1, double>), dim3((unsigned)ceil_div(total, kWG)), dim3(kWG), 0, s, part,
                       nsplit, pv.n, pv.npad, B, y);
  else
    hipLaunchKernelGGL((k_reduce_partials<1, float>), dim3((unsigned)ceil_div(total, kWG)), dim3(kWG), 0, s,
                       reinterpret_cast<const float*>(part), nsplit, pv.n, pv.npad, B, y);
}

}  // namespace nfr
