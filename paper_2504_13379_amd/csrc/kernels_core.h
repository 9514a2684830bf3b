// Core device kernels: problem packing, source preparation, the on-the-fly
// tiled pair sum, partial reduction, the RK4 stage combination, and the FP32
// precomputed-W build and apply.
//
// Operator (paper section 2.2, eq. NFODETilde):
//     K_i(u) = sum_j w(|x_i - x_j|) q_j f(u_j),   all j including j = i.
#pragma once

#include "common.h"

namespace nfr {

// ------------------------------------------------------------------ packing

// xyz (n x 3 FP64) and q (n FP64) -> FP32 float4 coordinates, FP64 weights and
// FP64 coordinates, each padded to npad with zeros (weight 0: padding sources
// never contribute; padding targets are computed and discarded).  With
// period > 0, x and y are first reduced by whole periods to [-period/2,
// period/2] (the same points of the periodic plane).  The fourth component is
// the squared norm of the FP32 coordinates, rounded once from FP64 (0 with
// period > 0), for kernels that expand r^2 = |x_i|^2 + |x_j|^2 - 2 x_i . x_j.
__global__ __launch_bounds__(kWG) void k_pack(const double* __restrict__ xyz, const double* __restrict__ q,
                                              int64_t n, int64_t npad, double period, float4* __restrict__ src,
                                              double* __restrict__ qd, double* __restrict__ xyz64) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= npad) return;
  double x = 0.0, y = 0.0, z = 0.0, w = 0.0;
  if (i < n) {
    x = xyz[3 * i + 0];
    y = xyz[3 * i + 1];
    z = xyz[3 * i + 2];
    w = q[i];
    if (period > 0.0) {
      x -= period * rint(x / period);
      y -= period * rint(y / period);
    }
  }
  const float xf = (float)x, yf = (float)y, zf = (float)z;
  const double nrm = period > 0.0 ? 0.0 : (double)xf * xf + (double)yf * yf + (double)zf * zf;
  src[i] = make_float4(xf, yf, zf, (float)nrm);
  qd[i] = w;
  xyz64[3 * i + 0] = x;
  xyz64[3 * i + 1] = y;
  xyz64[3 * i + 2] = z;
}

// qmax[0] = max_j |q_j| and qmax[1] = max_j |x_j|^2 (the packed FP32 norms) over
// the npad packed nodes (one workgroup).
__global__ __launch_bounds__(kWG) void k_qmax(const double* __restrict__ qd, const float4* __restrict__ src, int64_t npad,
                                              double* __restrict__ qmax) {
  __shared__ double red[2][kWG];
  double m = 0.0, r = 0.0;
  for (int64_t j = threadIdx.x; j < npad; j += kWG) {
    m = fmax(m, fabs(qd[j]));
    r = fmax(r, (double)src[j].w);
  }
  red[0][threadIdx.x] = m;
  red[1][threadIdx.x] = r;
  __syncthreads();
  for (int s = kWG / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + s]);
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    qmax[0] = red[0][0];
    qmax[1] = red[1][0];
  }
}

// ------------------------------------------------------------------ sources

// g[b*npad + j] = s_j f_b(u[b*n + j]) in FP32 with s_j = q_j (with_q) or 1;
// zero on padding nodes.  Optionally copies u into v (the first RK4 stage input).
__global__ __launch_bounds__(kWG) void k_source_prep(const double* __restrict__ u, int64_t n, int64_t npad, int B,
                                                     const double* __restrict__ qd, int with_q, Firing fr,
                                                     float* __restrict__ g, double* __restrict__ v_copy) {
  const int64_t idx = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (idx >= npad * (int64_t)B) return;
  const int b = (int)(idx / npad);
  const int64_t j = idx - (int64_t)b * npad;
  float out = 0.0f;
  if (j < n) {
    const double uj = u[(int64_t)b * n + j];
    const double s = with_q ? qd[j] : 1.0;
    out = (float)(s * sigmoid(uj, fr.beta, state_theta(fr, b)));
    if (v_copy) v_copy[(int64_t)b * n + j] = uj;
  }
  g[idx] = out;
}

// ------------------------------------------------------------------ on-the-fly pair sum

// Length scales in an integer ratio, rho = 1/m with m in {2, 3, 4}: the
// excitatory exponential is the m-th power of the inhibitory one,
// exp2(-t) = exp2(-rho t)^m, so one exponential per pair suffices.  KIND bits
// 2-3 hold m - 1 (0: two exponentials); such launches scale the coordinates
// (and the period) by the inhibitory length, so the kernel's t is rho t.
template <int KIND>
constexpr int sym_pow() {
  return (KIND >> 2) == 0 ? 0 : (KIND >> 2) + 1;
}

template <int M>
__device__ __forceinline__ float ipow(float x) {
  if (M == 2) return x * x;
  if (M == 3) return x * x * x;
  const float x2 = x * x;
  return x2 * x2;
}

// Normalised kernel u = exp2(-t_e) + kappa exp2(-t_i) of one pair from its
// scaled distance t (r^2 or r).  Without an integer ratio, t = t_e and
// t_i = rho t; with sym_pow (coordinates in units of the inhibitory length)
// t = t_i, exp2(-t_e) = exp2(-t)^m and u = e (e^(m-1) + kappa), e = exp2(-t).
template <int KIND>
__device__ __forceinline__ float pair_u(float t, float rho, float kappa) {
  constexpr int M = sym_pow<KIND>();
  if (M == 0) return fmaf(__builtin_amdgcn_exp2f(-(t * rho)), kappa, __builtin_amdgcn_exp2f(-t));
  const float e = __builtin_amdgcn_exp2f(-t);
  if (M == 2) return e * (e + kappa);
  if (M == 3) return e * fmaf(e, e, kappa);
  const float e2 = e * e;
  return fmaf(e2, e2, kappa * e);
}

// Partial pair sums over one source chunk:
//   part[(split*B + b)*npad + i] = sum_{j in chunk(split)} w(|x_i - x_j|) g[b*npad + j]
// Grid: x = target tiles of kWG*TPT targets (thread t owns tile + t + kWG*k),
//       y = source chunks of `chunk` nodes (a multiple of kWG),
//       z = state blocks of BS states.
// Sources are staged kWG at a time in LDS as scaled float4 coordinates plus
// their g values and read back as broadcasts.  Each thread sums one LDS tile
// of kWG sources in FP32 (the normalised kernel u, see PairParams), then folds
// the tile sum into FP64 accumulators: amp * sum.
// Targets per thread for a block of BS states (TPT x BS accumulators per thread).
__host__ __device__ constexpr int otf_tpt(int bs) { return bs <= 4 ? 4 : 2; }

template <int KIND, int TPT, int BS>
__device__ inline void otf_tile(const float4* __restrict__ src, const float* __restrict__ g, int64_t npad, int B,
                                int64_t chunk, const PairParams& pp, double* __restrict__ part, int64_t tile,
                                int split, int b0, float4* s_src, float (*s_g)[kWG]) {
  const int tid = threadIdx.x;
  const int64_t tbase = tile * (kWG * TPT);

  float xi[TPT], yi[TPT], zi[TPT];
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    int64_t t = tbase + tid + (int64_t)kWG * k;
    if (t >= npad) t = npad - 1;
    const float4 p = src[t];
    xi[k] = p.x * pp.sig;
    yi[k] = p.y * pp.sig;
    zi[k] = p.z * pp.sig;
  }
  double acc[TPT][BS];
#pragma unroll
  for (int k = 0; k < TPT; ++k)
#pragma unroll
    for (int b = 0; b < BS; ++b) acc[k][b] = 0.0;

  const int64_t j_begin = (int64_t)split * chunk;
  int64_t j_end = j_begin + chunk;
  if (j_end > npad) j_end = npad;
  const float rho = pp.rho;
  const float kappa = pp.kappa;

  for (int64_t j0 = j_begin; j0 < j_end; j0 += kWG) {
    {
      const float4 s = src[j0 + tid];
      s_src[tid] = make_float4(s.x * pp.sig, s.y * pp.sig, s.z * pp.sig, 0.0f);
#pragma unroll
      for (int b = 0; b < BS; ++b)
        s_g[b][tid] = (b0 + b < B) ? g[(int64_t)(b0 + b) * npad + j0 + tid] : 0.0f;
    }
    __syncthreads();
    float a[TPT][BS];
#pragma unroll
    for (int k = 0; k < TPT; ++k)
#pragma unroll
      for (int b = 0; b < BS; ++b) a[k][b] = 0.0f;

#pragma unroll 4
    for (int jj = 0; jj < kWG; ++jj) {
      const float4 s = s_src[jj];
      float gv[BS];
#pragma unroll
      for (int b = 0; b < BS; ++b) gv[b] = s_g[b][jj];
#pragma unroll
      for (int k = 0; k < TPT; ++k) {
        const float r2 = pair_r2<KIND>(xi[k] - s.x, yi[k] - s.y, zi[k] - s.z, pp.per);
        const float t = ((KIND & 1) == 0) ? r2 : __builtin_amdgcn_sqrtf(r2);
        const float u = pair_u<KIND>(t, rho, kappa);
#pragma unroll
        for (int b = 0; b < BS; ++b) a[k][b] = fmaf(u, gv[b], a[k][b]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TPT; ++k)
#pragma unroll
      for (int b = 0; b < BS; ++b) acc[k][b] += pp.amp * (double)a[k][b];
  }

#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int64_t t = tbase + tid + (int64_t)kWG * k;
    if (t >= npad) continue;
#pragma unroll
    for (int b = 0; b < BS; ++b)
      if (b0 + b < B) part[((int64_t)split * B + b0 + b) * npad + t] = acc[k][b];
  }
}

template <int KIND, int TPT, int BS>
__global__ __launch_bounds__(kWG) void k_otf_pair_sum(const float4* __restrict__ src, const float* __restrict__ g,
                                                      int64_t npad, int B, int64_t chunk, PairParams pp,
                                                      double* __restrict__ part) {
  __shared__ float4 s_src[kWG];
  __shared__ float s_g[BS][kWG];
  otf_tile<KIND, TPT, BS>(src, g, npad, B, chunk, pp, part, blockIdx.x, blockIdx.y, blockIdx.z * BS, s_src, s_g);
}

// ------------------------------------------------------------------ symmetric on-the-fly pair sum

// The kernel is radial, so w_ij = w_ji: one evaluation of a pair can feed both
// y_i (weight g_j) and y_j (weight g_i).  Nodes are cut into tiles of kSymTile;
// workgroup p handles the tile pair (I, J), I <= J, decoded from p = J (J+1)/2 + I.
// Off-diagonal pairs (I < J) produce the row sums of tile I over sources in J
// and the column sums of tile J over sources in I; diagonal pairs only row sums.
// Slots: the row sums of (I, J) go to slot J of the nodes of I, the column
// sums to slot I of the nodes of J, so every node receives exactly one
// contribution per tile index and the combine adds slots 0..nt-1 in order.
//
// Each lane keeps kSymTPT targets in registers, so one wave holds the whole
// tile of 64 * kSymTPT targets; the kSymSplit waves of a workgroup share those
// targets and split the tile's source groups between them (group g goes to
// wave g mod kSymSplit).  A group of 64 sources is loaded one per lane and
// rotated around the wave 64 times (DPP wave rotate by one lane); each source
// carries its own column accumulators, so after a full turn they hold the sum
// over all the tile's targets and the source is back in its lane.  Row sums:
// FP32 per group of 64 sources, folded into FP64, then added over the waves
// in wave order through LDS; column sums: FP32 over the wave, complete.
#ifndef NFR_SYM_SPLIT
#define NFR_SYM_SPLIT 4
#endif
#ifndef NFR_SYM_TPT
#define NFR_SYM_TPT 4
#endif
constexpr int kSymSplit = NFR_SYM_SPLIT;
constexpr int kSymTPT = NFR_SYM_TPT;
constexpr int kSymThreads = 64 * kSymSplit;
constexpr int kSymTile = 64 * kSymTPT;   // 256 nodes by default
// Shape for small problems: one wave per tile pair and one target per lane
// (tiles of 64), so that a few thousand nodes still give hundreds of tile
// pairs; the large shape's 4-target tiles leave most of the chip idle there.
constexpr int kSymSmallTPT = 1;
constexpr int kSymSmallSplit = 1;

__device__ inline float wave_ror1(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x13C, 0xF, 0xF, false));
}

// v from another lane by the DPP pattern CTRL, in the rows of ROW_MASK (0 in
// the other rows); a double moves as its two 32-bit halves.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROW_MASK, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// FP64 sum over the 64 lanes of a wave in a fixed pattern of DPP moves (pairs,
// quads, half-rows, rows of 16, then rows 0 + 1 and 0..3 through the row
// broadcasts); the total is valid in lane 63.
__device__ __forceinline__ double wave_sum_f64(double v) {
  v += dpp_f64<0xB1, 0xF>(v);     // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4E, 0xF>(v);     // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141, 0xF>(v);    // row_half_mirror
  v += dpp_f64<0x140, 0xF>(v);    // row_mirror
  v += dpp_f64<0x142, 0xA>(v);    // row_bcast15 into rows 1 and 3
  v += dpp_f64<0x143, 0xC>(v);    // row_bcast31 into rows 2 and 3
  return v;
}

__host__ __device__ inline int64_t sym_pairs(int64_t nt) { return nt * (nt + 1) / 2; }

__device__ inline void sym_decode(int64_t p, int64_t* I, int64_t* J) {
  int64_t j = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
  while (j * (j + 1) / 2 > p) --j;
  while ((j + 1) * (j + 2) / 2 <= p) ++j;
  *J = j;
  *I = p - j * (j + 1) / 2;
}

template <int KIND, bool COLS, int TPT, int SPLIT>
__device__ inline void sym_tile(const float4* __restrict__ src, const float* __restrict__ g, int64_t npad,
                                const PairParams& pp, double* __restrict__ part, int64_t I, int64_t J,
                                double (*rowsum)[64 * TPT]) {
  constexpr int kSymTPT = TPT, kSymSplit = SPLIT, kSymTile = 64 * TPT, kSymThreads = 64 * SPLIT;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const float rho = pp.rho;
  const float kappa = pp.kappa;
  float xi[kSymTPT], yi[kSymTPT], zi[kSymTPT], gi[kSymTPT];
#pragma unroll
  for (int k = 0; k < kSymTPT; ++k) {
    const int64_t t = I * kSymTile + k * 64 + lane;
    const int64_t tc = t < npad ? t : npad - 1;
    const float4 p = src[tc];
    xi[k] = p.x * pp.sig;
    yi[k] = p.y * pp.sig;
    zi[k] = p.z * pp.sig;
    gi[k] = t < npad ? g[t] : 0.0f;
  }
  double racc[kSymTPT];
#pragma unroll
  for (int k = 0; k < kSymTPT; ++k) racc[k] = 0.0;

  int64_t nsrc = npad - J * kSymTile;
  if (nsrc > kSymTile) nsrc = kSymTile;
  const int ngroups = (int)(nsrc / 64);
  for (int grp = wave; grp < ngroups; grp += kSymSplit) {
    const int64_t j = J * kSymTile + grp * 64 + lane;
    const float4 s4 = src[j];
    float sx = s4.x * pp.sig, sy = s4.y * pp.sig, sz = s4.z * pp.sig, sg = g[j];
    float cs = 0.0f;
    float rs[kSymTPT];
#pragma unroll
    for (int k = 0; k < kSymTPT; ++k) rs[k] = 0.0f;
#pragma unroll 2
    for (int step = 0; step < 64; ++step) {
#pragma unroll
      for (int k = 0; k < kSymTPT; ++k) {
        const float r2 = pair_r2<KIND>(xi[k] - sx, yi[k] - sy, zi[k] - sz, pp.per);
        const float t = ((KIND & 1) == 0) ? r2 : __builtin_amdgcn_sqrtf(r2);
        const float u = pair_u<KIND>(t, rho, kappa);
        rs[k] = fmaf(u, sg, rs[k]);
        if (COLS) cs = fmaf(u, gi[k], cs);
      }
      sx = wave_ror1(sx);
      sy = wave_ror1(sy);
      sz = wave_ror1(sz);
      sg = wave_ror1(sg);
      if (COLS) cs = wave_ror1(cs);
    }
#pragma unroll
    for (int k = 0; k < kSymTPT; ++k) racc[k] += pp.amp * (double)rs[k];
    if (COLS) part[I * npad + j] = pp.amp * (double)cs;
  }
  if (kSymSplit == 1) {
#pragma unroll
    for (int k = 0; k < kSymTPT; ++k) {
      const int64_t t = I * kSymTile + k * 64 + lane;
      if (t < npad) part[J * npad + t] = racc[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < kSymTPT; ++k) rowsum[wave][k * 64 + lane] = racc[k];
    __syncthreads();
    for (int tt = threadIdx.x; tt < kSymTile; tt += kSymThreads) {
      const int64_t t = I * kSymTile + tt;
      if (t >= npad) continue;
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < kSymSplit; ++w) sum += rowsum[w][tt];
      part[J * npad + t] = sum;
    }
  }
}

// part[s * npad + i]: slot s of node i (see above); nt = ceil(npad / (64 TPT)).
template <int KIND, int TPT, int SPLIT>
__global__ __launch_bounds__(64 * SPLIT) void k_otf_sym(const float4* __restrict__ src, const float* __restrict__ g,
                                                        int64_t npad, PairParams pp, double* __restrict__ part) {
  __shared__ double rowsum[SPLIT][64 * TPT];
  int64_t I, J;
  sym_decode(blockIdx.x, &I, &J);
  if (I == J)
    sym_tile<KIND, false, TPT, SPLIT>(src, g, npad, pp, part, I, J, rowsum);
  else
    sym_tile<KIND, true, TPT, SPLIT>(src, g, npad, pp, part, I, J, rowsum);
}

// ------------------------------------------------------------------ reductions

// Partial sums part[(s*B + b)*npad + i] of element (b, i): the symmetric
// kernel has one slot per tile, so a combine reads many slots per element;
// it reads them with L threads per element (L a power of two dividing kWG).
// Slot sums shared by a workgroup: its E = kWG / L consecutive elements each
// get L threads; thread t serves element t mod E as sub r = t / E and adds
// slots r, r + L, r + 2L, ... in order, and the sub-0 thread then adds the L
// partial sums in r order (through LDS).  The threads of a wave read
// consecutive elements of one slot row, so every load is whole cache lines
// (L lanes of one element side by side would read L rows for few elements),
// while L threads per element keep enough loads in flight.  Every thread of
// the workgroup must call it; it returns true in the thread holding an
// element's total (in *total, the element index in *idx).  C channels (slot
// arrays chstride apart, as the adjoint's four) are summed together, their
// loads in flight at once, with one barrier.  `red`: C * kWG doubles of LDS.
template <int L, int C = 1, typename PT = double>
__device__ inline bool slot_total(const PT* __restrict__ part, int64_t chstride, int nsplit, int64_t n,
                                  int64_t npad, int B, double* red, int64_t* idx, double* total) {
  constexpr int E = kWG / L;
  const int t = threadIdx.x;
  const int e = t % E, r = t / E;
  const int64_t el = (int64_t)blockIdx.x * E + e;
  const bool valid = el < n * (int64_t)B;
  double y[C];
#pragma unroll
  for (int c = 0; c < C; ++c) y[c] = 0.0;
  if (valid) {
    const int b = (int)(el / n);
    const int64_t i = el - (int64_t)b * n;
    for (int sp = r; sp < nsplit; sp += L)
#pragma unroll
      for (int c = 0; c < C; ++c) y[c] += (double)part[c * chstride + ((int64_t)sp * B + b) * npad + i];
  }
  if (L > 1) {
#pragma unroll
    for (int c = 0; c < C; ++c) red[c * kWG + t] = y[c];
    __syncthreads();
    if (r == 0) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < L; ++q) s += red[c * kWG + q * E + e];
        y[c] = s;
      }
    }
  }
  *idx = el;
#pragma unroll
  for (int c = 0; c < C; ++c) total[c] = y[c];
  return valid && r == 0;
}

// y[b*n + i] = sum of the partials of (b, i), FP64 (partials FP64, or FP32 for
// the fused split forms).  Grid: n*B*L threads.
template <int L, typename PT = double>
__global__ __launch_bounds__(kWG) void k_reduce_partials(const PT* __restrict__ part, int nsplit, int64_t n,
                                                         int64_t npad, int B, double* __restrict__ y) {
  __shared__ double red[kWG];
  int64_t idx;
  double s;
  if (slot_total<L, 1, PT>(part, 0, nsplit, n, npad, B, red, &idx, &s)) y[idx] = s;
}

// RK4 stage combination, all FP64 (L threads per (i, b), i < n; see slot_total):
//   y   = sum of partials (= K(v_s)),  k = -v_s + y
//   s=1: ksum = k,        v <- u + dt/2 k
//   s=2: ksum += 2k,      v <- u + dt/2 k
//   s=3: ksum += 2k,      v <- u + dt k
//   s=4: u <- u + dt/6 (ksum + k),  v <- u
// then g[b*npad + i] = s_i f_b(v) for the next stage (s_i = q_i or 1).
// k1_out (may be null) receives k_1 = F(u_n) at stage 1 (the Adams-Bashforth start-up records it);
// gamma (may be null) is a forcing term added to k (B x n, at this stage's time).
struct Rk4Stage {
  int stage;
  double dt;
  double* u;
  double* v;
  double* ksum;
  const double* qd;
  int with_q;
  Firing fr;
  double* k1_out;
  const double* gamma;
};

// Values of element idx = (b, i) that the stage update reads, loaded ahead
// of time by kernels that can hide their latency behind the pair sum.
struct Rk4Pre {
  double v, u, ksum, gamma, q;
};

__device__ inline Rk4Pre rk4_preload(const Rk4Stage& st, int64_t idx, int64_t i) {
  Rk4Pre p;
  p.v = st.v[idx];
  p.u = st.u[idx];
  p.ksum = st.stage > 1 ? st.ksum[idx] : 0.0;
  p.gamma = st.gamma ? st.gamma[idx] : 0.0;
  p.q = st.with_q ? st.qd[i] : 1.0;
  return p;
}

// The update of element idx = (b, i) from its pair sum y (see above), with
// its operands already loaded.
__device__ inline void rk4_update_from(const Rk4Stage& st, const Rk4Pre& p, int64_t idx, int b, int64_t i,
                                       int64_t npad, double y, float* __restrict__ g) {
  const int stage = st.stage;
  const double dt = st.dt;
  const Firing& fr = st.fr;
  const double k = -p.v + y + p.gamma;
  double ui = p.u;
  double vn;
  if (stage == 1) {
    if (st.k1_out) st.k1_out[idx] = k;
    st.ksum[idx] = k;
    vn = ui + 0.5 * dt * k;
  } else if (stage == 2) {
    st.ksum[idx] = p.ksum + 2.0 * k;
    vn = ui + 0.5 * dt * k;
  } else if (stage == 3) {
    st.ksum[idx] = p.ksum + 2.0 * k;
    vn = ui + dt * k;
  } else {
    ui = ui + (dt / 6.0) * (p.ksum + k);
    st.u[idx] = ui;
    vn = ui;
  }
  st.v[idx] = vn;
  g[(int64_t)b * npad + i] = (float)(p.q * sigmoid(vn, fr.beta, state_theta(fr, b)));
}

// The update of element idx = (b, i) from its pair sum y (see above).
__device__ inline void rk4_update(const Rk4Stage& st, int64_t idx, int b, int64_t i, int64_t npad, double y,
                                  float* __restrict__ g) {
  rk4_update_from(st, rk4_preload(st, idx, i), idx, b, i, npad, y, g);
}

template <int L>
__global__ __launch_bounds__(kWG) void k_rk4_combine(const double* __restrict__ part, int nsplit, int64_t n,
                                                     int64_t npad, int B, Rk4Stage st, float* __restrict__ g) {
  __shared__ double red[kWG];
  int64_t idx;
  double y;
  if (!slot_total<L>(part, 0, nsplit, n, npad, B, red, &idx, &y)) return;
  const int b = (int)(idx / n);
  const int64_t i = idx - (int64_t)b * n;
  rk4_update(st, idx, b, i, npad, y, g);
}

// Pair sum of one state for small problems (a few thousand nodes), where the
// symmetric kernel has too few tile pairs to fill the chip: every target-
// source pair is evaluated once (twice the symmetric kernel's evaluations),
// but a workgroup owns only kSmallRows targets, so N = 2000 gives 512
// workgroups (4 targets each: at N = 1000 / 2000 / 4096 an RK4 step took
// 18.5 / 25.7 / 43.4 us, against 21.7 / 28.8 / 44.5 with 8 targets, 18.3 /
// 25.7 / 46.3 with 2 and 29.7 / 39.6 / 58.2 with 16).  Thread t takes
// sources t, t + kWG, ...; for each target it sums
// its sources in FP32; the threads' sums are then added in FP64 in a fixed
// tree (xor butterfly within a wave, then the waves in order), so the result
// is reproducible.  Without STAGE: part[i] = y_i, one slot per node.  With
// STAGE the workgroup applies the RK4 stage update of k_rk4_combine to its
// own targets straight away (one launch per stage, y added as the one-slot
// combine adds it); the next stage's sources then go to g_next, a second
// buffer, because other workgroups may still be reading g.
#ifndef NFR_SMALL_ROWS
#define NFR_SMALL_ROWS 4
#endif
constexpr int kSmallRows = NFR_SMALL_ROWS;

template <int KIND, bool STAGE>
__global__ __launch_bounds__(kWG) void k_otf_small(const float4* __restrict__ src, const float* __restrict__ g,
                                                   int64_t n, int64_t npad, PairParams pp, double* __restrict__ part,
                                                   Rk4Stage st, float* __restrict__ g_next) {
  __shared__ double red[kWG / 64][kSmallRows];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * kSmallRows;
  // the stage update's operands of this workgroup's targets, loaded now so
  // their latency hides behind the pair sum
  const int64_t ti = r0 + threadIdx.x;
  const bool updater = STAGE && threadIdx.x < kSmallRows && ti < n;
  Rk4Pre pre{};
  if (updater) pre = rk4_preload(st, ti, ti);
  float tx[kSmallRows], ty[kSmallRows], tz[kSmallRows], acc[kSmallRows];
#pragma unroll
  for (int r = 0; r < kSmallRows; ++r) {
    const float4 p = src[r0 + r];
    tx[r] = p.x * pp.sig;
    ty[r] = p.y * pp.sig;
    tz[r] = p.z * pp.sig;
    acc[r] = 0.0f;
  }
  // thread t takes sources t, t + kWG, ... (npad is a multiple of kWG) in
  // order: batches of 8, then of 4, then single sources, each batch's loads
  // issued together before any of its evaluations (no branch inside a batch)
  const int cnt = (int)(npad / kWG);
  auto batch = [&](auto nb_tag, int k0) {
    constexpr int NBT = decltype(nb_tag)::value;
    float4 s4[NBT];
    float sg[NBT];
#pragma unroll
    for (int e = 0; e < NBT; ++e) {
      const int64_t j = threadIdx.x + (int64_t)(k0 + e) * kWG;
      s4[e] = src[j];
      sg[e] = g[j];
    }
#pragma unroll
    for (int e = 0; e < NBT; ++e) {
      const float sx = s4[e].x * pp.sig, sy = s4[e].y * pp.sig, sz = s4[e].z * pp.sig;
#pragma unroll
      for (int r = 0; r < kSmallRows; ++r) {
        const float r2 = pair_r2<KIND>(tx[r] - sx, ty[r] - sy, tz[r] - sz, pp.per);
        const float t = ((KIND & 1) == 0) ? r2 : __builtin_amdgcn_sqrtf(r2);
        acc[r] = fmaf(pair_u<KIND>(t, pp.rho, pp.kappa), sg[e], acc[r]);
      }
    }
  };
  int k0 = 0;
  for (; k0 + 8 <= cnt; k0 += 8) batch(std::integral_constant<int, 8>{}, k0);
  if (k0 + 4 <= cnt) {
    batch(std::integral_constant<int, 4>{}, k0);
    k0 += 4;
  }
  for (; k0 < cnt; ++k0) batch(std::integral_constant<int, 1>{}, k0);
  double d[kSmallRows];
#pragma unroll
  for (int r = 0; r < kSmallRows; ++r) d[r] = wave_sum_f64((double)acc[r]);
  if (lane == 63)
#pragma unroll
    for (int r = 0; r < kSmallRows; ++r) red[wave][r] = d[r];
  __syncthreads();
  if (threadIdx.x < kSmallRows) {
    double y = 0.0;
#pragma unroll
    for (int w = 0; w < kWG / 64; ++w) y += red[w][threadIdx.x];
    const int64_t i = r0 + threadIdx.x;
    if (!STAGE) {
      part[i] = pp.amp * y;
    } else if (updater) {
      double ys = 0.0;            // as slot_total adds the single slot
      ys += pp.amp * y;
      rk4_update_from(st, pre, i, 0, i, npad, ys, g_next);
    } else {
      g_next[i] = 0.0f;           // padding sources stay zero in both buffers
    }
  }
}

// ------------------------------------------------------------------ Adams-Bashforth 5

// Weights of F_n, F_{n-1}, ..., F_{n-4} (times dt) of the five-step Adams-Bashforth method.
struct Ab5Weights {
  double a[5];
};

// One AB5 step (one thread per (i, b), i < n), all FP64:
//   F_n = -u_n + y (y = sum of partials),  hist[slot(n)] = F_n,
//   u_{n+1} = u_n + dt sum_k a_k hist[slot(n - k)],
// then g[b*npad + i] = s_i f_b(u_{n+1}).  hist holds 5 arrays of n*B; slots[k]
// is the array holding F_{n-k}.
template <int L>
__global__ __launch_bounds__(kWG) void k_ab5_combine(const double* __restrict__ part, int nsplit, int64_t n,
                                                     int64_t npad, int B, double dt, Ab5Weights wt, int4 slots03,
                                                     int slot4, double* __restrict__ u, double* __restrict__ hist,
                                                     const double* __restrict__ qd, int with_q, Firing fr,
                                                     float* __restrict__ g) {
  __shared__ double red[kWG];
  const int64_t nb = n * (int64_t)B;
  int64_t idx;
  double y;
  if (!slot_total<L>(part, 0, nsplit, n, npad, B, red, &idx, &y)) return;
  const int b = (int)(idx / n);
  const int64_t i = idx - (int64_t)b * n;
  const double ui = u[idx];
  const double F = -ui + y;
  hist[slots03.x * nb + idx] = F;
  const double incr = wt.a[0] * F + wt.a[1] * hist[slots03.y * nb + idx] + wt.a[2] * hist[slots03.z * nb + idx] +
                      wt.a[3] * hist[slots03.w * nb + idx] + wt.a[4] * hist[(int64_t)slot4 * nb + idx];
  const double un = ui + dt * incr;
  u[idx] = un;
  const double s = with_q ? qd[i] : 1.0;
  g[(int64_t)b * npad + i] = (float)(s * sigmoid(un, fr.beta, state_theta(fr, b)));
}

// ------------------------------------------------------------------ synaptic depression

// Neural field with synaptic depression (paper section 5.2, eq. nfsyndep): the
// sources carry the presynaptic efficacy a,
//   u' = -u + K(u, a),  K_i = sum_j w_ij q_j a_j f(u_j),   tau a' = 1 - a - beta_d a f(u).
// g[b*npad + j] = q_j a_j f_b(u_j) (zero on padding); copies u, a into the stage inputs.
__global__ __launch_bounds__(kWG) void k_syndep_prep(const double* __restrict__ u, const double* __restrict__ a,
                                                     int64_t n, int64_t npad, int B, const double* __restrict__ qd,
                                                     Firing fr, float* __restrict__ g, double* __restrict__ vu,
                                                     double* __restrict__ va) {
  const int64_t idx = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (idx >= npad * (int64_t)B) return;
  const int b = (int)(idx / npad);
  const int64_t j = idx - (int64_t)b * npad;
  float out = 0.0f;
  if (j < n) {
    const int64_t e = (int64_t)b * n + j;
    const double uj = u[e], aj = a[e];
    vu[e] = uj;
    va[e] = aj;
    out = (float)(qd[j] * aj * sigmoid(uj, fr.beta, state_theta(fr, b)));
  }
  g[idx] = out;
}

// RK4 stage combination of the coupled (u, a) system, all FP64; next sources
// g = q a f(u) at the new stage input.
template <int L>
__global__ __launch_bounds__(kWG) void k_syndep_combine(const double* __restrict__ part, int nsplit, int64_t n,
                                                        int64_t npad, int B, int stage, double dt, double inv_tau,
                                                        double beta_d, double* __restrict__ u, double* __restrict__ a,
                                                        double* __restrict__ vu, double* __restrict__ va,
                                                        double* __restrict__ ku_sum, double* __restrict__ ka_sum,
                                                        const double* __restrict__ qd, Firing fr,
                                                        float* __restrict__ g) {
  __shared__ double red[kWG];
  int64_t idx;
  double y;
  if (!slot_total<L>(part, 0, nsplit, n, npad, B, red, &idx, &y)) return;
  const int b = (int)(idx / n);
  const int64_t i = idx - (int64_t)b * n;
  const double th = state_theta(fr, b);
  const double cu = vu[idx], ca = va[idx];
  const double ku = -cu + y;
  const double ka = (1.0 - ca - beta_d * ca * sigmoid(cu, fr.beta, th)) * inv_tau;
  double ui = u[idx], ai = a[idx];
  double nu, na;
  if (stage == 1) {
    ku_sum[idx] = ku;
    ka_sum[idx] = ka;
    nu = ui + 0.5 * dt * ku;
    na = ai + 0.5 * dt * ka;
  } else if (stage == 2 || stage == 3) {
    ku_sum[idx] += 2.0 * ku;
    ka_sum[idx] += 2.0 * ka;
    const double c = stage == 2 ? 0.5 * dt : dt;
    nu = ui + c * ku;
    na = ai + c * ka;
  } else {
    ui = ui + (dt / 6.0) * (ku_sum[idx] + ku);
    ai = ai + (dt / 6.0) * (ka_sum[idx] + ka);
    u[idx] = ui;
    a[idx] = ai;
    nu = ui;
    na = ai;
  }
  vu[idx] = nu;
  va[idx] = na;
  g[(int64_t)b * npad + i] = (float)(qd[i] * na * sigmoid(nu, fr.beta, th));
}

// ------------------------------------------------------------------ W form (FP32)

struct KernelF64 {
  int kind;
  double Ae, se, Ai, si;
  double period;   // > 0: periodic problem (x, y reduced to one period window)
};

// Squared distance in FP64, with the per-axis nearest image of a periodic problem.
__device__ inline double pair_r2_64(const KernelF64& k, double dx, double dy, double dz) {
  if (k.period > 0.0) {
    dx = fabs(dx);
    dx = fmin(dx, k.period - dx);
    dy = fabs(dy);
    dy = fmin(dy, k.period - dy);
  }
  return dx * dx + dy * dy + dz * dz;
}

__device__ inline double kernel_w64(const KernelF64& k, double r2) {
  if (k.kind == 0) return k.Ae * exp(-r2 / (k.se * k.se)) - k.Ai * exp(-r2 / (k.si * k.si));
  const double r = sqrt(r2);
  return k.Ae * exp(-r / k.se) - k.Ai * exp(-r / k.si);
}

// W[i*npad + j] = w(|x_i - x_j|) q_j, FP64 arithmetic rounded once to FP32;
// rows i < n, columns j < npad (zero where q_j = 0).
// Grid: x = rows, y = column blocks of kWG.
__global__ __launch_bounds__(kWG) void k_w_build_f32(const double* __restrict__ xyz64, const double* __restrict__ qd,
                                                     int64_t n, int64_t npad, KernelF64 kp, float* __restrict__ W) {
  const int64_t i = blockIdx.x;
  const int64_t j = (int64_t)blockIdx.y * kWG + threadIdx.x;
  if (i >= n || j >= npad) return;
  const double r2 = pair_r2_64(kp, xyz64[3 * i] - xyz64[3 * j], xyz64[3 * i + 1] - xyz64[3 * j + 1],
                               xyz64[3 * i + 2] - xyz64[3 * j + 2]);
  const double wq = qd[j] == 0.0 ? 0.0 : kernel_w64(kp, r2) * qd[j];
  W[i * npad + j] = (float)wq;
}

// Row-blocked GEMV / small GEMM with W streamed from HBM:
//   part[(split*B + b)*npad + i] = sum_{j in chunk(split)} W[i*npad + j] G[b*npad + j]
// WG = 4 waves, each wave owns kRowsPerWave rows; a column step of kColStep
// stages G in LDS, every lane loads two float4 per row (coalesced 1 KB rows per
// wave instruction).  Lane partials are FP32 per column step, folded into FP64,
// then reduced across the wave in FP64.
constexpr int kRowsPerWave = 4;
constexpr int kGemvRows = 4 * kRowsPerWave;  // rows per workgroup
constexpr int kColStep = 2048;

template <int BS>
__global__ __launch_bounds__(kWG) void k_w_gemv_f32(const float* __restrict__ W, const float* __restrict__ G,
                                                    int64_t n, int64_t npad, int B, int64_t chunk,
                                                    double* __restrict__ part) {
  __shared__ float4 s_g[BS][kColStep / 4];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * kGemvRows + wave * kRowsPerWave;
  const int split = blockIdx.y;
  const int b0 = blockIdx.z * BS;
  const int64_t c_begin = (int64_t)split * chunk;
  int64_t c_end = c_begin + chunk;
  if (c_end > npad) c_end = npad;

  double acc[kRowsPerWave][BS];
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r)
#pragma unroll
    for (int b = 0; b < BS; ++b) acc[r][b] = 0.0;

  const f32x4* W4 = reinterpret_cast<const f32x4*>(W);
  const int64_t ld4 = npad / 4;

  for (int64_t c0 = c_begin; c0 < c_end; c0 += kColStep) {
    const int64_t cols = (c_end - c0) < kColStep ? (c_end - c0) : kColStep;   // multiple of 256
    const int64_t q4 = cols / 4;
    for (int e = threadIdx.x; e < kColStep / 4; e += kWG) {
#pragma unroll
      for (int b = 0; b < BS; ++b) {
        float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
        if (e < q4 && b0 + b < B) val = reinterpret_cast<const float4*>(G + (int64_t)(b0 + b) * npad + c0)[e];
        s_g[b][e] = val;
      }
    }
    __syncthreads();
    float pa[kRowsPerWave][BS];
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r)
#pragma unroll
      for (int b = 0; b < BS; ++b) pa[r][b] = 0.0f;
#pragma unroll
    for (int h = 0; h < kColStep / 4 / 64; ++h) {
      const int e = h * 64 + lane;
      if (e < q4) {
        float4 wv[kRowsPerWave];
#pragma unroll
        for (int r = 0; r < kRowsPerWave; ++r) {
          const int64_t row = row0 + r;
          if (row < n) {
            const f32x4 t = __builtin_nontemporal_load(&W4[row * ld4 + c0 / 4 + e]);
            wv[r] = make_float4(t.x, t.y, t.z, t.w);
          } else {
            wv[r] = make_float4(0.f, 0.f, 0.f, 0.f);
          }
        }
#pragma unroll
        for (int b = 0; b < BS; ++b) {
          const float4 gv = s_g[b][e];
#pragma unroll
          for (int r = 0; r < kRowsPerWave; ++r) {
            float s = pa[r][b];
            s = fmaf(wv[r].x, gv.x, s);
            s = fmaf(wv[r].y, gv.y, s);
            s = fmaf(wv[r].z, gv.z, s);
            s = fmaf(wv[r].w, gv.w, s);
            pa[r][b] = s;
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r)
#pragma unroll
      for (int b = 0; b < BS; ++b) acc[r][b] += (double)pa[r][b];
  }

#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r)
#pragma unroll
    for (int b = 0; b < BS; ++b) {
      double s = acc[r][b];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      acc[r][b] = s;
    }
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) {
      const int64_t row = row0 + r;
      if (row >= npad) continue;
#pragma unroll
      for (int b = 0; b < BS; ++b)
        if (b0 + b < B) part[((int64_t)split * B + b0 + b) * npad + row] = row < n ? acc[r][b] : 0.0;
    }
  }
}

}  // namespace nfr
