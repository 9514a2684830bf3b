// Discrete adjoint of the RK4 trajectory (single state).
//
// Forward step (paper eq. NFODETilde, classical RK4):
//   G(v)_i = -v_i + sum_j w_ij q_j f(v_j),  k_s = G(v_s),  u_{n+1} = u_n + dt/6 (k_1 + 2 k_2 + 2 k_3 + k_4).
// Reverse step, given ubar = dL/du_{n+1}:
//   lambda_4 = dt/6 ubar;  for s = 4, 3, 2, 1:
//     z_j      = sum_i w_ij lambda_i                      (w symmetric: the transposed sum)
//     vbar_s,j = -lambda_j + q_j f'(v_s,j) z_j,   u_n-bar += vbar_s
//     lambda_3 = dt/3 ubar + dt vbar_4,  lambda_2 = dt/3 ubar + dt/2 vbar_3,  lambda_1 = dt/6 ubar + dt/2 vbar_2
//   parameter cotangents at every stage: sum_j g_j sum_i lambda_i dw_ij/dp with g_j = q_j f(v_s,j),
//   and for the threshold -sum_j q_j f'(v_s,j) z_j.
// The pair kernel accumulates, per target j, the raw sums
//   S1 = sum_i lambda_i e1_ij,  S2 = sum_i lambda_i e2_ij,  T1 = sum_i lambda_i e1_ij t_ij,  T2 = sum_i lambda_i e2_ij t_ij
// with e1 = exp2(-t), e2 = exp2(-rho t) and t the scaled distance of the
// forward kernel; the combine turns them into z and the parameter terms.
#pragma once

#include "common.h"
#include "kernels_core.h"

namespace nfr {

// Symmetric transpose sum: every term of S1, S2, T1, T2 is symmetric in
// (i, j), so the tile-pair scheme of the forward symmetric kernel applies
// (kernels_core.h: tile pairs I <= J, the targets of tile I held kSymTPT per lane,
// source groups of J split over the waves, sources rotated by DPP carrying
// their column accumulators), here with four channels weighted by lambda.
// Slots: part[(c * nt + s) * npad + i] for channel c, slot s (the row sums of
// (I, J) go to slot J of the nodes of I, the column sums to slot I of the
// nodes of J).  The coordinates are in the forward kernel's units (t the
// excitatory argument); with rho = 1/m they are in units of the inhibitory
// length instead, t the inhibitory argument, e2 = exp2(-t) and e1 = e2^m, and
// the T channels hold sum lambda e t_i = T / m.
// Waves per workgroup of the transpose kernel (they split a tile's source
// groups like the forward kernel's; one group per wave measured fastest at
// N = 16384: 1, 2, 4 waves took 0.089, 0.082, 0.077 ms per pair launch).
#ifndef NFR_ADJ_SPLIT
#define NFR_ADJ_SPLIT 4
#endif
constexpr int kAdjSplit = NFR_ADJ_SPLIT;
constexpr int kAdjThreads = 64 * kAdjSplit;

template <int KIND, bool COLS>
__device__ inline void sym_adj_tile(const float4* __restrict__ src, const float* __restrict__ lam, int64_t npad,
                                    int nt, const PairParams& pp, double* __restrict__ part, int64_t I, int64_t J,
                                    double (*rowsum)[4][kSymTile]) {
  static_assert(kSymTile == 64 * kSymTPT, "one wave holds the tile's targets");
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const float rho = pp.rho;
  float xi[kSymTPT], yi[kSymTPT], zi[kSymTPT], li[kSymTPT];
#pragma unroll
  for (int k = 0; k < kSymTPT; ++k) {
    const int64_t t = I * kSymTile + k * 64 + lane;
    const int64_t tc = t < npad ? t : npad - 1;
    const float4 p = src[tc];
    xi[k] = p.x * pp.sig;
    yi[k] = p.y * pp.sig;
    zi[k] = p.z * pp.sig;
    li[k] = t < npad ? lam[t] : 0.0f;
  }
  double racc[kSymTPT][4];
#pragma unroll
  for (int k = 0; k < kSymTPT; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) racc[k][c] = 0.0;

  int64_t nsrc = npad - J * kSymTile;
  if (nsrc > kSymTile) nsrc = kSymTile;
  const int ngroups = (int)(nsrc / 64);
  for (int grp = wave; grp < ngroups; grp += kAdjSplit) {
    const int64_t j = J * kSymTile + grp * 64 + lane;
    const float4 s4 = src[j];
    float sx = s4.x * pp.sig, sy = s4.y * pp.sig, sz = s4.z * pp.sig, sl = lam[j];
    float col[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float acc[kSymTPT][4];
#pragma unroll
    for (int k = 0; k < kSymTPT; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[k][c] = 0.0f;
#pragma unroll 2
    for (int step = 0; step < 64; ++step) {
#pragma unroll
      for (int k = 0; k < kSymTPT; ++k) {
        const float r2 = pair_r2<KIND>(xi[k] - sx, yi[k] - sy, zi[k] - sz, pp.per);
        const float t = ((KIND & 1) == 0) ? r2 : __builtin_amdgcn_sqrtf(r2);
        // with rho = 1/m the coordinates are in units of the inhibitory length
        // (t is the inhibitory argument; the combine scales T1, T2 by m)
        const float e2 = sym_pow<KIND>() == 0 ? __builtin_amdgcn_exp2f(-(t * rho)) : __builtin_amdgcn_exp2f(-t);
        const float e1 = sym_pow<KIND>() == 0 ? __builtin_amdgcn_exp2f(-t) : ipow<sym_pow<KIND>()>(e2);
        const float e1t = e1 * t;
        const float e2t = e2 * t;
        acc[k][0] = fmaf(e1, sl, acc[k][0]);
        acc[k][1] = fmaf(e2, sl, acc[k][1]);
        acc[k][2] = fmaf(e1t, sl, acc[k][2]);
        acc[k][3] = fmaf(e2t, sl, acc[k][3]);
        if (COLS) {
          col[0] = fmaf(e1, li[k], col[0]);
          col[1] = fmaf(e2, li[k], col[1]);
          col[2] = fmaf(e1t, li[k], col[2]);
          col[3] = fmaf(e2t, li[k], col[3]);
        }
      }
      sx = wave_ror1(sx);
      sy = wave_ror1(sy);
      sz = wave_ror1(sz);
      sl = wave_ror1(sl);
      if (COLS) {
#pragma unroll
        for (int c = 0; c < 4; ++c) col[c] = wave_ror1(col[c]);
      }
    }
#pragma unroll
    for (int k = 0; k < kSymTPT; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) racc[k][c] += (double)acc[k][c];
    if (COLS) {
#pragma unroll
      for (int c = 0; c < 4; ++c) part[((int64_t)c * nt + I) * npad + j] = (double)col[c];
    }
  }
  if (kAdjSplit > 1) {
#pragma unroll
    for (int k = 0; k < kSymTPT; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) rowsum[wave][c][k * 64 + lane] = racc[k][c];
    __syncthreads();
    for (int tt = threadIdx.x; tt < kSymTile; tt += kAdjThreads) {
      const int64_t t = I * kSymTile + tt;
      if (t >= npad) continue;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < kAdjSplit; ++w) sum += rowsum[w][c][tt];
        part[((int64_t)c * nt + J) * npad + t] = sum;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < kSymTPT; ++k) {
      const int64_t t = I * kSymTile + k * 64 + lane;
      if (t >= npad) continue;
#pragma unroll
      for (int c = 0; c < 4; ++c) part[((int64_t)c * nt + J) * npad + t] = racc[k][c];
    }
  }
}

// One launch per reverse stage: nt (nt + 1) / 2 workgroups, nt = ceil(npad / kSymTile).
template <int KIND>
__global__ __launch_bounds__(kAdjThreads) void k_sym_adjoint(const float4* __restrict__ src,
                                                             const float* __restrict__ lam, int64_t npad, int nt,
                                                             PairParams pp, double* __restrict__ part) {
  __shared__ double rowsum[kAdjSplit][4][kSymTile];
  int64_t I, J;
  sym_decode(blockIdx.x, &I, &J);
  if (I == J)
    sym_adj_tile<KIND, false>(src, lam, npad, nt, pp, part, I, J, rowsum);
  else
    sym_adj_tile<KIND, true>(src, lam, npad, nt, pp, part, I, J, rowsum);
}

// Coefficients turning the raw sums into dw/dp terms:
//   sum_i lambda_i dw_ij/dA_e = S1,   dw/dA_i -> -S2,
//   sum_i lambda_i dw_ij/ds_e = A_e kse T1,   dw/ds_i -> -A_i ksi T2, with
//   exponential: kse = 1 / (s_e log2 e),       ksi = s_e / (s_i^2 log2 e)
//   Gaussian:    kse = 2 / (s_e log2 e),       ksi = 2 s_e^2 / (s_i^3 log2 e).
struct AdjCoef {
  double Ae, Ai, kse, ksi;
};

// lambda_4 = dt/6 ubar (FP64 and FP32 copies; FP32 padding zeroed), unbar = ubar.
__global__ __launch_bounds__(kWG) void k_adj_init(const double* __restrict__ ubarT, int64_t n, int64_t npad, double dt,
                                                  double* __restrict__ ubar, double* __restrict__ unbar,
                                                  double* __restrict__ lam, float* __restrict__ lam32) {
  const int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (j >= npad) return;
  if (j < n) {
    const double ub = ubarT[j];
    ubar[j] = ub;
    unbar[j] = ub;
    lam[j] = dt / 6.0 * ub;
    lam32[j] = (float)(dt / 6.0 * ub);
  } else {
    lam32[j] = 0.0f;
  }
}

// One reverse stage (L threads per node j < n, see slot_total); see the file comment.  Block
// partial sums of the five parameter terms are added to pblk[block * 8 + c]
// by thread 0 of the block (the launches are ordered on one stream, so the
// accumulation order is fixed).
template <int L>
__global__ __launch_bounds__(kWG) void k_adj_combine(const double* __restrict__ part, int nsplit, int64_t n,
                                                     int64_t npad, int stage, double dt, AdjCoef co,
                                                     const double* __restrict__ qd, Firing fr,
                                                     const double* __restrict__ vs, double* __restrict__ ubar,
                                                     double* __restrict__ unbar, double* __restrict__ lam,
                                                     float* __restrict__ lam32, double* __restrict__ pblk) {
  __shared__ double red[5][kWG];
  __shared__ double sred[4 * kWG];    // slot sums of the four channels (not shared with red)
  int64_t j = 0;
  double S[4];
  const bool lead = slot_total<L, 4>(part, (int64_t)nsplit * npad, nsplit, n, npad, 1, sred, &j, S);
  double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0, c4 = 0.0;
  if (lead) {
    const double z = co.Ae * S[0] - co.Ai * S[1];
    const double f = sigmoid(vs[j], fr.beta, fr.theta);
    const double fp = fr.beta * f * (1.0 - f);
    const double q = qd[j];
    const double vbar = -lam[j] + q * fp * z;
    const double un = unbar[j] + vbar;
    unbar[j] = un;
    const double g = q * f;
    c0 = g * S[0];
    c1 = g * co.Ae * co.kse * S[2];
    c2 = -g * S[1];
    c3 = -g * co.Ai * co.ksi * S[3];
    c4 = -q * fp * z;
    const double ub = ubar[j];
    double ln;
    if (stage == 4) {
      ln = dt / 3.0 * ub + dt * vbar;
    } else if (stage == 3) {
      ln = dt / 3.0 * ub + 0.5 * dt * vbar;
    } else if (stage == 2) {
      ln = dt / 6.0 * ub + 0.5 * dt * vbar;
    } else {
      ubar[j] = un;           // dL/du_n: the next reverse step starts from it
      ln = dt / 6.0 * un;
    }
    lam[j] = ln;
    lam32[j] = (float)ln;
  }
  red[0][threadIdx.x] = c0;
  red[1][threadIdx.x] = c1;
  red[2][threadIdx.x] = c2;
  red[3][threadIdx.x] = c3;
  red[4][threadIdx.x] = c4;
  __syncthreads();
  for (int s = kWG / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
#pragma unroll
      for (int c = 0; c < 5; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int c = 0; c < 5; ++c) pblk[(int64_t)blockIdx.x * 8 + c] += red[c][0];
}

// Zero-fills n doubles (used instead of a memset so the sequence stays a plain
// chain of kernels).
__global__ __launch_bounds__(kWG) void k_fill_zero(double* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// pbar[c] = sum over blocks (in order) of pblk[block * 8 + c], c < 5.  One wave.
__global__ __launch_bounds__(64) void k_adj_finalize(const double* __restrict__ pblk, int64_t nblocks,
                                                     double* __restrict__ pbar) {
  if (threadIdx.x < 5) {
    double s = 0.0;
    for (int64_t b = 0; b < nblocks; ++b) s += pblk[b * 8 + threadIdx.x];
    pbar[threadIdx.x] = s;
  }
}

}  // namespace nfr
