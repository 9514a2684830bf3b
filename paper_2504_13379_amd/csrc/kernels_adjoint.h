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

namespace nfr {

constexpr int kAdjTPT = 4;

template <int KIND>
__global__ __launch_bounds__(kWG) void k_otf_adjoint(const float4* __restrict__ src, const float* __restrict__ lam,
                                                     int64_t npad, int64_t chunk, int nsplit, PairParams pp,
                                                     double* __restrict__ part) {
  __shared__ float4 s_src[kWG];
  const int tid = threadIdx.x;
  const int64_t tbase = (int64_t)blockIdx.x * (kWG * kAdjTPT);
  const int split = blockIdx.y;
  float xi[kAdjTPT], yi[kAdjTPT], zi[kAdjTPT];
#pragma unroll
  for (int k = 0; k < kAdjTPT; ++k) {
    int64_t t = tbase + tid + (int64_t)kWG * k;
    if (t >= npad) t = npad - 1;
    const float4 p = src[t];
    xi[k] = p.x * pp.sig;
    yi[k] = p.y * pp.sig;
    zi[k] = p.z * pp.sig;
  }
  double acc[kAdjTPT][4];
#pragma unroll
  for (int k = 0; k < kAdjTPT; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[k][c] = 0.0;
  const int64_t j_begin = (int64_t)split * chunk;
  int64_t j_end = j_begin + chunk;
  if (j_end > npad) j_end = npad;
  const float rho = pp.rho;
  for (int64_t j0 = j_begin; j0 < j_end; j0 += kWG) {
    {
      const float4 s = src[j0 + tid];
      s_src[tid] = make_float4(s.x * pp.sig, s.y * pp.sig, s.z * pp.sig, lam[j0 + tid]);
    }
    __syncthreads();
    float a[kAdjTPT][4];
#pragma unroll
    for (int k = 0; k < kAdjTPT; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) a[k][c] = 0.0f;
#pragma unroll 4
    for (int jj = 0; jj < kWG; ++jj) {
      const float4 s = s_src[jj];
#pragma unroll
      for (int k = 0; k < kAdjTPT; ++k) {
        const float r2 = pair_r2<KIND>(xi[k] - s.x, yi[k] - s.y, zi[k] - s.z, pp.per);
        const float t = ((KIND & 1) == 0) ? r2 : __builtin_amdgcn_sqrtf(r2);
        const float e1 = __builtin_amdgcn_exp2f(-t);
        const float e2 = __builtin_amdgcn_exp2f(-(t * rho));
        const float l1 = e1 * s.w;
        const float l2 = e2 * s.w;
        a[k][0] += l1;
        a[k][1] += l2;
        a[k][2] = fmaf(l1, t, a[k][2]);
        a[k][3] = fmaf(l2, t, a[k][3]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kAdjTPT; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[k][c] += (double)a[k][c];
  }
#pragma unroll
  for (int k = 0; k < kAdjTPT; ++k) {
    const int64_t t = tbase + tid + (int64_t)kWG * k;
    if (t >= npad) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) part[((int64_t)c * nsplit + split) * npad + t] = acc[k][c];
  }
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

// One reverse stage (one thread per node j < n); see the file comment.  Block
// partial sums of the five parameter terms are added to pblk[block * 8 + c]
// by thread 0 of the block (the launches are ordered on one stream, so the
// accumulation order is fixed).
__global__ __launch_bounds__(kWG) void k_adj_combine(const double* __restrict__ part, int nsplit, int64_t n,
                                                     int64_t npad, int stage, double dt, AdjCoef co,
                                                     const double* __restrict__ qd, Firing fr,
                                                     const double* __restrict__ vs, double* __restrict__ ubar,
                                                     double* __restrict__ unbar, double* __restrict__ lam,
                                                     float* __restrict__ lam32, double* __restrict__ pblk) {
  __shared__ double red[5][kWG];
  const int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x;
  double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0, c4 = 0.0;
  if (j < n) {
    double S[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double s = 0.0;
      for (int sp = 0; sp < nsplit; ++sp) s += part[((int64_t)c * nsplit + sp) * npad + j];
      S[c] = s;
    }
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
