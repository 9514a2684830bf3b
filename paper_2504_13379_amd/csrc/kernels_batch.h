// Uneven batch: many problems (different N, kernel parameters, firing rates
// and state counts) advanced together, one persistent pair-sum launch and one
// combine launch per RK4 stage for the whole batch.
//
// Work items are (problem, target tile of kWG * batch_tpt(bs) targets, source
// chunk, state block); they are sorted by decreasing cost on the host and a fixed grid of
// workgroups walks them round-robin, so every stage is a single launch whose
// largest items start first.
#pragma once

#include "common.h"
#include "kernels_core.h"

namespace nfr {

struct BatchProblemDev {
  const float4* src;
  const double* q;
  int64_t n, npad;
  int B, bs, kind, nsplit;   // kind: pair-kernel code (kernel kind, + 2 if periodic)
  int64_t chunk;
  PairParams pp;
  Firing fr;
  float* g;        // B x npad
  double* part;    // nsplit x B x npad
  double* u;       // B x n (caller's state)
  double* v;       // B x n
  double* ksum;    // B x n
  int64_t elem_off;   // prefix sum of n * B
  int64_t gel_off;    // prefix sum of npad * B
};

struct BatchItem {
  int p;
  int tile;
  int split;
  int sb;
};

// State block of a problem with B states (1, 4 or 16; see batch_tpt for the
// targets per thread that go with it).
__host__ __device__ constexpr int batch_bs(int B) { return B == 1 ? 1 : (B <= 4 ? 4 : 16); }

// Targets per thread of a batch item with state block bs.  One kernel serves
// every block size and takes the register allocation of the largest, so the
// two targets per thread that the single-problem 16-state sum uses (201
// registers) would cut the occupancy of every item; one target (148
// registers) is faster over the uneven batch (1.39e13 against 1.30e13
// pair-interactions/s).
#ifndef NFR_BATCH_TPT16
#define NFR_BATCH_TPT16 1
#endif
__host__ __device__ constexpr int batch_tpt(int bs) { return bs == 16 ? NFR_BATCH_TPT16 : otf_tpt(bs); }

template <int KIND>
__device__ inline void batch_item(const BatchProblemDev& P, const BatchItem& w, float4* s_src, float (*s_g)[kWG]) {
  if (P.bs == 1)
    otf_tile<KIND, batch_tpt(1), 1>(P.src, P.g, P.npad, P.B, P.chunk, P.pp, P.part, w.tile, w.split, w.sb, s_src, s_g);
  else if (P.bs == 4)
    otf_tile<KIND, batch_tpt(4), 4>(P.src, P.g, P.npad, P.B, P.chunk, P.pp, P.part, w.tile, w.split, w.sb * 4, s_src,
                                  s_g);
  else
    otf_tile<KIND, batch_tpt(16), 16>(P.src, P.g, P.npad, P.B, P.chunk, P.pp, P.part, w.tile, w.split, w.sb * 16,
                                    s_src, s_g);
}

__global__ __launch_bounds__(kWG) void k_batch_pairs(const BatchProblemDev* __restrict__ probs,
                                                     const BatchItem* __restrict__ items, int nitems) {
  __shared__ float4 s_src[kWG];
  __shared__ float s_g[16][kWG];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const BatchItem w = items[it];
    const BatchProblemDev& P = probs[w.p];
    switch (P.kind) {
      case 0: batch_item<0>(P, w, s_src, s_g); break;
      case 1: batch_item<1>(P, w, s_src, s_g); break;
      case 2: batch_item<2>(P, w, s_src, s_g); break;
      default: batch_item<3>(P, w, s_src, s_g); break;
    }
  }
}

__device__ inline int batch_find(const BatchProblemDev* __restrict__ probs, int P, int64_t idx, bool padded) {
  int lo = 0, hi = P - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t off = padded ? probs[mid].gel_off : probs[mid].elem_off;
    if (off <= idx)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// g = q f(u) for every problem (zero on padding nodes), v = u.
__global__ __launch_bounds__(kWG) void k_batch_prep(const BatchProblemDev* __restrict__ probs, int P, int64_t total) {
  const int64_t idx = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (idx >= total) return;
  const int p = batch_find(probs, P, idx, true);
  const BatchProblemDev& Q = probs[p];
  const int64_t loc = idx - Q.gel_off;
  const int b = (int)(loc / Q.npad);
  const int64_t j = loc - (int64_t)b * Q.npad;
  float out = 0.0f;
  if (j < Q.n) {
    const double uj = Q.u[(int64_t)b * Q.n + j];
    Q.v[(int64_t)b * Q.n + j] = uj;
    out = (float)(Q.q[j] * sigmoid(uj, Q.fr.beta, state_theta(Q.fr, b)));
  }
  Q.g[loc] = out;
}

// RK4 stage combination for every (problem, state, node); as k_rk4_combine.
__global__ __launch_bounds__(kWG) void k_batch_combine(const BatchProblemDev* __restrict__ probs, int P,
                                                       int64_t total, int stage, double dt) {
  const int64_t idx = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (idx >= total) return;
  const int p = batch_find(probs, P, idx, false);
  const BatchProblemDev& Q = probs[p];
  const int64_t loc = idx - Q.elem_off;
  const int b = (int)(loc / Q.n);
  const int64_t i = loc - (int64_t)b * Q.n;
  double y = 0.0;
  for (int sp = 0; sp < Q.nsplit; ++sp) y += Q.part[((int64_t)sp * Q.B + b) * Q.npad + i];
  const double k = -Q.v[loc] + y;
  double ui = Q.u[loc];
  double vn;
  if (stage == 1) {
    Q.ksum[loc] = k;
    vn = ui + 0.5 * dt * k;
  } else if (stage == 2) {
    Q.ksum[loc] += 2.0 * k;
    vn = ui + 0.5 * dt * k;
  } else if (stage == 3) {
    Q.ksum[loc] += 2.0 * k;
    vn = ui + dt * k;
  } else {
    ui = ui + (dt / 6.0) * (Q.ksum[loc] + k);
    Q.u[loc] = ui;
    vn = ui;
  }
  Q.v[loc] = vn;
  Q.g[(int64_t)b * Q.npad + i] = (float)(Q.q[i] * sigmoid(vn, Q.fr.beta, state_theta(Q.fr, b)));
}

}  // namespace nfr
