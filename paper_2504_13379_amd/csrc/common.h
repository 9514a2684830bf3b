// Internal definitions shared by the kernels and the C ABI implementation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nfr {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWG = 256;        // threads per workgroup (four wave64s)
constexpr int kPad = 256;       // node padding granule
constexpr double kLog2e = 1.4426950408889634074;

// Device-side view of a packed problem.  Layout inside the caller's buffer:
//   float4 src[npad]   (x, y, z, |x|^2) in FP32 (|x|^2 = 0 when periodic)
//   double q[npad]     quadrature weights, 0 on padding nodes
//   double xyz[3*npad] FP64 coordinates (row-major), 0 on padding nodes
// A periodic problem (period > 0) has its (x, y) plane doubly periodic with
// that period (the flat domains of the paper's section 4, eq. dist); its x and
// y are stored reduced to [-period/2, period/2].
struct ProblemView {
  int64_t n = 0, npad = 0;
  double period = 0.0;
  const float4* src = nullptr;
  const double* q = nullptr;
  const double* xyz = nullptr;
  const double* qmax = nullptr;   // on the device: [0] max_j |q_j|, [1] max_j |x_j|^2 (FP32 coordinates)
  // Tile order (kernels_tile.h): perm[s] = node in slot s, the packed
  // coordinates and weights in slot order, and bounding spheres of blocks of
  // 32 and 16 slots.  A view with `tiled` set has src and q in slot order.
  const int* perm = nullptr;
  const float4* src_t = nullptr;
  const double* q_t = nullptr;
  const float4* bnd32 = nullptr;
  const float4* bnd16 = nullptr;
  bool tiled = false;
};

// The problem seen in its tile order (states indexed by slot).
inline ProblemView tile_view(const ProblemView& pv) {
  ProblemView t = pv;
  t.src = pv.src_t;
  t.q = pv.q_t;
  t.xyz = nullptr;
  t.tiled = true;
  return t;
}

// Kernel evaluation in the on-the-fly pair sum.  Coordinates are multiplied by
// `sig` so that the excitatory exponent becomes exp2(-t) with
//   Gaussian:    t = |sig (x_i - x_j)|^2,  sig = sqrt(log2 e) / s_e,  rho = s_e^2 / s_i^2
//   exponential: t = |sig (x_i - x_j)|,    sig = log2 e / s_e,        rho = s_e / s_i
// and the inhibitory one exp2(-rho t); w = A_e exp2(-t) - A_i exp2(-rho t).
// `per` is the scaled period sig * L of a periodic problem (0 otherwise).
// The forward pair sums accumulate the normalised kernel
//   u = exp2(-t) + kappa exp2(-rho t),  kappa = -A_i / A_e,  w = amp u (amp = A_e),
// one value per pair instead of the two exponentials separately (a kernel with
// A_e = 0 is first rewritten as its single inhibitory term, see norm_kernel).
//
// Pair kernels take KIND = kernel kind (bit 0: 0 Gaussian, 1 exponential)
// plus 2 for a periodic problem.
struct PairParams {
  float sig;
  float rho;
  double Ae;
  double Ai;
  float per;
  float kappa;
  double amp;
};

// Squared scaled distance of a pair from its coordinate differences.  For a
// periodic problem both points lie in one period window, so |d| <= per along
// x and y and the nearest of the lattice images (eq. dist: shifts by -L, 0, L
// per axis) is at distance min(|d|, per - |d|) along each axis independently.
template <int KIND>
__device__ __forceinline__ float pair_r2(float dx, float dy, float dz, float per) {
  if (KIND & 2) {
    dx = fabsf(dx);
    dx = fminf(dx, per - dx);
    dy = fabsf(dy);
    dy = fminf(dy, per - dy);
  }
  return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

// Sigmoid firing rate; FP64.
struct Firing {
  double beta;
  double theta;
  const double* theta_dev;  // per state, may be null
};

__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

__device__ inline double sigmoid(double u, double beta, double theta) {
  return 1.0 / (1.0 + exp(-beta * (u - theta)));
}

__device__ inline double state_theta(const Firing& f, int b) {
  return f.theta_dev ? f.theta_dev[b] : f.theta;
}

}  // namespace nfr
