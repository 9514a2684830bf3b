// Surface quadrature weights on the GPU (paper section 3.3, eqs. integral and
// functional_stencil): for every flat triangle E_j of a closed surface,
//   1. stencil S(E_j): the k nodes nearest to the centroid c_j;
//   2. projection point p_j (the origin for star-shaped surfaces; otherwise
//      the common point of the three cutting planes through E_j's edges);
//   3. stencil nodes pulled back along rays from p_j onto E_j's plane, with
//      the Jacobian of the central projection;
//   4. planar RBF-QF on E_j (phi = r^3 plus degree-2 polynomials): one
//      (k+6) x (k+6) saddle-point solve, right-hand side the exact integrals of
//      the basis over E_j;
//   5. q_i = sum of the scaled element weights of node i over all triangles,
//      added in increasing (triangle, slot) order.
// All arithmetic is FP64.  One wave per centroid group (k-nearest) and one
// wave per triangle (the solve); no float atomics, so q is reproducible.
#pragma once

#include "common.h"

namespace nfr {

// |p - c|^2 as (dx dx + dy dy) + dz dz with every operation rounded on its
// own (no fused multiply-add): stencil ranks are decided on this value.
__device__ inline double quad_sqdist(double px, double py, double pz, double cx, double cy, double cz) {
#pragma clang fp contract(off)
  const double dx = px - cx;
  const double dy = py - cy;
  const double dz = pz - cz;
  const double xy = dx * dx + dy * dy;
  return xy + dz * dz;
}

// Centroids (a + b + c) / 3 (summed in vertex order) and unit plane normals
// (b - a) x (c - a) / |.| of every triangle.
__global__ __launch_bounds__(kWG) void k_quad_centroids(const double* __restrict__ xyz, const int* __restrict__ tri,
                                                        int64_t ntri, double* __restrict__ cen,
                                                        double* __restrict__ nrm_tri) {
#pragma clang fp contract(off)
  const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (t >= ntri) return;
  const double* a = xyz + 3 * (int64_t)tri[3 * t];
  const double* b = xyz + 3 * (int64_t)tri[3 * t + 1];
  const double* c = xyz + 3 * (int64_t)tri[3 * t + 2];
  for (int d = 0; d < 3; ++d) cen[3 * t + d] = (a[d] + b[d] + c[d]) / 3.0;
  const double u0 = b[0] - a[0], u1 = b[1] - a[1], u2 = b[2] - a[2];
  const double v0 = c[0] - a[0], v1 = c[1] - a[1], v2 = c[2] - a[2];
  const double n0 = u1 * v2 - u2 * v1, n1 = u2 * v0 - u0 * v2, n2 = u0 * v1 - u1 * v0;
  const double len = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
  nrm_tri[3 * t] = n0 / len;
  nrm_tri[3 * t + 1] = n1 / len;
  nrm_tri[3 * t + 2] = n2 / len;
}

// ------------------------------------------------------------------ k nearest nodes

// Nodes are binned into a uniform grid of cubic cells; a centroid's search
// visits the cells in Chebyshev rings r = 0, 1, 2, ... around its own cell and
// stops once its k-th key is below the squared distance from the centroid to
// the boundary of the rings visited (every node outside lies beyond it; a
// relative margin of 1e-12 covers the rounding of the binning and of that
// bound).  The result is the exact k smallest (squared distance, index), the
// same as a full scan.

struct QuadGrid {
  double ox, oy, oz, h;   // origin (lower corner) and cell size
  int nx, ny, nz;
};

// One workgroup of kWG threads: bounding box of the nodes, then (thread 0) a
// grid with about 4 nodes per cell of the box's volume (a surface fills a
// small share of its box, so occupied cells hold a few tens of nodes), at most
// max_cells cells.
__global__ __launch_bounds__(kWG) void k_quad_grid(const double* __restrict__ xyz, int64_t n, int64_t max_cells,
                                                   QuadGrid* __restrict__ grid) {
  __shared__ double s_lo[3][kWG], s_hi[3][kWG];
  double lo[3] = {xyz[0], xyz[1], xyz[2]}, hi[3] = {xyz[0], xyz[1], xyz[2]};
  for (int64_t i = threadIdx.x; i < n; i += kWG)
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], xyz[3 * i + d]);
      hi[d] = fmax(hi[d], xyz[3 * i + d]);
    }
  for (int d = 0; d < 3; ++d) {
    s_lo[d][threadIdx.x] = lo[d];
    s_hi[d][threadIdx.x] = hi[d];
  }
  __syncthreads();
  for (int w = kWG / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int d = 0; d < 3; ++d) {
        s_lo[d][threadIdx.x] = fmin(s_lo[d][threadIdx.x], s_lo[d][threadIdx.x + w]);
        s_hi[d][threadIdx.x] = fmax(s_hi[d][threadIdx.x], s_hi[d][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  double ext[3], emax = 0.0;
  for (int d = 0; d < 3; ++d) {
    ext[d] = s_hi[d][0] - s_lo[d][0];
    emax = fmax(emax, ext[d]);
  }
  if (!(emax > 0.0)) emax = 1.0;
  // volume, with flat directions given a thousandth of the largest extent
  double h = cbrt(fmax(ext[0], emax * 1e-3) * fmax(ext[1], emax * 1e-3) * fmax(ext[2], emax * 1e-3) * 4.0 / (double)n);
  int dim[3];
  for (;;) {
    int64_t cells = 1;
    for (int d = 0; d < 3; ++d) {
      dim[d] = (int)fmin(floor(ext[d] / h) + 1.0, 2048.0);
      cells *= dim[d];
    }
    if (cells <= max_cells) break;
    h *= 1.25;
  }
  grid->ox = s_lo[0][0];
  grid->oy = s_lo[1][0];
  grid->oz = s_lo[2][0];
  grid->h = h;
  grid->nx = dim[0];
  grid->ny = dim[1];
  grid->nz = dim[2];
}

__device__ inline int quad_cell_coord(double x, double o, double h, int dim) {
  const double c = floor((x - o) / h);
  return c < 0.0 ? 0 : (c >= (double)dim ? dim - 1 : (int)c);
}

__device__ inline int64_t quad_cell_of(const QuadGrid& g, double x, double y, double z) {
  const int cx = quad_cell_coord(x, g.ox, g.h, g.nx);
  const int cy = quad_cell_coord(y, g.oy, g.h, g.ny);
  const int cz = quad_cell_coord(z, g.oz, g.h, g.nz);
  return ((int64_t)cz * g.ny + cy) * g.nx + cx;
}

__global__ __launch_bounds__(kWG) void k_quad_bin_count(const double* __restrict__ xyz, int64_t n,
                                                        const QuadGrid* __restrict__ grid, int* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= n) return;
  atomicAdd(&cnt[quad_cell_of(*grid, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2])], 1);
}

// Node i goes to a free place of its cell's list (order inside a cell is
// irrelevant: the ranking key is a total order).
__global__ __launch_bounds__(kWG) void k_quad_bin_fill(const double* __restrict__ xyz, int64_t n,
                                                       const QuadGrid* __restrict__ grid,
                                                       const int64_t* __restrict__ start, int* __restrict__ cursor,
                                                       int* __restrict__ nodes) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= n) return;
  const int64_t c = quad_cell_of(*grid, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
  nodes[start[c] + atomicAdd(&cursor[c], 1)] = (int)i;
}

__device__ inline bool key_less(double d, int i, double d2, int i2) { return d < d2 || (d == d2 && i < i2); }

// st[t*k + r], r < k: the k nodes with the smallest (squared distance, index)
// to centroid t, in increasing order; one wave per centroid.  Lane r holds
// entry r of the sorted list; a candidate below the k-th key is inserted by a
// ballot (its rank) and a one-lane shift.  cnt / start: nodes per cell and
// their offsets into `nodes`.  Requires k <= 64 and k <= n.
__global__ __launch_bounds__(kWG) void k_quad_knn(const double* __restrict__ xyz, const QuadGrid* __restrict__ grid_p,
                                                  const int* __restrict__ cnt, const int64_t* __restrict__ start,
                                                  const int* __restrict__ nodes, const double* __restrict__ cen,
                                                  int64_t ntri, int k, int* __restrict__ st) {
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * (kWG / 64) + (threadIdx.x >> 6);
  if (t >= ntri) return;
  const QuadGrid g = *grid_p;
  const double cx = cen[3 * t], cy = cen[3 * t + 1], cz = cen[3 * t + 2];
  const int ix = quad_cell_coord(cx, g.ox, g.h, g.nx);
  const int iy = quad_cell_coord(cy, g.oy, g.h, g.ny);
  const int iz = quad_cell_coord(cz, g.oz, g.h, g.nz);
  double ld = __builtin_inf(), thr = __builtin_inf();
  int li = 0x7fffffff, thr_i = 0x7fffffff;
  const int rmax = max(max(g.nx, g.ny), g.nz);
  for (int r = 0; r <= rmax; ++r) {
    for (int dz = -r; dz <= r; ++dz) {
      const int z = iz + dz;
      if (z < 0 || z >= g.nz) continue;
      for (int dy = -r; dy <= r; ++dy) {
        const int y = iy + dy;
        if (y < 0 || y >= g.ny) continue;
        const bool face = dz == -r || dz == r || dy == -r || dy == r;
        for (int dx = -r; dx <= r; dx += (face || r == 0) ? 1 : 2 * r) {   // only the ring's shell
          const int x = ix + dx;
          if (x < 0 || x >= g.nx) continue;
          const int64_t c = ((int64_t)z * g.ny + y) * g.nx + x;
          const int64_t c0 = start[c];
          const int m = cnt[c];
          for (int b = 0; b < m; b += 64) {
            const bool valid = b + lane < m;
            const int j = valid ? nodes[c0 + b + lane] : 0;
            const double key = valid ? quad_sqdist(xyz[3 * (int64_t)j], xyz[3 * (int64_t)j + 1],
                                                   xyz[3 * (int64_t)j + 2], cx, cy, cz)
                                     : 0.0;
            uint64_t mask = __ballot(valid && key_less(key, j, thr, thr_i));
            while (mask) {
              const int src = __builtin_ctzll(mask);
              mask &= mask - 1;
              const double cd = __shfl(key, src);
              const int ci = __shfl(j, src);
              if (!key_less(cd, ci, thr, thr_i)) continue;
              const bool before = lane < k && key_less(ld, li, cd, ci);
              const int pos = __popcll(__ballot(before));
              const double up_d = __shfl_up(ld, 1);
              const int up_i = __shfl_up(li, 1);
              if (lane == pos) {
                ld = cd;
                li = ci;
              } else if (lane > pos && lane < k) {
                ld = up_d;
                li = up_i;
              }
              thr = __shfl(ld, k - 1);
              thr_i = __shfl(li, k - 1);
            }
          }
        }
      }
    }
    // distance from the centroid to the boundary of rings 0..r (sides with no
    // cells beyond them do not count)
    double bound = __builtin_inf();
    const double o[3] = {g.ox, g.oy, g.oz};
    const double p[3] = {cx, cy, cz};
    const int ic[3] = {ix, iy, iz};
    const int dims[3] = {g.nx, g.ny, g.nz};
    for (int d = 0; d < 3; ++d) {
      if (ic[d] - r > 0) bound = fmin(bound, p[d] - (o[d] + (double)(ic[d] - r) * g.h));
      if (ic[d] + r < dims[d] - 1) bound = fmin(bound, (o[d] + (double)(ic[d] + r + 1) * g.h) - p[d]);
    }
    if (bound == __builtin_inf()) break;                                   // every cell visited
    if (thr_i != 0x7fffffff && bound > 0.0 && thr < bound * bound * (1.0 - 1e-12)) break;
  }
  if (lane < k) st[t * k + lane] = li;
}

// ------------------------------------------------------------------ projection points

// Singular values of a 3 x 3 matrix (rows m[0..2]) by one-sided Jacobi
// rotations of its columns; returns sigma_max / sigma_min (inf if singular).
__device__ inline double cond3(const double m[3][3]) {
  double a[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) a[r][c] = m[r][c];
  for (int sweep = 0; sweep < 30; ++sweep) {
    bool rotated = false;
    for (int i = 0; i < 2; ++i)
      for (int j = i + 1; j < 3; ++j) {
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int r = 0; r < 3; ++r) {
          al += a[r][i] * a[r][i];
          be += a[r][j] * a[r][j];
          ga += a[r][i] * a[r][j];
        }
        if (fabs(ga) <= 1e-15 * sqrt(al * be)) continue;
        rotated = true;
        const double zeta = (be - al) / (2.0 * ga);
        const double tn = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + tn * tn);
        const double sn = cs * tn;
        for (int r = 0; r < 3; ++r) {
          const double x = a[r][i], y = a[r][j];
          a[r][i] = cs * x - sn * y;
          a[r][j] = sn * x + cs * y;
        }
      }
    if (!rotated) break;
  }
  double smax = 0.0, smin = __builtin_inf();
  for (int c = 0; c < 3; ++c) {
    const double s = sqrt(a[0][c] * a[0][c] + a[1][c] * a[1][c] + a[2][c] * a[2][c]);
    smax = fmax(smax, s);
    smin = fmin(smin, s);
  }
  return smin > 0.0 ? smax / smin : __builtin_inf();
}

// p_j for every triangle (written to proj[3*t]; a NaN row means "orthogonal
// projection onto E_j's plane").  mode 1 (origin): p_j = 0; mode 2
// (orthogonal): a NaN row for every triangle.  Mode 0 (planes): row e of the
// 3 x 3 system is the unit normal of the cutting plane through edge e
// (vertex e to vertex e+1), n_j - n_{neighbour across e} normalised, with
// right-hand side its product with (vertex e - c_j); p_j = c_j + solution.
// A system with condition number above cond_max (or a zero row) falls back
// to orthogonal projection.
__global__ __launch_bounds__(kWG) void k_quad_proj(const double* __restrict__ xyz, const int* __restrict__ tri,
                                                   const int* __restrict__ nbr, const double* __restrict__ cen,
                                                   const double* __restrict__ nrm_tri, int64_t ntri, int mode,
                                                   double cond_max, double* __restrict__ proj) {
  const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (t >= ntri) return;
  if (mode == 1) {
    proj[3 * t] = proj[3 * t + 1] = proj[3 * t + 2] = 0.0;
    return;
  }
  if (mode == 2) {
    const double nan = __builtin_nan("");
    proj[3 * t] = proj[3 * t + 1] = proj[3 * t + 2] = nan;
    return;
  }
  double m[3][3], rhs[3];
  bool ok = true;
  for (int e = 0; e < 3; ++e) {
    const int64_t o = nbr[3 * t + e];
    double row[3], len2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      row[d] = nrm_tri[3 * t + d] - nrm_tri[3 * o + d];
      len2 += row[d] * row[d];
    }
    const double len = sqrt(len2);
    if (!(len > 0.0)) ok = false;
    double r = 0.0;
    const double* v = xyz + 3 * (int64_t)tri[3 * t + e];
    for (int d = 0; d < 3; ++d) {
      m[e][d] = row[d] / len;
      r += m[e][d] * (v[d] - cen[3 * t + d]);
    }
    rhs[e] = r;
  }
  if (ok && !(cond3(m) <= cond_max)) ok = false;
  if (!ok) {
    const double nan = __builtin_nan("");
    proj[3 * t] = proj[3 * t + 1] = proj[3 * t + 2] = nan;
    return;
  }
  // Gaussian elimination with partial pivoting on [m | rhs]
  int perm[3] = {0, 1, 2};
  for (int c = 0; c < 3; ++c) {
    int piv = c;
    for (int r = c + 1; r < 3; ++r)
      if (fabs(m[perm[r]][c]) > fabs(m[perm[piv]][c])) piv = r;
    const int tmp = perm[c];
    perm[c] = perm[piv];
    perm[piv] = tmp;
    for (int r = c + 1; r < 3; ++r) {
      const double f = m[perm[r]][c] / m[perm[c]][c];
      for (int cc = c; cc < 3; ++cc) m[perm[r]][cc] -= f * m[perm[c]][cc];
      rhs[perm[r]] -= f * rhs[perm[c]];
    }
  }
  double x[3];
  for (int c = 2; c >= 0; --c) {
    double s = rhs[perm[c]];
    for (int cc = c + 1; cc < 3; ++cc) s -= m[perm[c]][cc] * x[cc];
    x[c] = s / m[perm[c]][c];
  }
  for (int d = 0; d < 3; ++d) proj[3 * t + d] = cen[3 * t + d] + x[d];
}

// ------------------------------------------------------------------ element weights

// Integral of |s - P|^3 over the triangle (P, p, q) (2-D, unsigned).  In
// polar coordinates about P it is (d^5 / 5) times the antiderivative of
// sec^5 between the angles of p and q, d the distance from P to the line pq;
// with rho = d sec(alpha) and l = d tan(alpha) (l measured along p -> q from
// the foot of the perpendicular) the antiderivative times d^4 reads
//   rho^3 l / 4 + 3 d^2 rho l / 8 + 3 d^4 log(rho + l) / 8.
// log(rho + l) for l < 0 is taken as 2 log d - log(rho - l) (no cancellation).
__device__ inline double r3_apex(double Px, double Py, double px, double py, double qx, double qy) {
  const double ex = qx - px, ey = qy - py;
  const double len = sqrt(ex * ex + ey * ey);
  const double ux = ex / len, uy = ey / len;
  const double wx = px - Px, wy = py - Py;
  const double lp = wx * ux + wy * uy;
  const double lq = lp + len;
  const double d = fabs(wx * uy - wy * ux);
  const double d2 = d * d;
  const double rp = sqrt(d2 + lp * lp);
  const double rq = sqrt(d2 + lq * lq);
  double val = 0.25 * (rq * rq * rq * lq - rp * rp * rp * lp) + 0.375 * d2 * (rq * lq - rp * lp);
  if (d > 0.0) {
    const double Lq = lq >= 0.0 ? log(rq + lq) : 2.0 * log(d) - log(rq - lq);
    const double Lp = lp >= 0.0 ? log(rp + lp) : 2.0 * log(d) - log(rp - lp);
    val += 0.375 * d2 * d2 * (Lq - Lp);
  }
  return d * val / 5.0;
}

__device__ inline double cross2(double ax, double ay, double bx, double by) { return ax * by - ay * bx; }

__device__ inline double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

// Integral of |s - P|^3 over the triangle (v0, v1, v2): the three triangles
// with apex P, each signed by its orientation relative to the triangle's.
__device__ inline double r3_triangle(double Px, double Py, const double v[3][2]) {
  const double o = sgn(cross2(v[1][0] - v[0][0], v[1][1] - v[0][1], v[2][0] - v[0][0], v[2][1] - v[0][1]));
  double total = 0.0;
  for (int e = 0; e < 3; ++e) {
    const double* p = v[e];
    const double* q = v[(e + 1) % 3];
    const double s = sgn(cross2(p[0] - Px, p[1] - Py, q[0] - Px, q[1] - Py)) * o;
    if (s != 0.0) total += s * r3_apex(Px, Py, p[0], p[1], q[0], q[1]);
  }
  return total;
}

__device__ inline double mono2(int m, double x, double y) {
  switch (m) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return x * x;
    case 4: return x * y;
    default: return y * y;
  }
}

constexpr int kQuadMaxK = 57;   // k + 7 <= 64: one lane per column of the system and its right-hand side

// One wave per triangle t: pull-back, Jacobian, planar system in LDS
// ((k+6) rows of k+7 FP64: matrix and right-hand side), LU with partial
// pivoting (largest magnitude, first row on ties), back substitution;
// wE[t*k + r] = w_r h_t^2 J_r.  Dynamic LDS: (k+6)(k+7) doubles + 2k doubles.
__global__ __launch_bounds__(64) void k_quad_elements(const double* __restrict__ xyz, const double* __restrict__ nrm,
                                                      const int* __restrict__ tri, const double* __restrict__ cen,
                                                      const double* __restrict__ nrm_tri,
                                                      const double* __restrict__ proj, const int* __restrict__ st,
                                                      int64_t n, int64_t ntri, int k, double* __restrict__ wE) {
  extern __shared__ double lds[];
  const int dim = k + 6;
  const int ld = k + 7;
  double* M = lds;                 // dim x ld
  double* s2 = lds + dim * ld;     // k x 2 planar stencil coordinates
  const int64_t t = blockIdx.x;
  const int lane = threadIdx.x;
  if (t >= ntri) return;

  double A[3], B[3], C[3], nj[3], cj[3], p[3];
  for (int d = 0; d < 3; ++d) {
    A[d] = xyz[3 * (int64_t)tri[3 * t] + d];
    B[d] = xyz[3 * (int64_t)tri[3 * t + 1] + d];
    C[d] = xyz[3 * (int64_t)tri[3 * t + 2] + d];
    nj[d] = nrm_tri[3 * t + d];
    cj[d] = cen[3 * t + d];
    p[d] = proj[3 * t + d];
  }
  const bool orth = p[0] != p[0];
  // frame of E_j: e1 along B - A, e2 = n_j x e1
  double e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
  {
    const double l = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (int d = 0; d < 3; ++d) e1[d] /= l;
  }
  const double e2[3] = {nj[1] * e1[2] - nj[2] * e1[1], nj[2] * e1[0] - nj[0] * e1[2], nj[0] * e1[1] - nj[1] * e1[0]};

  // lane r < k: stencil node, its pre-image xi on E_j's plane and the Jacobian
  double J = 0.0, rel1 = 0.0, rel2 = 0.0, rlen = 0.0;
  if (lane < k) {
    const int64_t s = st[t * k + lane];
    const bool in_range = s >= 0 && s < n;   // a stencil slot left unfilled (non-finite coordinates) gives NaN
    double X[3], Ns[3], xi[3];
    for (int d = 0; d < 3; ++d) {
      X[d] = in_range ? xyz[3 * s + d] : __builtin_nan("");
      Ns[d] = in_range ? nrm[3 * s + d] : __builtin_nan("");
    }
    if (!orth) {
      double dxp[3], num = 0.0, den = 0.0, nx = 0.0;
      for (int d = 0; d < 3; ++d) {
        dxp[d] = X[d] - p[d];
        num += nj[d] * (A[d] - p[d]);
        den += nj[d] * dxp[d];
        nx += dxp[d] * dxp[d];
      }
      const double tt = num / den;
      double nxi = 0.0, cp = 0.0, cs = 0.0;
      nx = sqrt(nx);
      for (int d = 0; d < 3; ++d) {
        xi[d] = p[d] + tt * dxp[d];
        const double diff = xi[d] - p[d];
        nxi += diff * diff;
        cp += nj[d] * dxp[d] / nx;
        cs += Ns[d] * dxp[d] / nx;
      }
      const double ratio = nx / sqrt(nxi);
      J = ratio * ratio * fabs(cp) / fabs(cs);
    } else {
      double h = 0.0, c = 0.0;
      for (int d = 0; d < 3; ++d) {
        h += nj[d] * (X[d] - A[d]);
        c += Ns[d] * nj[d];
      }
      for (int d = 0; d < 3; ++d) xi[d] = X[d] - h * nj[d];
      J = 1.0 / fabs(c);
    }
    double rel[3];
    for (int d = 0; d < 3; ++d) rel[d] = xi[d] - cj[d];
    rel1 = rel[0] * e1[0] + rel[1] * e1[1] + rel[2] * e1[2];
    rel2 = rel[0] * e2[0] + rel[1] * e2[1] + rel[2] * e2[2];
    rlen = sqrt(rel[0] * rel[0] + rel[1] * rel[1] + rel[2] * rel[2]);
  }
  // h_t = largest stencil radius (wave maximum)
  double h = rlen;
  for (int off = 32; off > 0; off >>= 1) h = fmax(h, __shfl_xor(h, off));
  double v[3][2];
  {
    const double* V[3] = {A, B, C};
    for (int i = 0; i < 3; ++i) {
      double r0 = 0.0, r1 = 0.0;
      for (int d = 0; d < 3; ++d) {
        r0 += (V[i][d] - cj[d]) * e1[d];
        r1 += (V[i][d] - cj[d]) * e2[d];
      }
      v[i][0] = r0 / h;
      v[i][1] = r1 / h;
    }
  }
  const double sx = rel1 / h, sy = rel2 / h;
  if (lane < k) {
    s2[2 * lane] = sx;
    s2[2 * lane + 1] = sy;
  }
  __syncthreads();

  // assemble: rows r < k: [|s_r - s_c|^3 (c < k) | pi_m(s_r) | int_E |s - s_r|^3]
  //           rows k + m: [pi_m(s_c) (c < k) | 0 | int_E pi_m]
  if (lane < k) {
    double* row = M + lane * ld;
    for (int c = 0; c < k; ++c) {
      const double dx = sx - s2[2 * c], dy = sy - s2[2 * c + 1];
      const double r = sqrt(dx * dx + dy * dy);
      row[c] = r * r * r;
    }
    for (int m = 0; m < 6; ++m) row[k + m] = mono2(m, sx, sy);
    row[dim] = r3_triangle(sx, sy, v);
  } else if (lane < dim) {
    const int m = lane - k;
    double* row = M + lane * ld;
    for (int c = 0; c < k; ++c) row[c] = mono2(m, s2[2 * c], s2[2 * c + 1]);
    for (int c = k; c < dim; ++c) row[c] = 0.0;
    // exact for degree 2: area / 3 times the sum over the edge midpoints
    const double area = 0.5 * fabs(cross2(v[1][0] - v[0][0], v[1][1] - v[0][1], v[2][0] - v[0][0], v[2][1] - v[0][1]));
    double acc = 0.0;
    for (int e = 0; e < 3; ++e) {
      const int f = (e + 1) % 3;
      acc += mono2(m, 0.5 * (v[e][0] + v[f][0]), 0.5 * (v[e][1] + v[f][1]));
    }
    row[dim] = acc * (area / 3.0);
  }
  __syncthreads();

  // LU with partial pivoting; lane c owns column c of the trailing update
  for (int col = 0; col < dim; ++col) {
    double best = (lane >= col && lane < dim) ? fabs(M[lane * ld + col]) : -1.0;
    int bi = lane;
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (bi != col && lane <= dim) {
      const double a = M[col * ld + lane];
      M[col * ld + lane] = M[bi * ld + lane];
      M[bi * ld + lane] = a;
    }
    __syncthreads();
    const double pv = M[col * ld + col];
    if (lane > col && lane < dim) M[lane * ld + col] /= pv;
    __syncthreads();
    if (lane > col && lane <= dim) {
      const double top = M[col * ld + lane];
      for (int r = col + 1; r < dim; ++r) M[r * ld + lane] -= M[r * ld + col] * top;
    }
    __syncthreads();
  }
  // back substitution on the right-hand-side column
  for (int r = dim - 1; r >= 0; --r) {
    const double xr = M[r * ld + dim] / M[r * ld + r];
    __syncthreads();
    if (lane < r) M[lane * ld + dim] -= M[lane * ld + r] * xr;
    if (lane == r) M[r * ld + dim] = xr;
    __syncthreads();
  }
  if (lane < k) wE[t * k + lane] = M[lane * ld + dim] * h * h * J;
}

// ------------------------------------------------------------------ accumulation

__global__ __launch_bounds__(kWG) void k_quad_count(const int* __restrict__ st, int64_t total, int64_t n,
                                                    int* __restrict__ cnt) {
  const int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (e >= total) return;
  const int i = st[e];
  if (i >= 0 && i < n) atomicAdd(&cnt[i], 1);
}

// Exclusive prefix sums in three passes: block totals, a single-workgroup
// scan of the totals, then each block's own scan plus its offset.
__global__ __launch_bounds__(kWG) void k_scan_blocks(const int* __restrict__ cnt, int64_t n,
                                                     int64_t* __restrict__ bsum) {
  __shared__ int64_t s[kWG];
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  s[threadIdx.x] = i < n ? cnt[i] : 0;
  __syncthreads();
  for (int w = kWG / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kWG) void k_scan_totals(int64_t* __restrict__ bsum, int64_t nb) {
  __shared__ int64_t s[kWG];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kWG) {
    const int64_t b = b0 + threadIdx.x;
    const int64_t v = b < nb ? bsum[b] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = 1; w < kWG; w <<= 1) {
      const int64_t add = threadIdx.x >= w ? s[threadIdx.x - w] : 0;
      __syncthreads();
      s[threadIdx.x] += add;
      __syncthreads();
    }
    if (b < nb) bsum[b] = carry + s[threadIdx.x] - v;
    carry += s[kWG - 1];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kWG) void k_scan_apply(const int* __restrict__ cnt, int64_t n,
                                                    const int64_t* __restrict__ bsum, int64_t* __restrict__ off) {
  __shared__ int64_t s[kWG];
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  const int64_t v = i < n ? cnt[i] : 0;
  s[threadIdx.x] = v;
  __syncthreads();
  for (int w = 1; w < kWG; w <<= 1) {
    const int64_t add = threadIdx.x >= w ? s[threadIdx.x - w] : 0;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  if (i < n) off[i] = bsum[blockIdx.x] + s[threadIdx.x] - v;
}

// Entry e = t*k + r of the stencil table goes to a free place in its node's
// segment (the order inside a segment is fixed afterwards by sorting).
__global__ __launch_bounds__(kWG) void k_quad_fill(const int* __restrict__ st, int64_t total, int64_t n,
                                                   const int64_t* __restrict__ off, int* __restrict__ cursor,
                                                   int* __restrict__ list) {
  const int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (e >= total) return;
  const int i = st[e];
  if (i < 0 || i >= n) return;
  list[off[i] + atomicAdd(&cursor[i], 1)] = (int)e;
}

// q_i = sum of wE over node i's segment in increasing entry order (insertion
// sort of the segment first).
__global__ __launch_bounds__(kWG) void k_quad_sum(const int64_t* __restrict__ off, const int* __restrict__ cnt,
                                                  int64_t n, int* __restrict__ list, const double* __restrict__ wE,
                                                  double* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= n) return;
  int* seg = list + off[i];
  const int len = cnt[i];
  for (int a = 1; a < len; ++a) {
    const int key = seg[a];
    int b = a - 1;
    while (b >= 0 && seg[b] > key) {
      seg[b + 1] = seg[b];
      --b;
    }
    seg[b + 1] = key;
  }
  double acc = 0.0;
  for (int a = 0; a < len; ++a) acc += wE[seg[a]];
  q[i] = acc;
}

}  // namespace nfr
