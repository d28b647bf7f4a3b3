// kernels_diag.hpp -- turbulence diagnostics off the step's hot path:
// Eulerian structure functions (SI, eq. structure-fun-sm) and the sums of
// the SI's moment-space analysis of a collision (m_diff against m_neq with
// the MRT matrix M).  Sums are float64 block partials reduced in a fixed
// order.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels_fwd.hpp"

namespace lbm {

constexpr int DIAG_BLOCKS = 64;
constexpr int SF_PMAX = 8;

// Block-wide sum of v (256 threads) into red[0]; every thread must call it.
__device__ inline double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Separation l = blockIdx.y + 1; for every node, field and axis a < D the
// longitudinal increment d = u_a(x + l e_a) - u_a(x) (periodic, in float64);
// partial[(l - 1) * DIAG_BLOCKS + block][k]: sum of d^(k+1) for k < pmax,
// then sum of |d|^(k+1).
template <int D>
__global__ __launch_bounds__(256) void structure_kernel(const float* __restrict__ u, Grid G,
                                                        int pmax, double* __restrict__ partial) {
  const int l = blockIdx.y + 1;
  double s[SF_PMAX], sa[SF_PMAX];
#pragma unroll
  for (int p = 0; p < SF_PMAX; ++p) s[p] = sa[p] = 0.0;
  const long long total = (long long)G.plane * G.batch;
  for (long long n = blockIdx.x * 256LL + threadIdx.x; n < total;
       n += (long long)gridDim.x * 256) {
    int x, y, z, b;
    decode(G, n, x, y, z, b);
    const long long node = n - (long long)b * G.plane;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      int r[3] = {x, y, z};
      const int dim = a == 0 ? G.nx : (a == 1 ? G.ny : G.nz);
      r[a] = (r[a] + l) % dim;
      const float* ua = u + ((long long)b * D + a) * G.plane;
      const double d = (double)ua[((long long)r[2] * G.ny + r[1]) * G.nx + r[0]] - (double)ua[node];
      double v = 1.0, va = 1.0;
#pragma unroll
      for (int p = 0; p < SF_PMAX; ++p) {
        v *= d;
        va *= d < 0.0 ? -d : d;
        s[p] += v;
        sa[p] += va;
      }
    }
  }
  __shared__ double red[256];
  double* out = partial + ((long long)blockIdx.y * gridDim.x + blockIdx.x) * 2 * pmax;
  for (int p = 0; p < pmax; ++p) {
    const double t = block_sum(s[p], red), ta = block_sum(sa[p], red);
    if (threadIdx.x == 0) {
      out[p] = t;
      out[pmax + p] = ta;
    }
  }
}

// S[p][l] and Sabs[p][l] (row-major [pmax][lmax]) from the partials, summed
// over the blocks in order and divided by the sample count.
static __global__ __launch_bounds__(256) void structure_reduce_kernel(const double* __restrict__ partial,
                                                               int nblk, int lmax, int pmax,
                                                               double inv_count,
                                                               double* __restrict__ S,
                                                               double* __restrict__ Sabs) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= lmax * 2 * pmax) return;
  const int l = t / (2 * pmax), k = t % (2 * pmax);
  double acc = 0.0;
  for (int b = 0; b < nblk; ++b) acc += partial[((long long)l * nblk + b) * 2 * pmax + k];
  if (k < pmax)
    S[k * lmax + l] = acc * inv_count;
  else
    Sabs[(k - pmax) * lmax + l] = acc * inv_count;
}

// The MRT moment matrix M of the SI (D3Q19, velocity order of Table S1;
// rows rho, e, eps, jx, qx, jy, qy, jz, qz, pxx, pixx, pww, piww, pxy, pyz,
// pxz, mx, my, mz).
static __constant__ signed char kMrtM[19][19] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-30, -11, -11, -11, -11, -11, -11, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8},
    {12, -4, -4, -4, -4, -4, -4, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, -1, 0, 0, 0, 0, 1, -1, -1, -1, -1, 0, 0, 0, 0, 1, 1, 1, 1},
    {0, 4, 0, 0, 0, 0, -4, -1, -1, -1, -1, 0, 0, 0, 0, 1, 1, 1, 1},
    {0, 0, -1, 0, 0, 1, 0, -1, 0, 0, 1, -1, -1, 1, 1, -1, 0, 0, 1},
    {0, 0, 4, 0, 0, -4, 0, -1, 0, 0, 1, -1, -1, 1, 1, -1, 0, 0, 1},
    {0, 0, 0, -1, 1, 0, 0, 0, -1, 1, 0, -1, 1, -1, 1, 0, -1, 1, 0},
    {0, 0, 0, 4, -4, 0, 0, 0, -1, 1, 0, -1, 1, -1, 1, 0, -1, 1, 0},
    {0, 2, -1, -1, -1, -1, 2, 1, 1, 1, 1, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, -4, 2, 2, 2, 2, -4, 1, 1, 1, 1, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 0, 1, -1, -1, 1, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, -2, 2, 2, -2, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 0, 0, 1, 0, 0, -1, 0, 0, 0, 0, -1, 0, 0, 1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 0, 0, -1, 1, 0},
    {0, 0, 0, 0, 0, 0, 0, -1, 1, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 0, 0, 1, 0, 0, -1, -1, -1, 1, 1, 1, 0, 0, -1},
    {0, 0, 0, 0, 0, 0, 0, 0, -1, 1, 0, 1, -1, 1, -1, 0, -1, 1, 0},
};

// Moment i = blockIdx.y: with pre = A_n gathered at x, post = A_n1(x) (the
// post-collision populations of x in the pull-shifted layout),
//   m_diff = M_i (post - pre - f_ext),  m_neq = M_i (f_eq - pre),
// partial[i][block][0..4] = sums of m_neq, m_diff, m_neq^2, m_neq m_diff,
// m_diff^2 (float64).
static __global__ __launch_bounds__(256) void mrt_sums_kernel(const float* __restrict__ An,
                                                       const float* __restrict__ An1, Grid G,
                                                       Force Fc, float rho0,
                                                       double* __restrict__ partial) {
  using L = D3Q19;
  const int i = blockIdx.y;
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const long long total = (long long)G.plane * G.batch;
  for (long long n = blockIdx.x * 256LL + threadIdx.x; n < total;
       n += (long long)gridDim.x * 256) {
    int x, y, z, b;
    decode(G, n, x, y, z, b);
    float g[19], geq[19], fe[19], F[3];
    gather<L>(An, G, b, x, y, z, g);
    float drho, j[3];
    moments<L>(g, drho, j);
    const float rho = rho0 + drho, inv = 1.f / rho;
    const float uv[3] = {j[0] * inv, j[1] * inv, j[2] * inv};
    Unroll<L>::feq(drho, rho, uv, uv[0] * uv[0] + uv[1] * uv[1] + uv[2] * uv[2], geq);
    body_force(Fc, G, x, y, z, F);
    const float du[3] = {F[0] * inv, F[1] * inv, F[2] * inv};
    const float dd = du[0] * (2.f * uv[0] + du[0]) + du[1] * (2.f * uv[1] + du[1]) +
                     du[2] * (2.f * uv[2] + du[2]);
    Unroll<L>::fext(rho, uv, du, dd, fe);
    double md = 0.0, mn = 0.0;
#pragma unroll
    for (int q = 0; q < 19; ++q) {
      const double post = An1[cell(G, b, q, 19, x, y, z)];
      const double m = kMrtM[i][q];
      md += m * (post - (double)g[q] - (double)fe[q]);
      mn += m * ((double)geq[q] - (double)g[q]);
    }
    s[0] += mn;
    s[1] += md;
    s[2] += mn * mn;
    s[3] += mn * md;
    s[4] += md * md;
  }
  __shared__ double red[256];
  for (int k = 0; k < 5; ++k) {
    const double t = block_sum(s[k], red);
    if (threadIdx.x == 0) partial[((long long)i * gridDim.x + blockIdx.x) * 5 + k] = t;
  }
}

// stats[i][k] = sum over the blocks (in order) of partial[i][block][k].
static __global__ __launch_bounds__(128) void mrt_reduce_kernel(const double* __restrict__ partial,
                                                         int nblk, double* __restrict__ stats) {
  const int t = threadIdx.x;
  if (t >= 19 * 5) return;
  const int i = t / 5, k = t % 5;
  double acc = 0.0;
  for (int b = 0; b < nblk; ++b) acc += partial[((long long)i * nblk + b) * 5 + k];
  stats[t] = acc;
}

}  // namespace lbm
