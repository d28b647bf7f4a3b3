// kernels_aux.hpp -- training-side kernels: the velocity mean-squared-error
// loss and its gradient, the Adam update, and the block-average filter used
// to coarse-grain fine fields.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels_fwd.hpp"

namespace lbm {

// L = mean_{b, x, a} (u_a - ut_a)^2 with u = (j + F/2) / rho of the
// pre-collision state; dL/dg_q(x) = 2/count * sum_a e_a (c_qa - u_a) / rho,
// written to the pull-shifted position dLdA_q(x - c_q) (the gather is a
// permutation, so its transpose is a conflict-free scatter).  Block partial
// sums in float64, reduced in a fixed order.
template <class L>
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ A,
                                                   const float* __restrict__ ut,
                                                   float* __restrict__ dLdA,
                                                   double* __restrict__ partial, Grid G,
                                                   float rho0, Force Fc, double inv_count) {
  double acc = 0.0;
  const long long total = (long long)G.plane * G.batch;
  for (long long n = blockIdx.x * 256LL + threadIdx.x; n < total;
       n += (long long)gridDim.x * 256) {
    int x, y, z, b;
    decode(G, n, x, y, z, b);
    long long node = n - (long long)b * G.plane;
    float g[L::Q];
    gather<L>(A, G, b, x, y, z, g);
    float drho, j[3], F[3];
    moments<L>(g, drho, j);
    body_force(Fc, G, x, y, z, F);
    float rho = rho0 + drho, inv = 1.f / rho;
    float uv[3] = {0.f, 0.f, 0.f}, e[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < L::D; ++a) {
      uv[a] = (j[a] + 0.5f * F[a]) * inv;
      e[a] = uv[a] - ut[((long long)b * L::D + a) * G.plane + node];
      acc += (double)e[a] * (double)e[a];
    }
    if (dLdA) {
      const float s = (float)(2.0 * inv_count) * inv;
      float eu = e[0] * uv[0] + e[1] * uv[1] + e[2] * uv[2];
#pragma unroll
      for (int q = 0; q < L::Q; ++q) {
        float ec = 0.f;  // e . c_q
        if (L::cx[q] > 0) ec += e[0];
        if (L::cx[q] < 0) ec -= e[0];
        if (L::cy[q] > 0) ec += e[1];
        if (L::cy[q] < 0) ec -= e[1];
        if (L::cz[q] > 0) ec += e[2];
        if (L::cz[q] < 0) ec -= e[2];
        int xd = wrap_sub(x, L::cx[q], G.nx), yd = wrap_sub(y, L::cy[q], G.ny),
            zd = wrap_sub(z, L::cz[q], G.nz);
        dLdA[cell(G, b, q, L::Q, xd, yd, zd)] = s * (ec - eu);
      }
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// out = scale * sum of n partials, one block, fixed order.
static __global__ __launch_bounds__(256) void sum_partials_kernel(const double* __restrict__ partial,
                                                           int n, double scale,
                                                           double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) s += partial[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] * scale;
}

// Adam with L2 weight decay folded into the gradient.
static __global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p,
                                                   const float* __restrict__ grad,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   long long n, float lr, float b1, float b2,
                                                   float omb1, float omb2, float eps, float wd,
                                                   float bc1, float bc2) {
  // omb1 = 1 - b1 and omb2 = 1 - b2 come from the host in float64: formed
  // here from the float32 betas, 1 - 0.999f would be off by 1.3e-5
  long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n) return;
  float g = grad[i] + wd * p[i];
  float mi = b1 * m[i] + omb1 * g;
  float vi = b2 * v[i] + omb2 * g * g;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// dst[b][c][Z][Y][X] = mean over the f x f (x f) block of src.
static __global__ __launch_bounds__(256) void box_filter_kernel(const float* __restrict__ src,
                                                         float* __restrict__ dst, int batch,
                                                         int ch, int nx, int ny, int nz, int f,
                                                         int fz) {
  const int cx = nx / f, cy = ny / f, cz = nz / fz;
  long long total = (long long)batch * ch * cz * cy * cx;
  long long n = blockIdx.x * 256LL + threadIdx.x;
  if (n >= total) return;
  int X = (int)(n % cx);
  long long r = n / cx;
  int Y = (int)(r % cy);
  r /= cy;
  int Z = (int)(r % cz);
  long long bc = r / cz;
  const float* s = src + bc * (long long)nz * ny * nx;
  float acc = 0.f;
  for (int dz = 0; dz < fz; ++dz)
    for (int dy = 0; dy < f; ++dy)
      for (int dx = 0; dx < f; ++dx)
        acc += s[((long long)(Z * fz + dz) * ny + (Y * f + dy)) * nx + X * f + dx];
  dst[n] = acc / (float)(f * f * fz);
}

// Sub-sampling filter of the SI's training set ("Definition of the Training
// Dataset": keep one lattice point in every f along each axis) applied to a
// pull-shifted fine state: the coarse canonical population at X is the fine
// one at f X, and in the pull-shifted form of both grids that reads
//   dst_q(X) = src_q(f X + (f - 1) c_q)   (periodic on the fine grid).
// fz = f for 3-D grids, 1 for 2-D ones.
template <class L>
__global__ __launch_bounds__(256) void subsample_kernel(const float* __restrict__ src,
                                                        float* __restrict__ dst, int batch,
                                                        int nx, int ny, int nz, int f, int fz) {
  const int cx = nx / f, cy = ny / f, cz = nz / fz;
  const long long total = (long long)batch * cz * cy * cx;
  const long long n = blockIdx.x * 256LL + threadIdx.x;
  if (n >= total) return;
  const int X = (int)(n % cx);
  long long r = n / cx;
  const int Y = (int)(r % cy);
  r /= cy;
  const int Z = (int)(r % cz);
  const int b = (int)(r / cz);
  const long long fplane = (long long)nx * ny * nz, cplane = (long long)cx * cy * cz;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    int xs = (X * f + (f - 1) * L::cx[q]) % nx, ys = (Y * f + (f - 1) * L::cy[q]) % ny,
        zs = (Z * fz + (fz - 1) * L::cz[q]) % nz;
    xs += xs < 0 ? nx : 0;
    ys += ys < 0 ? ny : 0;
    zs += zs < 0 ? nz : 0;
    dst[((long long)b * L::Q + q) * cplane + ((long long)Z * cy + Y) * cx + X] =
        src[((long long)b * L::Q + q) * fplane + ((long long)zs * ny + ys) * nx + xs];
  }
}

// Population loss of eq. nn-loss on a node subset S: L = sum over the listed
// nodes and q of (A_q(x) - T_q(x))^2, with A the model's state after the
// unrolled steps and T the target, both pull-shifted, so that A_q(x) is the
// post-collision population of node x (the anti-streaming of the SI's
// Fig. 2 is the layout itself).  nodes: flat indices b * plane + node,
// distinct.  dLdA (may be null) gets 2 (A - T) at the listed nodes only.  An
// index outside [0, batch * plane) makes the loss NaN.  Block partials in
// float64, reduced in a fixed order.
template <class L>
__global__ __launch_bounds__(256) void population_sse_kernel(const float* __restrict__ A,
                                                             const float* __restrict__ T,
                                                             const int* __restrict__ nodes,
                                                             int n, float* __restrict__ dLdA,
                                                             double* __restrict__ partial, Grid G) {
  double acc = 0.0;
  const long long total = (long long)G.plane * G.batch;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const int k = nodes[i];
    if (k < 0 || k >= total) {
      acc += __builtin_nan("");
      continue;
    }
    const long long b = k / G.plane, node = k - b * G.plane;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      const long long e = (b * L::Q + q) * G.plane + node;
      const double d = (double)A[e] - (double)T[e];
      acc += d * d;
      if (dLdA) dLdA[e] = (float)(2.0 * d);
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

}  // namespace lbm
