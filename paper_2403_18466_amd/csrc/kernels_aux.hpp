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
__global__ __launch_bounds__(256) void sum_partials_kernel(const double* __restrict__ partial,
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
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p,
                                                   const float* __restrict__ grad,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   long long n, float lr, float b1, float b2,
                                                   float eps, float wd, float bc1, float bc2) {
  long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n) return;
  float g = grad[i] + wd * p[i];
  float mi = b1 * m[i] + (1.f - b1) * g;
  float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// dst[b][c][Z][Y][X] = mean over the f x f (x f) block of src.
__global__ __launch_bounds__(256) void box_filter_kernel(const float* __restrict__ src,
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

}  // namespace lbm
