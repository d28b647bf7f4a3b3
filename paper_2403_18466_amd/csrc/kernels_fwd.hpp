// kernels_fwd.hpp -- forward kernels of the lattice Boltzmann step:
// equilibrium initialisation, pull-shift conversion, moments and
// diagnostics, the BGK stream-collide step and the learned-collision
// stream-collide step.
//
// Storage: float32 deviations A_q = f_q - w_q rho0, [batch][Q][nz][ny][nx],
// in pull-shifted form (pre-collision f_q(x) - w_q rho0 = A_q(x - c_q)).
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.hpp"
#include "mlp.hpp"

namespace lbm {

// Decoded position of flat node index n of one field.
__device__ inline void decode(const Grid& G, long long n, int& x, int& y, int& z, int& b) {
  x = (int)(n % G.nx);
  long long r = n / G.nx;
  y = (int)(r % G.ny);
  r /= G.ny;
  z = (int)(r % G.nz);
  b = (int)(r / G.nz);
}

__device__ inline long long cell(const Grid& G, int b, int q, int Q, int x, int y, int z) {
  return (((long long)(b * Q + q) * G.nz + z) * G.ny + y) * G.nx + x;
}

// Gather the pre-collision deviations of node (x, y, z) of field b:
// g_q = A_q(x - c_q).
template <class L>
__device__ inline void gather(const float* __restrict__ A, const Grid& G, int b, int x, int y,
                              int z, float g[L::Q]) {
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    int xs = wrap_sub(x, L::cx[q], G.nx), ys = wrap_sub(y, L::cy[q], G.ny),
        zs = wrap_sub(z, L::cz[q], G.nz);
    g[q] = A[cell(G, b, q, L::Q, xs, ys, zs)];
  }
}

// ---------------------------------------------------------------------------
// Equilibrium initial state: A_q(x - c_q) = f^eq_q(rho(x), u(x)) - w_q rho0.
// ---------------------------------------------------------------------------
template <class L>
__global__ void init_kernel(const float* __restrict__ rho, const float* __restrict__ u,
                            float* __restrict__ A, Grid G, float rho0) {
  long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  long long total = (long long)G.plane * G.batch;
  if (n >= total) return;
  int x, y, z, b;
  decode(G, n, x, y, z, b);
  long long node = n - (long long)b * G.plane;
  float r = rho[n];
  float uv[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < L::D; ++a) uv[a] = u[((long long)b * L::D + a) * G.plane + node];
  float uu = uv[0] * uv[0] + uv[1] * uv[1] + uv[2] * uv[2];
  float geq[L::Q];
  Unroll<L>::feq(r - rho0, r, uv, uu, geq);
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    int xd = wrap_sub(x, L::cx[q], G.nx), yd = wrap_sub(y, L::cy[q], G.ny),
        zd = wrap_sub(z, L::cz[q], G.nz);
    A[cell(G, b, q, L::Q, xd, yd, zd)] = geq[q];
  }
}

// dir = +1: dst_q(x) = src_q(x - c_q); dir = -1: dst_q(x) = src_q(x + c_q).
template <class L>
__global__ void shift_kernel(const float* __restrict__ src, float* __restrict__ dst, Grid G,
                             int dir) {
  long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  long long total = (long long)G.plane * G.batch;
  if (n >= total) return;
  int x, y, z, b;
  decode(G, n, x, y, z, b);
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    int xs = wrap_sub(x, dir * L::cx[q], G.nx), ys = wrap_sub(y, dir * L::cy[q], G.ny),
        zs = wrap_sub(z, dir * L::cz[q], G.nz);
    dst[cell(G, b, q, L::Q, x, y, z)] = src[cell(G, b, q, L::Q, xs, ys, zs)];
  }
}

// ---------------------------------------------------------------------------
// Moments and float64 diagnostics.  Grid (MOM_BLOCKS, batch) x 256 threads;
// each block writes {mass, kinetic energy, non-finite count} partials, summed
// in a fixed order by diag_reduce_kernel.
// ---------------------------------------------------------------------------
constexpr int MOM_BLOCKS = 512;

template <class L>
__global__ __launch_bounds__(256) void moments_kernel(const float* __restrict__ A,
                                                      float* __restrict__ rho,
                                                      float* __restrict__ u,
                                                      double* __restrict__ partial, Grid G,
                                                      float rho0, Force Fc) {
  const int b = blockIdx.y;
  double mass = 0.0, ke = 0.0, bad = 0.0;
  for (long long node = blockIdx.x * 256LL + threadIdx.x; node < G.plane;
       node += (long long)gridDim.x * 256) {
    int x, y, z, bb;
    decode(G, node, x, y, z, bb);
    float g[L::Q];
    gather<L>(A, G, b, x, y, z, g);
    bool finite = true;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) finite = finite && __builtin_isfinite(g[q]);
    float drho, j[3], F[3];
    moments<L>(g, drho, j);
    body_force(Fc, G, x, y, z, F);
    float r = rho0 + drho;
    float inv = 1.f / r;
    float uv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) uv[a] = (j[a] + 0.5f * F[a]) * inv;
    long long pn = (long long)b * G.plane + node;
    if (rho) rho[pn] = r;
    if (u) {
#pragma unroll
      for (int a = 0; a < L::D; ++a) u[((long long)b * L::D + a) * G.plane + node] = uv[a];
    }
    if (finite) {
      double rd = r, uu = 0.0;
#pragma unroll
      for (int a = 0; a < L::D; ++a) uu += (double)uv[a] * (double)uv[a];
      mass += rd;
      ke += 0.5 * rd * uu;
    } else {
      bad += 1.0;
    }
  }
  __shared__ double red[3][256];
  red[0][threadIdx.x] = mass;
  red[1][threadIdx.x] = ke;
  red[2][threadIdx.x] = bad;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
      red[2][threadIdx.x] += red[2][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) partial[((long long)b * gridDim.x + blockIdx.x) * 3 + threadIdx.x] =
      red[threadIdx.x][0];
}

// One block of 256 threads per field; partial: [batch][nblk][3].
__global__ __launch_bounds__(256) void diag_reduce_kernel(const double* __restrict__ partial,
                                                          double* __restrict__ diag, int nblk) {
  const int b = blockIdx.x;
  __shared__ double red[3][256];
  double s[3] = {0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < nblk; k += 256)
    for (int c = 0; c < 3; ++c) s[c] += partial[((long long)b * nblk + k) * 3 + c];
  for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = s[c];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 4) diag[b * 4 + threadIdx.x] = threadIdx.x < 3 ? red[threadIdx.x][0] : 0.0;
}

// ---------------------------------------------------------------------------
// Node-local collision pieces shared by the step kernels (all float32).
// ---------------------------------------------------------------------------

// BGK part: moments, equilibrium and Omega_q = (f^eq_q - f_q)/tau
// (eq. bgk-sm with dt = 1, eq. feq).
template <class L>
__device__ inline void bgk_update(const float g[L::Q], float rho0, float omega, float upd[L::Q],
                                  float& rho, float u[3]) {
  float drho, j[3];
  moments<L>(g, drho, j);
  rho = rho0 + drho;
  float inv = 1.f / rho;
  u[0] = j[0] * inv;
  u[1] = j[1] * inv;
  u[2] = j[2] * inv;
  float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  float geq[L::Q];
  Unroll<L>::feq(drho, rho, u, uu, geq);
#pragma unroll
  for (int q = 0; q < L::Q; ++q) upd[q] = (geq[q] - g[q]) * omega;
}

// Projection of the whole update (kappa layer), then the EDM force, then
// post = pre + update + force (eq. lbe-sm).
template <class L>
__device__ inline void finish_collision(const float g[L::Q], float upd[L::Q], float rho,
                                        const float u[3], const float F[3], bool forced,
                                        float post[L::Q]) {
  project<L>(upd);
  if (forced) {
    float inv = 1.f / rho;
    float du[3] = {F[0] * inv, F[1] * inv, F[2] * inv};
    float dd = du[0] * (2.f * u[0] + du[0]) + du[1] * (2.f * u[1] + du[1]) +
               du[2] * (2.f * u[2] + du[2]);
    float fe[L::Q];
    Unroll<L>::fext(rho, u, du, dd, fe);
#pragma unroll
    for (int q = 0; q < L::Q; ++q) post[q] = g[q] + upd[q] + fe[q];
  } else {
#pragma unroll
    for (int q = 0; q < L::Q; ++q) post[q] = g[q] + upd[q];
  }
}

// ---------------------------------------------------------------------------
// BGK stream-collide, one node per thread.  Blocks cover 256 consecutive x
// of one row (b, z, y); the launch is 1-D over rows x ceil(nx / 256).
// ---------------------------------------------------------------------------
template <class L>
__global__ __launch_bounds__(256) void bgk_step_kernel(const float* __restrict__ Ain,
                                                       float* __restrict__ Aout, Grid G,
                                                       Force Fc, float rho0, float omega,
                                                       int nxc) {
  const int row = blockIdx.x / nxc, xc = blockIdx.x - row * nxc;
  const int x = xc * 256 + threadIdx.x;
  if (x >= G.nx) return;
  const int y = row % G.ny, t = row / G.ny, z = t % G.nz, b = t / G.nz;
  float g[L::Q];
  gather<L>(Ain, G, b, x, y, z, g);
  float upd[L::Q], rho, u[3], F[3];
  bgk_update<L>(g, rho0, omega, upd, rho, u);
  body_force(Fc, G, x, y, z, F);
  float post[L::Q];
  finish_collision<L>(g, upd, rho, u, F, Fc.kind != 0, post);
#pragma unroll
  for (int q = 0; q < L::Q; ++q) Aout[cell(G, b, q, L::Q, x, y, z)] = post[q];
}

__device__ inline void wave_lds_sync() {
  // LDS operations of one wavefront complete in issue order; the fences keep
  // the compiler from moving a lane's read of another lane's write across.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Learned-collision stream-collide (eq. nn-model-full with the kappa layer).
//
// Persistent: every wavefront keeps the network weights in registers and
// walks a contiguous range of work items; an item is 64 consecutive x of
// one row, one node per lane.  Lanes gather, compute the BGK part and the
// projection in node layout; the network runs on the matrix cores for the
// four 16-node groups of the item, with the input and output crossing
// between node layout and MFMA layout through a per-wave LDS tile.  The next
// item's populations are loaded before the current item's network runs.
// Workgroups are numbered so that each XCD walks one contiguous part of the
// domain.
// ---------------------------------------------------------------------------
template <class L, int H>
struct StepLds {
  using S = Shape<L::Q, H>;
  static constexpr int SX = 16 * S::KX + 4;  // row stride (floats) of the input tile
  static constexpr int SY = 16 * S::QB + 4;  // row stride of the output tile
  static constexpr int per_wave = 64 * (SX + SY);
};

template <class L, int H, int P>
__global__ __launch_bounds__(256) void nlbm_step_kernel(const float* __restrict__ Ain,
                                                        float* __restrict__ Aout,
                                                        const float* __restrict__ theta, Grid G,
                                                        Force Fc, float rho0, float omega,
                                                        float knn, int nitems, int nxc) {
  using S = Shape<L::Q, H>;
  using LD = StepLds<L, H>;
  using F = typename Frag<P>::T;
  constexpr int Q = L::Q;
  __shared__ float lds[4 * LD::per_wave];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, lg = lane >> 4, li = lane & 15;
  float* X = lds + wave * LD::per_wave;
  float* Y = X + 64 * LD::SX;

  const int nb = gridDim.x, bid = blockIdx.x;
  const int lb = (nb % 8 == 0) ? (bid % 8) * (nb / 8) + bid / 8 : bid;
  const int nw = nb * 4, wv = lb * 4 + wave;
  const int per = (nitems + nw - 1) / nw;
  const int it0 = wv * per, it1 = min(it0 + per, nitems);
  if (it0 >= it1) return;

  Weights<P, S> W;
  W.load(theta);

  auto locate = [&](int it, int& b, int& x, int& y, int& z) {
    int row = it / nxc, xc = it - row * nxc;
    x = xc * 64 + lane;
    y = row % G.ny;
    int t = row / G.ny;
    z = t % G.nz;
    b = t / G.nz;
  };
  auto load = [&](int it, float g[Q]) {
    int b, x, y, z;
    locate(it, b, x, y, z);
    if (x < G.nx) {
      gather<L>(Ain, G, b, x, y, z, g);
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q) g[q] = 0.f;
    }
  };

  float gc[Q];
  load(it0, gc);
  for (int it = it0; it < it1; ++it) {
    float gn[Q];
    if (it + 1 < it1) load(it + 1, gn);

    int b, x, y, z;
    locate(it, b, x, y, z);
    float upd[Q], rho, u[3];
    bgk_update<L>(gc, rho0, omega, upd, rho, u);

    // stage the network input (populations, a constant 1 for the bias
    // column, zero padding) in node-major rows
#pragma unroll
    for (int c = 0; c < 4 * S::KX; ++c) {
      f4 v;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int k = 4 * c + r;
        v[r] = k < Q ? gc[k] : (k == Q ? 1.f : 0.f);
      }
      *reinterpret_cast<f4*>(X + lane * LD::SX + 4 * c) = v;
    }
    wave_lds_sync();
#pragma unroll
    for (int jg = 0; jg < 4; ++jg) {
      const int nrow = 16 * jg + li;
      F xin[S::KX];
#pragma unroll
      for (int c = 0; c < S::KX; ++c)
        xin[c] = to_frag<P>(*reinterpret_cast<const f4*>(X + nrow * LD::SX + 16 * c + 4 * lg));
      F h1[S::HB], h2[S::HB];
#pragma unroll
      for (int ob = 0; ob < S::HB; ++ob) {
        f4 a = mma_row<P, S::KX>(f4{0.f, 0.f, 0.f, 0.f}, W.w1[ob], xin);
        h1[ob] = to_frag<P>(tanh4<P>(a));
      }
#pragma unroll
      for (int ob = 0; ob < S::HB; ++ob) {
        f4 a = mma_row<P, S::HB>(W.b2[ob], W.w2[ob], h1);
        h2[ob] = to_frag<P>(tanh4<P>(a));
      }
#pragma unroll
      for (int ob = 0; ob < S::QB; ++ob) {
        f4 yv = mma_row<P, S::HB>(W.b3[ob], W.w3[ob], h2);
        *reinterpret_cast<f4*>(Y + nrow * LD::SY + 16 * ob + 4 * lg) = yv;
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < Q; ++q) upd[q] = __builtin_fmaf(knn, Y[lane * LD::SY + q], upd[q]);

    float F3[3] = {0.f, 0.f, 0.f};
    if (Fc.kind != 0) body_force(Fc, G, x, y, z, F3);
    float post[Q];
    finish_collision<L>(gc, upd, rho, u, F3, Fc.kind != 0, post);
    if (x < G.nx) {
#pragma unroll
      for (int q = 0; q < Q; ++q) Aout[cell(G, b, q, Q, x, y, z)] = post[q];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) gc[q] = gn[q];
  }
}

}  // namespace lbm
