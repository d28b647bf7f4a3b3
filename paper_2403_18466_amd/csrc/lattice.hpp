// lattice.hpp -- velocity sets and the node-local physics of one collision,
// in float32, for the GPU kernels.
//
// Paper: Ortali et al., "Kinetic data-driven approach to turbulence subgrid
// modeling" (arXiv:2403.18466), SI section "Numerical Method".
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

// D2Q9 in the ordering convention of the SI's Table S1 (rest vector, axis
// vectors in lexicographic order, diagonals in lexicographic order).
struct D2Q9 {
  static constexpr int Q = 9, D = 2;
  static constexpr int cx[Q] = {0, -1, 0, 0, 1, -1, -1, 1, 1};
  static constexpr int cy[Q] = {0, 0, -1, 1, 0, -1, 1, -1, 1};
  static constexpr int cz[Q] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr float w[Q] = {4.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f,
                                 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
  static constexpr double wd[Q] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                                   1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
  static constexpr float csum2 = 6.f;  // sum_q c_qx^2 (the kappa denominator)
};

// D3Q19: velocities and weights of Table S1, in its order.
struct D3Q19 {
  static constexpr int Q = 19, D = 3;
  static constexpr int cx[Q] = {0, -1, 0, 0, 0, 0, 1, -1, -1, -1, -1, 0, 0, 0, 0, 1, 1, 1, 1};
  static constexpr int cy[Q] = {0, 0, -1, 0, 0, 1, 0, -1, 0, 0, 1, -1, -1, 1, 1, -1, 0, 0, 1};
  static constexpr int cz[Q] = {0, 0, 0, -1, 1, 0, 0, 0, -1, 1, 0, -1, 1, -1, 1, 0, -1, 1, 0};
  static constexpr float w[Q] = {1.f / 3.f,  1.f / 18.f, 1.f / 18.f, 1.f / 18.f, 1.f / 18.f,
                                 1.f / 18.f, 1.f / 18.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f,
                                 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f,
                                 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
  static constexpr double wd[Q] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                                   1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                   1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                   1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
  static constexpr float csum2 = 10.f;
};

// Geometry of one launch: a batch of periodic fields stored as
// [batch][Q][nz][ny][nx] float32 planes.
struct Grid {
  int nx, ny, nz, batch;
  int plane;  // nx * ny * nz
};

// Body force of eq. fext at integer node (x, y, z).
struct Force {
  int kind;  // 0 none, 1 Kolmogorov F_x(y), 2 three-component sine
  int k;
  float amp;
};

__device__ inline float sin_frac(long long num, long long den) {
  // sin(2 pi num / den) with the argument reduced exactly in integers
  long long r = num % den;
  if (r < 0) r += den;
  return (float)sinpi(2.0 * (double)r / (double)den);
}

__device__ inline void body_force(const Force& f, const Grid& G, int x, int y, int z,
                                  float F[3]) {
  F[0] = F[1] = F[2] = 0.f;
  if (f.kind == 1) {
    F[0] = f.amp * sin_frac((long long)f.k * y, G.ny);
  } else if (f.kind == 2) {
    F[0] = f.amp * sin_frac((long long)f.k * y, G.ny);
    F[1] = f.amp * sin_frac((long long)f.k * z, G.nz);
    F[2] = f.amp * sin_frac((long long)f.k * x, G.nx);
  }
}

// Node moments of a deviation vector g (SI: rho = sum f, rho u = sum f c);
// the w rho0 part sums to rho0 and contributes no momentum.
template <class L>
__device__ inline void moments(const float g[L::Q], float& drho, float j[3]) {
  float s = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    s += g[q];
    if (L::cx[q] > 0) jx += g[q];
    if (L::cx[q] < 0) jx -= g[q];
    if (L::cy[q] > 0) jy += g[q];
    if (L::cy[q] < 0) jy -= g[q];
    if (L::cz[q] > 0) jz += g[q];
    if (L::cz[q] < 0) jz -= g[q];
  }
  drho = s;
  j[0] = jx;
  j[1] = jy;
  j[2] = jz;
}

template <class L, int q>
__device__ inline float cdot(const float v[3]) {
  float r = 0.f;
  if (L::cx[q] > 0) r += v[0];
  if (L::cx[q] < 0) r -= v[0];
  if (L::cy[q] > 0) r += v[1];
  if (L::cy[q] < 0) r -= v[1];
  if (L::D == 3) {
    if (L::cz[q] > 0) r += v[2];
    if (L::cz[q] < 0) r -= v[2];
  }
  return r;
}

template <class L, int q = 0>
struct Unroll {
  // Equilibrium deviation of eq. feq (c_s^2 = 1/3):
  //   f^eq_q - w_q rho0 = w_q [drho + rho (3 c.u + 9/2 (c.u)^2 - 3/2 |u|^2)]
  static __device__ inline void feq(float drho, float rho, const float u[3], float uu,
                                    float geq[L::Q]) {
    if constexpr (q < L::Q) {
      float cu = cdot<L, q>(u);
      float p = __builtin_fmaf(4.5f * cu, cu, __builtin_fmaf(3.f, cu, -1.5f * uu));
      geq[q] = L::w[q] * __builtin_fmaf(rho, p, drho);
      Unroll<L, q + 1>::feq(drho, rho, u, uu, geq);
    }
  }
  // Exact-difference-method force term of eq. fext,
  //   f^eq(rho, u + du) - f^eq(rho, u),  du = F / rho,
  // written as a difference so that no large terms cancel:
  //   w rho [3 c.du + 9/2 c.du (2 c.u + c.du) - 3/2 du.(2u + du)].
  static __device__ inline void fext(float rho, const float u[3], const float du[3],
                                     float dd, float out[L::Q]) {
    if constexpr (q < L::Q) {
      float cu = cdot<L, q>(u);
      float cd = cdot<L, q>(du);
      float p = 3.f * cd + 4.5f * cd * (2.f * cu + cd) - 1.5f * dd;
      out[q] = L::w[q] * rho * p;
      Unroll<L, q + 1>::fext(rho, u, du, dd, out);
    }
  }
};

// Orthogonal projection off span{1, c_x, c_y[, c_z]} (the kappa layer of the
// SI, with the D2Q9 denominators Q = 9 and sum c^2 = 6, and the printed D3Q19
// ones 19 and 10):  v_q += k1 + k2 c_qx + k3 c_qy + k4 c_qz,
// k1 = -sum v / Q, k_{a+1} = -sum v c_a / sum c_a^2.
template <class L>
__device__ inline void project(float v[L::Q]) {
  float s, m[3];
  moments<L>(v, s, m);
  float k1 = -s * (1.f / L::Q);
  float ka[3] = {-m[0] * (1.f / L::csum2), -m[1] * (1.f / L::csum2), -m[2] * (1.f / L::csum2)};
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    float d = k1;
    if (L::cx[q] > 0) d += ka[0];
    if (L::cx[q] < 0) d -= ka[0];
    if (L::cy[q] > 0) d += ka[1];
    if (L::cy[q] < 0) d -= ka[1];
    if (L::cz[q] > 0) d += ka[2];
    if (L::cz[q] < 0) d -= ka[2];
    v[q] += d;
  }
}

// Periodic neighbour index: (i - c) mod n for c in {-1, 0, 1}.
__device__ inline int wrap_sub(int i, int c, int n) {
  int r = i - c;
  if (r < 0) r += n;
  if (r >= n) r -= n;
  return r;
}

}  // namespace lbm
