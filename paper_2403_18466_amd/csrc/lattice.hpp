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

// Body force of eq. fext at integer node (x, y, z), read from tables that
// the context fills once in float64 on the host (rounded to float32):
// F_x(y) for both forcing kinds, F_y(z) and F_z(x) for the three-component
// forcing.  The pointers are null where a kind does not use them.
struct Force {
  int kind;           // 0 none, 1 Kolmogorov F_x(y), 2 three-component sine
  const float* fx_y;  // [ny]
  const float* fy_z;  // [nz]
  const float* fz_x;  // [nx]
};

// Lanes past the end of a row (x >= nx, whose results are never stored)
// read the table entry of the row's last node.
__device__ inline void body_force(const Force& f, const Grid& G, int x, int y, int z,
                                  float F[3]) {
  F[0] = F[1] = F[2] = 0.f;
  if (f.kind != 0) F[0] = f.fx_y[y];
  if (f.kind == 2) {
    F[1] = f.fy_z[z];
    F[2] = f.fz_x[x < G.nx ? x : G.nx - 1];
  }
}

// Component a of a velocity vector of population q (compile-time constant).
template <class L>
__device__ constexpr int comp(int q, int a) {
  return a == 0 ? L::cx[q] : (a == 1 ? L::cy[q] : L::cz[q]);
}

// sum_q c_qa v_q with the signs resolved at compile time; the first nonzero
// term starts the sum (no float additions of zero).
template <class L, int a, int q = 0>
__device__ inline float csum_from(const float v[L::Q], float acc, bool started) {
  if constexpr (q == L::Q) {
    return started ? acc : 0.f;
  } else {
    constexpr int c = comp<L>(q, a);
    if constexpr (c == 0) {
      return csum_from<L, a, q + 1>(v, acc, started);
    } else {
      const float term = c > 0 ? v[q] : -v[q];
      return csum_from<L, a, q + 1>(v, started ? acc + term : term, true);
    }
  }
}
template <class L, int a>
__device__ inline float csum(const float v[L::Q]) {
  return csum_from<L, a, 0>(v, 0.f, false);
}
template <class L>
__device__ inline float qsum(const float v[L::Q]) {
  float s = v[0];
#pragma unroll
  for (int q = 1; q < L::Q; ++q) s += v[q];
  return s;
}

// Node moments of a deviation vector g (SI: rho = sum f, rho u = sum f c);
// the w rho0 part sums to rho0 and contributes no momentum.  j[2] = 0 for
// two-dimensional lattices.
template <class L>
__device__ inline void moments(const float g[L::Q], float& drho, float j[3]) {
  drho = qsum<L>(g);
  j[0] = csum<L, 0>(g);
  j[1] = csum<L, 1>(g);
  j[2] = L::D == 3 ? csum<L, 2>(g) : 0.f;
}

// c_q . v with compile-time signs (z ignored for two-dimensional lattices).
template <class L, int q>
__device__ inline float cdot(const float v[3]) {
  float r = 0.f;
  bool started = false;
#pragma unroll
  for (int a = 0; a < L::D; ++a) {
    const int c = comp<L>(q, a);
    if (c != 0) {
      const float t = c > 0 ? v[a] : -v[a];
      r = started ? r + t : t;
      started = true;
    }
  }
  return r;
}

template <class L>
__device__ inline float dot3(const float a[3], const float b[3]) {
  float r = a[0] * b[0];
  r = __builtin_fmaf(a[1], b[1], r);
  if constexpr (L::D == 3) r = __builtin_fmaf(a[2], b[2], r);
  return r;
}

template <class L, int q = 0>
struct Unroll {
  // Equilibrium deviation of eq. feq (c_s^2 = 1/3):
  //   f^eq_q - w_q rho0 = w_q [drho + rho (3 c.u + 9/2 (c.u)^2 - 3/2 |u|^2)]
  static __device__ inline void feq(float drho, float rho, const float u[3], float uu,
                                    float geq[L::Q]) {
    if constexpr (q < L::Q) {
      if constexpr (L::cx[q] == 0 && L::cy[q] == 0 && L::cz[q] == 0) {
        geq[q] = L::w[q] * __builtin_fmaf(rho, -1.5f * uu, drho);
      } else {
        float cu = cdot<L, q>(u);
        // 3 cu + 9/2 cu^2 - 3/2 |u|^2 as cu (3 + 9/2 cu) - 3/2 |u|^2: two FMAs
        float p = __builtin_fmaf(cu, __builtin_fmaf(4.5f, cu, 3.f), -1.5f * uu);
        geq[q] = L::w[q] * __builtin_fmaf(rho, p, drho);
      }
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
  const float k1 = -s * (1.f / L::Q);
  const float ka[3] = {-m[0] * (1.f / L::csum2), -m[1] * (1.f / L::csum2),
                       -m[2] * (1.f / L::csum2)};
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    float d = k1;
#pragma unroll
    for (int a = 0; a < L::D; ++a) {
      const int c = comp<L>(q, a);
      if (c > 0) d += ka[a];
      if (c < 0) d -= ka[a];
    }
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
