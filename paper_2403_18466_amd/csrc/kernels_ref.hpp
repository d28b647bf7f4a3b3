// kernels_ref.hpp -- float64 reference instance of the learned-collision
// step: the same map as the float32 / bf16 kernels (eq. lbe-sm with the
// collision of eq. nn-model-full, the kappa projection of the SI's network
// section, the exact difference method of eq. fext), with every quantity in
// float64: the stored populations, the parameters, the network and the
// physics.  One thread per node and no blocking: a GPU run of the reference
// precision for workloads too long for the CPU (thousands of steps of a
// 1024^2 field), itself checked against the oracle on small grids.
//
// Storage: float64 deviations A_q = f_q - w_q rho0, [batch][Q][nz][ny][nx],
// pull-shifted like the float32 state (pre-collision f_q(x) = A_q(x - c_q)).
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.hpp"

namespace lbm {

// F(x) of the configured body force in float64, the argument reduced
// exactly in integers (sin(2 pi m / n) with m = k s mod n).
__device__ inline double ref_sin_frac(long long num, long long den) {
  long long r = num % den;
  if (r < 0) r += den;
  return sinpi(2.0 * (double)r / (double)den);
}

struct RefParams {
  int force_kind, force_k;
  double force_amp, rho0, tau, knn;  // knn = s_out / tau
};

// Second-order equilibrium deviation (eq. feq, c_s^2 = 1/3) from drho and j.
template <class L>
__device__ inline void ref_feq(double rho0, double drho, const double j[3], double out[L::Q]) {
  const double rho = rho0 + drho;
  const double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    const double cu = L::cx[q] * u[0] + L::cy[q] * u[1] + L::cz[q] * u[2];
    out[q] = L::wd[q] * (drho + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
  }
}

// One step over every node: gather, moments, BGK, the network Q -> H -> H ->
// Q with tanh (H = 0: none), projection of the whole update, force, store.
// theta (packed [W1 b1 W2 b2 W3 b3], float64) is staged in LDS by the block.
template <class L, int H>
__global__ __launch_bounds__(128) void ref_step_f64_kernel(const double* __restrict__ A,
                                                           double* __restrict__ B,
                                                           const double* __restrict__ theta,
                                                           Grid G, RefParams p) {
  constexpr int Q = L::Q;
  constexpr int NP = H > 0 ? H * Q + H + H * H + H + Q * H + Q : 1;
  constexpr int oW1 = 0, ob1 = H * Q, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H,
                ob3 = oW3 + Q * H;
  __shared__ double th[NP];
  if constexpr (H > 0) {
    for (int i = threadIdx.x; i < NP; i += blockDim.x) th[i] = theta[i];
    __syncthreads();
  }
  const long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (n >= (long long)G.plane * G.batch) return;
  const int x = (int)(n % G.nx);
  long long r = n / G.nx;
  const int y = (int)(r % G.ny);
  r /= G.ny;
  const int z = (int)(r % G.nz);
  const int b = (int)(r / G.nz);
  auto at = [&](int q, int xx, int yy, int zz) {
    return (((long long)(b * Q + q) * G.nz + zz) * G.ny + yy) * G.nx + xx;
  };
  double g[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q)
    g[q] = A[at(q, wrap_sub(x, L::cx[q], G.nx), wrap_sub(y, L::cy[q], G.ny),
                wrap_sub(z, L::cz[q], G.nz))];
  // moments (the w rho0 part sums to rho0 and carries no momentum)
  double drho = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    drho += g[q];
    j[0] += L::cx[q] * g[q];
    j[1] += L::cy[q] * g[q];
    j[2] += L::cz[q] * g[q];
  }
  double geq[Q], upd[Q];
  ref_feq<L>(p.rho0, drho, j, geq);
#pragma unroll
  for (int q = 0; q < Q; ++q) upd[q] = -(g[q] - geq[q]) / p.tau;
  if constexpr (H > 0) {
    double h1[H], y3[Q];
#pragma unroll
    for (int o = 0; o < H; ++o) {
      double a = th[ob1 + o];
#pragma unroll
      for (int i = 0; i < Q; ++i) a += th[oW1 + o * Q + i] * g[i];
      h1[o] = tanh(a);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) y3[q] = th[ob3 + q];
    // layer 2 one unit at a time, each unit's output folded into layer 3
    for (int o = 0; o < H; ++o) {
      double a = th[ob2 + o];
#pragma unroll
      for (int k = 0; k < H; ++k) a += th[oW2 + o * H + k] * h1[k];
      const double h2 = tanh(a);
#pragma unroll
      for (int q = 0; q < Q; ++q) y3[q] += th[oW3 + q * H + o] * h2;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) upd[q] += p.knn * y3[q];
  }
  // kappa projection off span{1, c_x, c_y, c_z}
  {
    double s = 0.0, m[3] = {0.0, 0.0, 0.0}, n2[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      s += upd[q];
      m[0] += L::cx[q] * upd[q];
      m[1] += L::cy[q] * upd[q];
      m[2] += L::cz[q] * upd[q];
      n2[0] += L::cx[q] * L::cx[q];
      n2[1] += L::cy[q] * L::cy[q];
      n2[2] += L::cz[q] * L::cz[q];
    }
    const double k1 = -s / Q;
    double k[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) k[a] = n2[a] > 0.0 ? -m[a] / n2[a] : 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) upd[q] += k1 + k[0] * L::cx[q] + k[1] * L::cy[q] + k[2] * L::cz[q];
  }
  // exact-difference-method force: f^eq(rho, j + F) - f^eq(rho, j), not projected
  double F[3] = {0.0, 0.0, 0.0};
  if (p.force_kind == 1) {
    F[0] = p.force_amp * ref_sin_frac((long long)p.force_k * y, G.ny);
  } else if (p.force_kind == 2) {
    F[0] = p.force_amp * ref_sin_frac((long long)p.force_k * y, G.ny);
    F[1] = p.force_amp * ref_sin_frac((long long)p.force_k * z, G.nz);
    F[2] = p.force_amp * ref_sin_frac((long long)p.force_k * x, G.nx);
  }
  double fext[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) fext[q] = 0.0;
  if (p.force_kind != 0) {
    const double js[3] = {j[0] + F[0], j[1] + F[1], j[2] + F[2]};
    double e1[Q];
    ref_feq<L>(p.rho0, drho, js, e1);
#pragma unroll
    for (int q = 0; q < Q; ++q) fext[q] = e1[q] - geq[q];
  }
  // post-collision vector stored at x: the next step's pull-shifted state
#pragma unroll
  for (int q = 0; q < Q; ++q) B[at(q, x, y, z)] = g[q] + upd[q] + fext[q];
}

}  // namespace lbm
