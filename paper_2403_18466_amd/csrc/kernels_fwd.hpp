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
// Addressing of a 64-node work item (64 consecutive x of row (b, z, y)) with
// buffer instructions: the row part of every address is a wave-uniform
// scalar byte offset, the x part one of three per-lane offsets (x, x - 1,
// x + 1 with periodic wrap).  Buffer accesses are range-checked by the
// hardware against the array size.
// ---------------------------------------------------------------------------
typedef __amdgpu_buffer_rsrc_t rsrc_t;

__device__ inline rsrc_t make_rsrc(const float* p, unsigned bytes) {
  // last descriptor dword of gfx9: 32-bit data format, raw (unformatted) access
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), (short)0, (int)bytes,
                                           0x00020000);
}

struct Item {
  int b, y, z;    // wave-uniform
  int x;          // this lane
  bool active;    // x < nx
  int vx, vm, vp;  // byte offsets of x, (x - 1) mod nx, (x + 1) mod nx
};

// Item `it` of width W (64 for the persistent kernels, 256 for one-node-per-
// thread kernels); nxc = ceil(nx / W) items per row.
__device__ inline Item locate_item(int it, int nxc, const Grid& G, int lane, int W = 64) {
  Item t;
  const int row = it / nxc, xc = it - row * nxc;
  t.y = row % G.ny;
  const int r = row / G.ny;
  t.z = r % G.nz;
  t.b = r / G.nz;
  t.x = xc * W + lane;
  t.active = t.x < G.nx;
  const int xm = t.x == 0 ? G.nx - 1 : t.x - 1;
  const int xp = t.x + 1 >= G.nx ? 0 : t.x + 1;
  t.vx = t.x * 4;
  t.vm = xm * 4;
  t.vp = xp * 4;
  return t;
}

// Walks consecutive items of a contiguous range without integer division
// in the loop: `next()` advances x-chunk, then y, z and b.
struct ItemWalk {
  int xc, y, z, b;
  __device__ inline void start(int it, int nxc, const Grid& G) {
    const int row = it / nxc;
    xc = it - row * nxc;
    y = row % G.ny;
    const int r = row / G.ny;
    z = r % G.nz;
    b = r / G.nz;
  }
  __device__ inline void next(int nxc, const Grid& G) {
    if (++xc == nxc) {
      xc = 0;
      if (++y == G.ny) {
        y = 0;
        if (++z == G.nz) {
          z = 0;
          ++b;
        }
      }
    }
  }
  // s items further on (s >= 0); the carry loop runs floor((xc + s) / nxc)
  // times
  __device__ inline void advance(int s, int nxc, const Grid& G) {
    xc += s;
    while (xc >= nxc) {
      xc -= nxc;
      if (++y == G.ny) {
        y = 0;
        if (++z == G.nz) {
          z = 0;
          ++b;
        }
      }
    }
  }
  // Lane addressing; lanes past the end of the row read node nx - 1 (their
  // results are never stored).
  __device__ inline Item item(const Grid& G, int lane, int W = 64) const {
    Item t;
    t.b = b;
    t.y = y;
    t.z = z;
    t.x = xc * W + lane;
    t.active = t.x < G.nx;
    const int x = t.active ? t.x : G.nx - 1;
    const int xm = x == 0 ? G.nx - 1 : x - 1;
    const int xp = x + 1 >= G.nx ? 0 : x + 1;
    t.vx = x * 4;
    t.vm = xm * 4;
    t.vp = xp * 4;
    return t;
  }
};

// Byte offset of the start of row (z, y) of plane q of field b.
__device__ inline unsigned row_bytes(const Grid& G, int Q, int b, int q, int z, int y) {
  return (unsigned)(((b * Q + q) * G.nz + z) * G.ny + y) * (unsigned)G.nx * 4u;
}

// Offsets of A_q(x - c_q): the pull source of population q of this lane's
// node, which is also the push target of the adjoint.
template <class L, int q>
__device__ inline void pull_offsets(const Grid& G, const Item& t, unsigned& so, int& vo) {
  const int ys = wrap_sub(t.y, L::cy[q], G.ny), zs = wrap_sub(t.z, L::cz[q], G.nz);
  so = row_bytes(G, L::Q, t.b, q, zs, ys);
  vo = L::cx[q] > 0 ? t.vm : (L::cx[q] < 0 ? t.vp : t.vx);
}

// The rows of an item, for kernels that read and write them several times:
// row (zs, ys) of plane q of the item's field starts at byte
//   base + q plane + z[1 - dz] + y[1 - dy],  zs = z - dz, ys = y - dy (periodic),
// the same sum as row_bytes; every term is wave-uniform.
struct ItemRows {
  unsigned base, plane, y[3], z[3];
  __device__ inline ItemRows(const Grid& G, int Q, const Item& t) {
    const unsigned row = (unsigned)G.nx * 4u, slab = row * (unsigned)G.ny;
    plane = slab * (unsigned)G.nz;
    base = (unsigned)(t.b * Q) * plane;
    y[0] = (unsigned)wrap_sub(t.y, 1, G.ny) * row;
    y[1] = (unsigned)t.y * row;
    y[2] = (unsigned)wrap_sub(t.y, -1, G.ny) * row;
    z[0] = (unsigned)wrap_sub(t.z, 1, G.nz) * slab;
    z[1] = (unsigned)t.z * slab;
    z[2] = (unsigned)wrap_sub(t.z, -1, G.nz) * slab;
  }
};

// gather_item, load_local, store_local and scatter_item with the rows of an
// ItemRows.
template <class L>
__device__ inline void gather_rows(rsrc_t src, const ItemRows& r, const Item& t, float g[L::Q]) {
  unsigned qo = r.base;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    const unsigned so = qo + (r.z[1 - L::cz[q]] + r.y[1 - L::cy[q]]);
    const int vo = L::cx[q] > 0 ? t.vm : (L::cx[q] < 0 ? t.vp : t.vx);
    g[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(src, vo, (int)so, 0));
    qo += r.plane;
  }
}
template <class L>
__device__ inline void load_rows(rsrc_t src, const ItemRows& r, const Item& t, float v[L::Q]) {
  unsigned qo = r.base;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    v[q] = __builtin_bit_cast(
        float, __builtin_amdgcn_raw_buffer_load_b32(src, t.vx, (int)(qo + (r.z[1] + r.y[1])), 0));
    qo += r.plane;
  }
}
template <class L, int POLICY = 0>
__device__ inline void store_rows(rsrc_t dst, const ItemRows& r, const Item& t, const float v[L::Q]) {
  unsigned qo = r.base;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v[q]), dst, t.vx,
                                          (int)(qo + (r.z[1] + r.y[1])), POLICY);
    qo += r.plane;
  }
}
template <class L>
__device__ inline void scatter_rows(rsrc_t dst, const ItemRows& r, const Item& t,
                                    const float v[L::Q]) {
  unsigned qo = r.base;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    const unsigned so = qo + (r.z[1 - L::cz[q]] + r.y[1 - L::cy[q]]);
    const int vo = L::cx[q] > 0 ? t.vm : (L::cx[q] < 0 ? t.vp : t.vx);
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v[q]), dst, vo, (int)so, 0);
    qo += r.plane;
  }
}

template <class L, int q = 0>
__device__ inline void gather_item(rsrc_t src, const Grid& G, const Item& t, float g[L::Q]) {
  if constexpr (q < L::Q) {
    unsigned so;
    int vo;
    pull_offsets<L, q>(G, t, so, vo);
    g[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(src, vo, (int)so, 0));
    gather_item<L, q + 1>(src, G, t, g);
  }
}

// Node-local read of all Q planes at this lane's node.
template <class L>
__device__ inline void load_local(rsrc_t src, const Grid& G, const Item& t, float v[L::Q]) {
#pragma unroll
  for (int q = 0; q < L::Q; ++q)
    v[q] = __builtin_bit_cast(
        float, __builtin_amdgcn_raw_buffer_load_b32(src, t.vx, (int)row_bytes(G, L::Q, t.b, q, t.z, t.y), 0));
}

// Cache policy bit "nt" (non-temporal) for stores of a state that the next
// step reads back from HBM anyway.  Measured faster in the bandwidth-bound
// BGK step and in the D2Q9 learned-collision step (0.7% at 4096^2, 5% at
// 8 x 256^2, where less is left in the L2 to write back when the kernel
// ends); the adjoint's stores of lambda are faster without it.
constexpr int kStoreNT = 2;

template <class L, int POLICY = 0>
__device__ inline void store_local(rsrc_t dst, const Grid& G, const Item& t, const float v[L::Q]) {
#pragma unroll
  for (int q = 0; q < L::Q; ++q)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v[q]), dst, t.vx,
                                          (int)row_bytes(G, L::Q, t.b, q, t.z, t.y), POLICY);
}

template <class L, int q = 0>
__device__ inline void scatter_item(rsrc_t dst, const Grid& G, const Item& t, const float v[L::Q]) {
  if constexpr (q < L::Q) {
    unsigned so;
    int vo;
    pull_offsets<L, q>(G, t, so, vo);
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v[q]), dst, vo, (int)so, 0);
    scatter_item<L, q + 1>(dst, G, t, v);
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
// Moments and float64 diagnostics.  Grid (MOMENT_BLOCKS, batch) x 256
// threads; a block walks 256-node row chunks of its field (one node per
// thread, buffer loads as in the step kernels) and writes {mass, kinetic
// energy, non-finite count} partials, summed in a fixed order by
// diag_reduce_kernel.
// ---------------------------------------------------------------------------
constexpr int MOM_BLOCKS = 512;       // loss reductions
constexpr int MOMENT_BLOCKS = 4096;   // moments, per field

template <class L>
__global__ __launch_bounds__(256) void moments_kernel(const float* __restrict__ A,
                                                      float* __restrict__ rho,
                                                      float* __restrict__ u,
                                                      double* __restrict__ partial, Grid G,
                                                      float rho0, Force Fc, int nxc) {
  const int b = blockIdx.y;
  const int per_field = nxc * G.ny * G.nz;
  const unsigned bytes = (unsigned)G.plane * (unsigned)(G.batch * L::Q) * 4u;
  const rsrc_t src = make_rsrc(A, bytes);
  double mass = 0.0, ke = 0.0, bad = 0.0;
  for (int k = blockIdx.x; k < per_field; k += gridDim.x) {
    const Item t = locate_item(b * per_field + k, nxc, G, threadIdx.x, 256);
    if (!t.active) continue;
    float g[L::Q];
    gather_item<L>(src, G, t, g);
    bool finite = true;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) finite = finite && __builtin_isfinite(g[q]);
    float drho, j[3], F[3];
    moments<L>(g, drho, j);
    body_force(Fc, G, t.x, t.y, t.z, F);
    float r = rho0 + drho;
    float inv = 1.f / r;
    float uv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) uv[a] = (j[a] + 0.5f * F[a]) * inv;
    const long long node = ((long long)t.z * G.ny + t.y) * G.nx + t.x;
    // the fields are written with the non-temporal policy, like the step
    if (rho) __builtin_nontemporal_store(r, rho + (long long)b * G.plane + node);
    if (u) {
#pragma unroll
      for (int a = 0; a < L::D; ++a)
        __builtin_nontemporal_store(uv[a], u + ((long long)b * L::D + a) * G.plane + node);
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
static __global__ __launch_bounds__(256) void diag_reduce_kernel(const double* __restrict__ partial,
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
  const float inv = __builtin_amdgcn_rcpf(rho);
  u[0] = j[0] * inv;
  u[1] = j[1] * inv;
  u[2] = L::D == 3 ? j[2] * inv : 0.f;
  const float uu = dot3<L>(u, u);
  float geq[L::Q];
  Unroll<L>::feq(drho, rho, u, uu, geq);
#pragma unroll
  for (int q = 0; q < L::Q; ++q) upd[q] = (geq[q] - g[q]) * omega;
}

// sum_q c_qa c_qb d_q with compile-time signs (the first nonzero term starts
// the sum).
template <class L, int a, int b, int q = 0>
__device__ inline float pisum(const float d[L::Q], float acc = 0.f, bool started = false) {
  if constexpr (q == L::Q) {
    return started ? acc : 0.f;
  } else {
    constexpr int c = comp<L>(q, a) * comp<L>(q, b);
    if constexpr (c == 0) {
      return pisum<L, a, b, q + 1>(d, acc, started);
    } else {
      const float t = c > 0 ? d[q] : -d[q];
      return pisum<L, a, b, q + 1>(d, started ? acc + t : t, true);
    }
  }
}

// Relaxation rate 1 / tau_eff of the Smagorinsky model (SI, "Implementing
// the Smagorinsky Turbulence Model in LBM"; dt = 1, c_s^2 = 1/3, filter
// width 1):  Pi^neq_ab = sum_q c_qa c_qb (f_q - f^eq_q),
// |S| = (3 / (2 tau)) sqrt(2 Pi_ab Pi_ab), tau_eff = tau + 3 C_s^2 |S|.
// c15 = 3 / (2 tau), cs2x3 = 3 C_s^2.
template <class L>
__device__ inline float smag_omega(const float g[L::Q], const float geq[L::Q], float tau,
                                   float c15, float cs2x3) {
  float d[L::Q];
#pragma unroll
  for (int q = 0; q < L::Q; ++q) d[q] = g[q] - geq[q];
  const float pxx = pisum<L, 0, 0>(d), pyy = pisum<L, 1, 1>(d), pxy = pisum<L, 0, 1>(d);
  float diag = pxx * pxx + pyy * pyy, offd = pxy * pxy;
  if constexpr (L::D == 3) {
    const float pzz = pisum<L, 2, 2>(d), pxz = pisum<L, 0, 2>(d), pyz = pisum<L, 1, 2>(d);
    diag = __builtin_fmaf(pzz, pzz, diag);
    offd = __builtin_fmaf(pxz, pxz, __builtin_fmaf(pyz, pyz, offd));
  }
  const float smag = c15 * __builtin_sqrtf(2.f * __builtin_fmaf(2.f, offd, diag));
  return __builtin_amdgcn_rcpf(__builtin_fmaf(cs2x3, smag, tau));
}

// BGK part at the Smagorinsky relaxation time.
template <class L>
__device__ inline void smag_update(const float g[L::Q], float rho0, float tau, float c15,
                                   float cs2x3, float upd[L::Q], float& rho, float u[3]) {
  float drho, j[3];
  moments<L>(g, drho, j);
  rho = rho0 + drho;
  const float inv = __builtin_amdgcn_rcpf(rho);
  u[0] = j[0] * inv;
  u[1] = j[1] * inv;
  u[2] = L::D == 3 ? j[2] * inv : 0.f;
  const float uu = dot3<L>(u, u);
  float geq[L::Q];
  Unroll<L>::feq(drho, rho, u, uu, geq);
  const float omega = smag_omega<L>(g, geq, tau, c15, cs2x3);
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
    const float inv = __builtin_amdgcn_rcpf(rho);
    float du[3] = {F[0] * inv, F[1] * inv, F[2] * inv};
    const float u2[3] = {2.f * u[0] + du[0], 2.f * u[1] + du[1], 2.f * u[2] + du[2]};
    const float dd = dot3<L>(du, u2);
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
// R rows per thread (more loads in flight per thread); NT: non-temporal
// stores (the next step reads the output from HBM anyway); SMAG: relaxation
// at the Smagorinsky tau_eff of each node (tau, c15 = 3 / (2 tau),
// cs2x3 = 3 C_s^2) instead of the fixed rate omega.
template <class L, int R, bool NT, bool SMAG = false>
__global__ __launch_bounds__(256) void bgk_step_kernel(const float* __restrict__ Ain,
                                                       float* __restrict__ Aout, Grid G,
                                                       Force Fc, float rho0, float omega,
                                                       int nxc, float tau = 0.f, float c15 = 0.f,
                                                       float cs2x3 = 0.f) {
  const unsigned bytes = (unsigned)G.plane * (unsigned)(G.batch * L::Q) * 4u;
  const rsrc_t src = make_rsrc(Ain, bytes), dst = make_rsrc(Aout, bytes);
  const int nrow_groups = (G.ny + R - 1) / R;
  const int xc = blockIdx.x % nxc;
  const int rg = blockIdx.x / nxc;
  const int yg = rg % nrow_groups, zb = rg / nrow_groups;
  float g[R][L::Q];
  Item t[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int y = yg * R + r;
    const int yy = y < G.ny ? y : G.ny - 1;
    t[r] = locate_item((zb * G.ny + yy) * nxc + xc, nxc, G, threadIdx.x, 256);
    t[r].active = t[r].active && y < G.ny;
    if (t[r].active) gather_item<L>(src, G, t[r], g[r]);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (!t[r].active) continue;
    float upd[L::Q], rho, u[3], F[3];
    if constexpr (SMAG)
      smag_update<L>(g[r], rho0, tau, c15, cs2x3, upd, rho, u);
    else
      bgk_update<L>(g[r], rho0, omega, upd, rho, u);
    body_force(Fc, G, t[r].x, t[r].y, t[r].z, F);
    float post[L::Q];
    finish_collision<L>(g[r], upd, rho, u, F, Fc.kind != 0, post);
#pragma unroll
    for (int q = 0; q < L::Q; ++q)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, post[q]), dst, t[r].vx,
                                            (int)row_bytes(G, L::Q, t[r].b, q, t[r].z, t[r].y),
                                            NT ? kStoreNT : 0);
  }
}

__device__ inline void wave_lds_sync() {
  // LDS operations of one wavefront complete in issue order; the fences keep
  // the compiler from moving a lane's read of another lane's write across.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Waits until every vector-memory access the wavefront has issued is done
// (s_waitcnt vmcnt(0); the export and LDS counters are not waited on).  One
// counter covers loads and stores, and the compiler cannot assume that they
// complete in order: a wait for a load issued before a burst of stores also
// waits for the stores to be acknowledged.  Called just before such a burst,
// when the loads issued earlier have long arrived, it costs nothing and
// leaves the stores in flight past the later uses of those loads.
__device__ inline void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

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
  // One row per node: the network input (g, the constant 1 of the layer-1
  // bias, zeros up to YC), then the network output y (YQ columns from YO),
  // then 4 columns of padding.  Layer 1 reads 16 KX input columns: where the
  // LDS allows (D2Q9) the columns from YC to YO = 16 KX are stored zeros, so
  // that the read needs no masking; else (D3Q19) YO = YC and the input
  // columns past YC are read as zeros without being stored.  A row stride
  // that is a multiple of 32 floats would put every row on the same banks.
  static constexpr int YC = (L::Q + 1 + 3) / 4 * 4;
  static constexpr int YQ = (L::Q + 3) / 4 * 4;
  static constexpr int ZC = 16 * ((L::Q + 1 + 15) / 16);  // input columns layer 1 reads
  static constexpr int YO = L::Q == 9 ? ZC : YC;
  static constexpr bool ZERO_PAD = YO >= ZC;
  static constexpr int SX0 = YO + YQ + 4;
  static constexpr int SX = SX0 % 32 == 0 ? SX0 + 4 : SX0;  // row stride (floats)
  static constexpr int per_wave = 64 * SX;
  // the layer-3 bias sits in the padding columns of the first 4 QB rows
  // (row 4 ob + g holds b3[16 ob + 4 g .. + 3]), not in registers
  static constexpr int B3 = YO + YQ;
  // wavefronts per SIMD the compiler must leave room for: three for the
  // unforced 16-bit D3Q19 instances and the unforced fp32 D2Q9 one (which
  // the max-ILP scheduler otherwise takes to two: 8% slower), else no
  // constraint
  static constexpr int min_waves(int prec, bool forced) {
    return (!forced && ((L::Q == 19 && prec != P_F32) || (L::Q == 9 && prec == P_F32))) ? 3 : 1;
  }
  // wavefronts per workgroup: the 16-bit D2Q9 instances and the unforced
  // 16-bit D3Q19 one run one workgroup per compute unit (four wavefronts per
  // SIMD for D2Q9, three for D3Q19), so that the weights are staged once per
  // compute unit and each thread stages a quarter as many of them; the
  // others run workgroups of 4 (the forced 16-bit D3Q19 instance needs 187
  // registers per lane, and at three wavefronts per SIMD it would spill)
  static constexpr int waves_per_block(int prec, bool forced) {
    return (prec == P_F32 || (forced && L::Q == 19)) ? 4 : (L::Q == 19 ? 12 : 16);
  }
};

// FORCED: the body force of eq. fext is applied (Force::kind != 0).  The
// unforced instances leave out the force's registers: 108 instead of 120
// registers per lane for the 16-bit D2Q9 instance, 159 instead of 187 for
// D3Q19.
template <class L, int H, int P, bool FORCED>
__global__ __launch_bounds__((64 * StepLds<L, H>::waves_per_block(P, FORCED)))
__attribute__((amdgpu_waves_per_eu(StepLds<L, H>::min_waves(P, FORCED)))) void nlbm_step_kernel(
                                                        const float* __restrict__ Ain,
                                                        float* __restrict__ Aout,
                                                        const float* __restrict__ theta, Grid G,
                                                        Force Fc, float rho0, float omega,
                                                        float knn, int nitems, int nxc) {
  using S = Shape<L::Q, H>;
  using LD = StepLds<L, H>;
  using F = typename Frag<P>::T;
  constexpr int Q = L::Q, WB = LD::waves_per_block(P, FORCED);
  __shared__ __attribute__((aligned(16))) float lds[WB * LD::per_wave];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, lg = lane >> 4, li = lane & 15;
  float* X = lds + wave * LD::per_wave;
  float* Y = X + LD::YO;  // output columns of the same rows

  const int nb = gridDim.x, bid = blockIdx.x;
  const int lb = (nb % 8 == 0) ? (bid % 8) * (nb / 8) + bid / 8 : bid;
  // Items of this wavefront: it0, it0 + ST, ... below ib1.  D2Q9: a
  // contiguous range per wavefront.  D3Q19: the workgroup's range with its
  // wavefronts interleaved (wavefront w takes items ib0 + w, ib0 + w + WB,
  // ...), so that neighbouring items, which share the cache lines of the
  // x-shifted loads, are in flight on one compute unit at the same time; the
  // step then reads 1.01x its algorithmic bytes instead of 1.06x.  For D2Q9
  // the interleaving read more (1.04x against 1.03x) and ran 1% slower.
  constexpr int ST = L::Q == 19 ? WB : 1;
  int it0, ib1;
  if constexpr (ST > 1) {
    const int per = (nitems + nb - 1) / nb;
    const int ib0 = min(lb * per, nitems);
    ib1 = min(ib0 + per, nitems);
    it0 = ib0 + wave;
  } else {
    const int nw = nb * WB, per = (nitems + nw - 1) / nw;
    it0 = (lb * WB + wave) * per;
    ib1 = min(it0 + per, nitems);
  }

  const unsigned bytes = (unsigned)G.plane * (unsigned)(G.batch * Q) * 4u;
  const rsrc_t src = make_rsrc(Ain, bytes), dst = make_rsrc(Aout, bytes);
  // the first item's populations are loaded while the weights are staged
  ItemWalk cur, nxt;
  float gn[Q];
  if (it0 < ib1) {
    cur.start(it0, nxc, G);
    {
      const Item t0 = cur.item(G, lane);
      gather_rows<L>(src, ItemRows(G, Q, t0), t0, gn);
    }
  }

  // The weight fragments reach the registers through the (still unused)
  // tile memory: the workgroup stages them from coalesced reads of theta,
  // then every wave loads its copy with lane-contiguous reads.
  Weights<P, S> W;
  W.load_biases(theta);
  {
    using F = typename Frag<P>::T;
    constexpr int NF = S::HB * S::KX + S::HB * S::HB + S::QB * S::HB;
    static_assert(NF * 64 * (int)sizeof(F) <= WB * LD::per_wave * 4, "fragment staging");
    F* fr = reinterpret_cast<F*>(lds);
    stage_weight_fragments<P, S, 64 * WB>(fr, theta);
    W.load_staged(fr);
    __syncthreads();
  }
  if (it0 >= ib1) return;
  // the 16-bit instances hold the layer-3 bias in registers, in the MFMA
  // result layout (rows 16 ob + 4 lg + r); the float32 ones, which have no
  // registers to spare, read it from the tile's padding columns per group
  constexpr bool B3R = P != P_F32;
  f4 b3r[B3R ? S::QB : 1];
  if constexpr (B3R) {
#pragma unroll
    for (int ob = 0; ob < S::QB; ++ob)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = 16 * ob + 4 * lg + r;
        b3r[ob][r] = q < Q ? theta[S::ob3 + q] : 0.f;
      }
  }

  // the input columns past the populations never change: a constant 1 for
  // the bias of layer 1, then zeros
#pragma unroll
  for (int k = Q; k < LD::YO; ++k) X[lane * LD::SX + k] = k == Q ? 1.f : 0.f;
  if (lane < 4 * S::QB) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int q = 4 * lane + r;
      X[lane * LD::SX + LD::B3 + r] = q < Q ? theta[S::ob3 + q] : 0.f;
    }
  }

  // the biases and the first item's populations have arrived: no wait in the
  // loop has to cover loads issued before it
  wait_vmem();
  for (int it = it0; it < ib1; it += ST) {
    // this item's populations go to the LDS tile; the next item's loads are
    // issued before the network runs
#pragma unroll
    for (int q = 0; q < Q; ++q) X[lane * LD::SX + q] = gn[q];
    if (it + ST < ib1) {
      nxt = cur;
      if constexpr (ST > 1) {
        nxt.advance(ST, nxc, G);
      } else {
        nxt.next(nxc, G);
      }
      const Item tn = nxt.item(G, lane);
      gather_rows<L>(src, ItemRows(G, Q, tn), tn, gn);
    }
    // the body force is read here, so that it arrives while the network runs
    float F3[3] = {0.f, 0.f, 0.f};
    if constexpr (FORCED) {
      const Item tc = cur.item(G, lane);
      body_force(Fc, G, tc.x, tc.y, tc.z, F3);
    }
    wave_lds_sync();
#pragma unroll
    for (int jg = 0; jg < 4; ++jg) {
      const int nrow = 16 * jg + li;
      F xin[S::KX];
#pragma unroll
      for (int c = 0; c < S::KX; ++c) {
        const int col = 16 * c + 4 * lg;
        f4 v;
        if constexpr (LD::ZERO_PAD) {
          v = *reinterpret_cast<const f4*>(X + nrow * LD::SX + col);
        } else {
          v = *reinterpret_cast<const f4*>(X + nrow * LD::SX + (col < LD::YC ? col : 0));
          if (col >= LD::YC) v = f4{0.f, 0.f, 0.f, 0.f};
        }
        xin[c] = to_frag<P>(v);
      }
      F h1[S::HB], h2[S::HB];
#pragma unroll
      for (int ob = 0; ob < S::HB; ++ob)
        h1[ob] = to_frag<P>(tanh4<P>(mma_row<P, S::KX>(f4{0.f, 0.f, 0.f, 0.f}, W.w1[ob], xin)));
#pragma unroll
      for (int ob = 0; ob < S::HB; ++ob)
        h2[ob] = to_frag<P>(tanh4<P>(mma_row<P, S::HB>(W.b2[ob], W.w2[ob], h1)));
#pragma unroll
      for (int ob = 0; ob < S::QB; ++ob) {
        const f4 b3 = B3R ? b3r[B3R ? ob : 0]
                          : *reinterpret_cast<const f4*>(X + (4 * ob + lg) * LD::SX + LD::B3);
        const f4 y = mma_row<P, S::HB>(b3, W.w3[ob], h2);
        if (16 * ob + 4 * lg < LD::YQ)
          *reinterpret_cast<f4*>(Y + nrow * LD::SX + 16 * ob + 4 * lg) = y;
      }
    }
    wave_lds_sync();

    // node layout: BGK, network term, projection, force, store
    const Item t = cur.item(G, lane);
    float g[Q], upd[Q], rho, u[3];
#pragma unroll
    for (int q = 0; q < Q; ++q) g[q] = X[lane * LD::SX + q];
    bgk_update<L>(g, rho0, omega, upd, rho, u);
#pragma unroll
    for (int q = 0; q < Q; ++q) upd[q] = __builtin_fmaf(knn, Y[lane * LD::SX + q], upd[q]);
    float post[Q];
    finish_collision<L>(g, upd, rho, u, F3, FORCED, post);
    // the next item's populations arrived while the network ran
    wait_vmem();
    if (t.active) store_rows<L, kStoreNT>(dst, ItemRows(G, Q, t), t, post);
    wave_lds_sync();
    cur = nxt;
  }
}

// Workgroups for a persistent kernel: as many as fit on the chip at once
// (occ per compute unit), no more than there are work units, a multiple of
// the 8 XCDs when large.
inline unsigned persistent_grid(int ncu, int occ, long long units_per_block_min,
                                long long units) {
  if (occ < 1) occ = 1;
  long long want = (long long)ncu * occ;
  long long cap = (units + units_per_block_min - 1) / units_per_block_min;
  long long nb = want < cap ? want : cap;
  if (nb >= 16) nb -= nb % 8;
  if (nb < 1) nb = 1;
  return (unsigned)nb;
}

// Launch of the learned-collision step for (lattice, H, precision, forcing),
// defined in nlbm_fwd.hip: a persistent grid over the nitems 64-node items.
hipError_t nlbm_fwd_launch(bool d3q19, int hidden, int prec, bool forced, int ncu, hipStream_t s,
                           const float* Ain, float* Aout, const float* theta, Grid G, Force Fc,
                           float rho0, float omega, float knn, int nitems, int nxc);

}  // namespace lbm
