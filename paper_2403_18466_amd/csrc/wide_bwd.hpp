// wide_bwd.hpp -- adjoint of one step with the SI's network (Q -> 300 -> 300
// -> 100 -> Q, LeakyReLU), for unrolled training (SI, "Unrolled training").
//
// The step's adjoint needs, per node, every hidden activation (for the
// LeakyReLU derivative and the weight gradients) and the weight gradients
// are contractions over all nodes.  Training runs on coarse grids (32^3 -
// 64^3), so the adjoint is organised as dense products over the node
// dimension with the activations kept in a caller workspace:
//
//   prep      X0 = [g, 1, 0...]                       (node kernel, gather)
//   forward   H1 = leaky(X0 W1^T), H2 = leaky(H1 W2^T + b2), H3 = leaky(H2 W3^T + b3)
//   dY        dY = (s_out / tau) P mu                 (node kernel; mu = lam^{n+1}(x))
//   backward  dZ3 = (dY W4) . leaky'(H3), dZ2 = (dZ3 W3) . leaky'(H2),
//             dZ1 = (dZ2 W2) . leaky'(H1), dX0 = dZ1 W1
//   weights   dW4 = dY^T H3, dW3 = dZ3^T H2, dW2 = dZ2^T H1, dW1 = dZ1^T X0
//             (split over node chunks, summed in a fixed order)
//   post      lam^n_q(x - c_q) = (BGK, projection, force adjoint)_q + dX0_q
//
// Every product is C[i][j] = sum_k A[i][k] B[j][k] ("NT", both operands
// contiguous in k) on the matrix cores.  The forward epilogues write each
// activation matrix node-major (the next product's A operand) and
// feature-major (the weight-gradient operand).  Widths are padded to whole
// 16-row tiles (300 -> 304, 100 -> 112, Q -> 32); one padded column of each
// activation holds the constant 1 (X0 column Q, H1 and H2 column 300, H3
// column 100), so the weight-gradient products also produce the bias
// gradients.  The matching padded weight columns are zero, so the constant
// never reaches the next layer.
//
// Reduced precision (as in the forward): X0, H1-H3, dY and dZ1-dZ3 and the
// weights are rounded to the operand format; accumulation and the biases
// b2, b3 are float32.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels_bwd.hpp"
#include "kernels_fwd.hpp"
#include "mlp.hpp"
#include "wide.hpp"

namespace lbm {

template <int Q_>
struct WideBwd {
  static constexpr int Q = Q_;
  static constexpr int D0 = 32, D1 = 304, D2 = 304, D3 = 112, D4 = 32;  // padded widths
  static constexpr int ONE1 = 300, ONE2 = 300, ONE3 = 100;               // constant-1 columns
  // padded weight matrices, row-major [out][in], then their transposes
  static constexpr int nW1 = D1 * D0, nW2 = D2 * D1, nW3 = D3 * D2, nW4 = D4 * D3;
  static constexpr int oW1 = 0, oW2 = oW1 + nW1, oW3 = oW2 + nW2, oW4 = oW3 + nW3;
  static constexpr int oT1 = oW4 + nW4, oT2 = oT1 + nW1, oT3 = oT2 + nW2, oT4 = oT3 + nW3;
  static constexpr int nw = oT4 + nW4;  // operand-type entries
  // float32 epilogue vectors: e1 (layer 1: only the constant column), b2p, b3p
  static constexpr int fE1 = 0, fB2 = D1, fB3 = D1 + D2, nb = D1 + D2 + D3;
  // one split of the weight gradients: dW4p, dW3p, dW2p, dW1p (padded)
  static constexpr int gW4 = 0, gW3 = gW4 + nW4, gW2 = gW3 + nW3, gW1 = gW2 + nW2,
                       ngrad = gW1 + nW1;
  // the caller's packed parameter vector
  static constexpr int N1 = 300, N2 = 300, N3 = 100;
  static constexpr int pW1 = 0, pb1 = N1 * Q, pW2 = pb1 + N1, pb2 = pW2 + N2 * N1,
                       pW3 = pb2 + N2, pb3 = pW3 + N3 * N2, pW4 = pb3 + N3, pb4 = pW4 + Q * N3,
                       nparam = pb4 + Q;
};

// Operand storage type of a precision.
template <int P>
struct OpT;
template <>
struct OpT<P_F32> {
  using T = float;
};
template <>
struct OpT<P_BF16> {
  using T = __bf16;
};
template <>
struct OpT<P_F16> {
  using T = _Float16;
};

template <int P>
__device__ inline typename OpT<P>::T to_op(float v) {
  return (typename OpT<P>::T)v;
}

// packed[i] = theta[idx[i]], 0 where idx = -1, 1 where idx = -2; the first
// nw entries in the operand type, the nb after them in float32.
template <int P>
__global__ __launch_bounds__(256) void wide_bwd_pack_kernel(const float* __restrict__ theta,
                                                            const int* __restrict__ idx,
                                                            unsigned char* __restrict__ packed,
                                                            int nw, int nb) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nw + nb) return;
  const int j = idx[i];
  const float v = j >= 0 ? theta[j] : (j == -2 ? 1.f : 0.f);
  using T = typename OpT<P>::T;
  if (i < nw)
    reinterpret_cast<T*>(packed)[i] = to_op<P>(v);
  else
    reinterpret_cast<float*>(packed + (size_t)nw * sizeof(T))[i - nw] = v;
}

// X0 (node-major [Np][32]) and its transpose ([32][Np]) from the gathered
// pre-collision populations; rows past the last node are zero.
template <class L, int P>
__global__ __launch_bounds__(256) void wide_prep_kernel(const float* __restrict__ A, Grid G,
                                                        long long Np,
                                                        typename OpT<P>::T* __restrict__ X0,
                                                        typename OpT<P>::T* __restrict__ X0t) {
  const long long n = blockIdx.x * 256LL + threadIdx.x;
  if (n >= Np) return;
  const long long total = (long long)G.plane * G.batch;
  float g[L::Q];
  if (n < total) {
    int x, y, z, b;
    decode(G, n, x, y, z, b);
    gather<L>(A, G, b, x, y, z, g);
  }
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const float v = n < total ? (k < L::Q ? g[k] : (k == L::Q ? 1.f : 0.f)) : 0.f;
    X0[n * 32 + k] = to_op<P>(v);
    X0t[(long long)k * Np + n] = to_op<P>(v);
  }
}

// dY = (s_out / tau) P mu, mu = lam^{n+1}(x) (local read of the pull-shifted
// adjoint), node-major [Np][32] and transposed.
template <class L, int P>
__global__ __launch_bounds__(256) void wide_dy_kernel(const float* __restrict__ A,
                                                      const float* __restrict__ lam1, Grid G,
                                                      Force Fc, float rho0, float omega, float knn,
                                                      long long Np,
                                                      typename OpT<P>::T* __restrict__ dY,
                                                      typename OpT<P>::T* __restrict__ dYt) {
  const long long n = blockIdx.x * 256LL + threadIdx.x;
  if (n >= Np) return;
  const long long total = (long long)G.plane * G.batch;
  float nu[L::Q];
  if (n < total) {
    int x, y, z, b;
    decode(G, n, x, y, z, b);
    float g[L::Q], mu[L::Q], lam[L::Q], F[3];
    gather<L>(A, G, b, x, y, z, g);
#pragma unroll
    for (int q = 0; q < L::Q; ++q) mu[q] = lam1[cell(G, b, q, L::Q, x, y, z)];
    body_force(Fc, G, x, y, z, F);
    collide_adjoint<L>(g, mu, rho0, omega, F, Fc.kind != 0, nu, lam);
  }
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const float v = (n < total && k < L::Q) ? knn * nu[k] : 0.f;
    dY[n * 32 + k] = to_op<P>(v);
    dYt[(long long)k * Np + n] = to_op<P>(v);
  }
}

// lam^n_q(x - c_q) = l_q(x) + dX0[x][q]: the non-network adjoint plus the
// network's input gradient, scattered to the pull positions.
template <class L>
__global__ __launch_bounds__(256) void wide_post_kernel(const float* __restrict__ A,
                                                        const float* __restrict__ lam1,
                                                        const float* __restrict__ dX0,
                                                        float* __restrict__ lam0, Grid G, Force Fc,
                                                        float rho0, float omega) {
  const long long n = blockIdx.x * 256LL + threadIdx.x;
  const long long total = (long long)G.plane * G.batch;
  if (n >= total) return;
  int x, y, z, b;
  decode(G, n, x, y, z, b);
  float g[L::Q], mu[L::Q], nu[L::Q], lam[L::Q], F[3];
  gather<L>(A, G, b, x, y, z, g);
#pragma unroll
  for (int q = 0; q < L::Q; ++q) mu[q] = lam1[cell(G, b, q, L::Q, x, y, z)];
  body_force(Fc, G, x, y, z, F);
  collide_adjoint<L>(g, mu, rho0, omega, F, Fc.kind != 0, nu, lam);
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    const int xd = wrap_sub(x, L::cx[q], G.nx), yd = wrap_sub(y, L::cy[q], G.ny),
              zd = wrap_sub(z, L::cz[q], G.nz);
    lam0[cell(G, b, q, L::Q, xd, yd, zd)] = lam[q] + dX0[n * 32 + q];
  }
}

// ---------------------------------------------------------------------------
// C[i][j] = sum_k A[i][k] B[j][k] on the matrix cores: 64 x 64 tiles, four
// wavefronts of 32 x 32, K steps of 32 staged in LDS; rows / columns past M /
// N and k past K read as zero.  blockIdx.z selects a K range [z kc, z kc +
// kc) (split over nodes for the weight gradients).
// ---------------------------------------------------------------------------
enum GemmEpi {
  EPI_LEAKY = 0,    // C, Ct = leaky(acc + bias[j]) in the operand type
  EPI_MASK = 1,     // C, Ct = acc * leaky'(mask[i][j]) in the operand type
  EPI_F32 = 2,      // Cf = acc (float32)
  EPI_PARTIAL = 3,  // Cf[z][i][j] = acc (float32), one slab per K range
};

struct GemmArgs {
  const void* A;
  const void* B;
  long long lda, ldb;
  int M, N;
  long long K, kc;
  void* C;
  void* Ct;
  long long ldc, ldct;
  const float* bias;
  const void* mask;
  long long slab;  // EPI_PARTIAL: elements between consecutive K-range slabs
};

// Epilogue of a wavefront's 32 x 32 block at (ib, jb); D layout: lane
// (lg, li) holds rows 4 lg + r, column li of each 16 x 16 tile.
template <int P, int EPI>
__device__ inline void gemm_epilogue(const GemmArgs& a, const f4 (&acc)[2][2], int ib, int jb,
                                     int lg, int li) {
  using T = typename OpT<P>::T;
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int j = jb + 16 * t + li;
      if (j >= a.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = ib + 16 * s + 4 * lg + r;
        if (i >= a.M) continue;
        float v = acc[s][t][r];
        if constexpr (EPI == EPI_LEAKY) {
          v += a.bias[j];
          v = v > 0.f ? v : kLeakySlope * v;
        } else if constexpr (EPI == EPI_MASK) {
          const float m = (float)static_cast<const T*>(a.mask)[(long long)i * a.ldc + j];
          v = m > 0.f ? v : kLeakySlope * v;
        }
        if constexpr (EPI == EPI_LEAKY || EPI == EPI_MASK) {
          static_cast<T*>(a.C)[(long long)i * a.ldc + j] = to_op<P>(v);
          if (a.Ct) static_cast<T*>(a.Ct)[(long long)j * a.ldct + i] = to_op<P>(v);
        } else if constexpr (EPI == EPI_F32) {
          static_cast<float*>(a.C)[(long long)i * a.ldc + j] = v;
        } else {
          static_cast<float*>(a.C)[(long long)blockIdx.z * a.slab + (long long)i * a.ldc + j] = v;
        }
      }
    }
}

template <int P, int EPI>
__global__ __launch_bounds__(256) void gemm_nt_kernel(GemmArgs a) {
  using T = typename OpT<P>::T;
  using F = typename Frag<P>::T;
  constexpr int SK = 32 + 8;  // LDS row stride (elements)
  __shared__ __attribute__((aligned(16))) T As[64 * SK];
  __shared__ __attribute__((aligned(16))) T Bs[64 * SK];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, lg = lane >> 4, li = lane & 15;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const long long k_begin = (long long)blockIdx.z * a.kc;
  long long k_end = k_begin + a.kc;
  if (k_end > a.K) k_end = a.K;
  const T* A = static_cast<const T*>(a.A);
  const T* B = static_cast<const T*>(a.B);
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  f4 acc[2][2];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int t = 0; t < 2; ++t) acc[s][t] = f4{0.f, 0.f, 0.f, 0.f};
  // staging: thread -> (row tid / 4, k (tid % 4) * 8 .. + 7)
  const int sr = tid >> 2, sk = (tid & 3) * 8;
  for (long long k0 = k_begin; k0 < k_end; k0 += 32) {
    {
      const int ra = i0 + sr, rb = j0 + sr;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const long long k = k0 + sk + e;
        As[sr * SK + sk + e] = (ra < a.M && k < k_end) ? A[(long long)ra * a.lda + k] : T(0.f);
        Bs[sr * SK + sk + e] = (rb < a.N && k < k_end) ? B[(long long)rb * a.ldb + k] : T(0.f);
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      F af[2], bf[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        f4 va, vb;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          va[r] = (float)As[(wi + 16 * s + li) * SK + 16 * c + 4 * lg + r];
          vb[r] = (float)Bs[(wj + 16 * s + li) * SK + 16 * c + 4 * lg + r];
        }
        af[s] = to_frag<P>(va);
        bf[s] = to_frag<P>(vb);
      }
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[s][t] = mma_chunk<P>(acc[s][t], af[s], bf[t]);
    }
    __syncthreads();
  }
  gemm_epilogue<P, EPI>(a, acc, i0 + wi, j0 + wj, lg, li);
}

// The same product for 16-bit operands, 64 x 64 tiles of four wavefronts
// (32 x 32 each, 2 x 2 MFMA tiles), K steps of 32:
//  * every thread loads 8 consecutive k of one row of A and of B per step
//    (16-byte loads; M, N and K are multiples of 8 here, so a chunk is
//    either wholly inside or wholly outside the operand);
//  * the next step's chunks are in registers while the current step's
//    MFMAs run, then go to the other of two LDS buffers (one barrier per
//    step);
//  * a lane's operand of one 16 x 16 x 32 MFMA is one 16-byte LDS read: row
//    li of the tile, k = 8 lg .. 8 lg + 7, for A and for B alike, so the
//    contraction pairs the same k on both sides.
template <int P, int EPI>
__global__ __launch_bounds__(256) void gemm_nt16_kernel(GemmArgs a) {
  static_assert(P != P_F32, "16-bit operands");
  using T = typename OpT<P>::T;
  constexpr int SK = 32 + 8;  // LDS row stride (elements): 80 bytes
  __shared__ __attribute__((aligned(16))) T As[2][64 * SK];
  __shared__ __attribute__((aligned(16))) T Bs[2][64 * SK];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, lg = lane >> 4, li = lane & 15;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const long long k_begin = (long long)blockIdx.z * a.kc;
  long long k_end = k_begin + a.kc;
  if (k_end > a.K) k_end = a.K;
  const T* A = static_cast<const T*>(a.A);
  const T* B = static_cast<const T*>(a.B);
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  // staging: thread -> row tid / 4 of each tile, k (tid % 4) * 8 .. + 7
  const int sr = tid >> 2, sk = (tid & 3) * 8;
  const bool rowA = i0 + sr < a.M, rowB = j0 + sr < a.N;
  const T* pa = A + (long long)(rowA ? i0 + sr : 0) * a.lda + sk;
  const T* pb = B + (long long)(rowB ? j0 + sr : 0) * a.ldb + sk;
  auto fetch = [&](long long k0, u4& va, u4& vb) {
    const bool in = k0 + sk < k_end;
    va = (rowA && in) ? *reinterpret_cast<const u4*>(pa + k0) : u4{0u, 0u, 0u, 0u};
    vb = (rowB && in) ? *reinterpret_cast<const u4*>(pb + k0) : u4{0u, 0u, 0u, 0u};
  };
  f4 acc[2][2];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int t = 0; t < 2; ++t) acc[s][t] = f4{0.f, 0.f, 0.f, 0.f};
  u4 va, vb;
  fetch(k_begin, va, vb);
  *reinterpret_cast<u4*>(&As[0][sr * SK + sk]) = va;
  *reinterpret_cast<u4*>(&Bs[0][sr * SK + sk]) = vb;
  __syncthreads();
  int buf = 0;
  for (long long k0 = k_begin; k0 < k_end; k0 += 32) {
    const bool more = k0 + 32 < k_end;
    if (more) fetch(k0 + 32, va, vb);
    u4 af[2], bf[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      af[s] = *reinterpret_cast<const u4*>(&As[buf][(wi + 16 * s + li) * SK + 8 * lg]);
      bf[s] = *reinterpret_cast<const u4*>(&Bs[buf][(wj + 16 * s + li) * SK + 8 * lg]);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        if constexpr (P == P_BF16)
          acc[s][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              __builtin_bit_cast(b8, af[s]), __builtin_bit_cast(b8, bf[t]), acc[s][t], 0, 0, 0);
        else
          acc[s][t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
              __builtin_bit_cast(h8, af[s]), __builtin_bit_cast(h8, bf[t]), acc[s][t], 0, 0, 0);
      }
    if (more) {
      *reinterpret_cast<u4*>(&As[buf ^ 1][sr * SK + sk]) = va;
      *reinterpret_cast<u4*>(&Bs[buf ^ 1][sr * SK + sk]) = vb;
    }
    __syncthreads();
    buf ^= 1;
  }
  if constexpr (EPI == EPI_LEAKY || EPI == EPI_MASK) {
    // The activations of the 64 x 64 tile go through LDS (the A buffers are
    // free after the last barrier), so that both C and its transpose Ct are
    // written as 16-byte row chunks.
    constexpr int SO = 64 + 8;  // row stride of the output tile (elements)
    static_assert(64 * SO <= 2 * 64 * SK, "output tile fits in the A buffers");
    T* Ts = &As[0][0];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int jl = wj + 16 * t + li, j = j0 + jl;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int il = wi + 16 * s + 4 * lg + r, i = i0 + il;
          float v = acc[s][t][r];
          if constexpr (EPI == EPI_LEAKY) {
            v += j < a.N ? a.bias[j] : 0.f;
            v = v > 0.f ? v : kLeakySlope * v;
          } else {
            const float m = (i < a.M && j < a.N)
                                ? (float)static_cast<const T*>(a.mask)[(long long)i * a.ldc + j]
                                : 0.f;
            v = m > 0.f ? v : kLeakySlope * v;
          }
          Ts[il * SO + jl] = to_op<P>(v);
        }
      }
    __syncthreads();
    T* C = static_cast<T*>(a.C);
    T* Ct = static_cast<T*>(a.Ct);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = tid + 256 * h, row = c >> 3, ch = (c & 7) * 8;
      // C: row i0 + row, columns j0 + ch .. + 7
      if (i0 + row < a.M && j0 + ch < a.N)
        *reinterpret_cast<u4*>(C + (long long)(i0 + row) * a.ldc + j0 + ch) =
            *reinterpret_cast<const u4*>(Ts + row * SO + ch);
      // Ct: row j0 + row of the transpose, columns i0 + ch .. + 7
      if (Ct && j0 + row < a.N && i0 + ch < a.M) {
        T v8[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v8[e] = Ts[(ch + e) * SO + row];
        *reinterpret_cast<u4*>(Ct + (long long)(j0 + row) * a.ldct + i0 + ch) =
            __builtin_bit_cast(u4, v8);
      }
    }
  } else {
    gemm_epilogue<P, EPI>(a, acc, i0 + wi, j0 + wj, lg, li);
  }
}

// dtheta[p] += sum over the nsplit slabs (fixed order) of the padded weight
// gradient entry that parameter p maps to.
template <int Q>
__global__ __launch_bounds__(256) void wide_grad_reduce_kernel(const float* __restrict__ part,
                                                               int nsplit,
                                                               float* __restrict__ dtheta) {
  using W = WideBwd<Q>;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= W::nparam) return;
  int e;
  if (p < W::pb1) {
    e = W::gW1 + (p / Q) * W::D0 + p % Q;
  } else if (p < W::pW2) {
    e = W::gW1 + (p - W::pb1) * W::D0 + Q;  // the constant input column
  } else if (p < W::pb2) {
    const int r = p - W::pW2;
    e = W::gW2 + (r / W::N1) * W::D1 + r % W::N1;
  } else if (p < W::pW3) {
    e = W::gW2 + (p - W::pb2) * W::D1 + W::ONE1;
  } else if (p < W::pb3) {
    const int r = p - W::pW3;
    e = W::gW3 + (r / W::N2) * W::D2 + r % W::N2;
  } else if (p < W::pW4) {
    e = W::gW3 + (p - W::pb3) * W::D2 + W::ONE2;
  } else if (p < W::pb4) {
    const int r = p - W::pW4;
    e = W::gW4 + (r / W::N3) * W::D3 + r % W::N3;
  } else {
    e = W::gW4 + (p - W::pb4) * W::D3 + W::ONE3;
  }
  float s = 0.f;
  for (int k = 0; k < nsplit; ++k) s += part[(long long)k * W::ngrad + e];
  dtheta[p] += s;
}

// Launch of the whole adjoint (defined in wide_bwd.hip).  ws: device
// workspace of wide_bwd_workspace_bytes(); packed: the fragment buffer the
// context owns, filled from theta by the call.
size_t wide_bwd_workspace_bytes(bool d3q19, int prec, long long nodes);
hipError_t wide_bwd_launch(bool d3q19, int prec, hipStream_t s, const float* A,
                           const float* theta, const float* lam1, float* lam0, float* dtheta,
                           void* ws, const int* idx, unsigned char* packed, Grid G, Force Fc,
                           float rho0, float omega, float knn);

}  // namespace lbm
