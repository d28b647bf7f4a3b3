// kernels_bwd.hpp -- adjoint (reverse-mode derivative) of one stream-collide
// step, used to backpropagate a loss through unrolled time steps (SI,
// "Unrolled training").
//
// One step maps the pull-shifted state A^n to A^{n+1}(x) = C(g(x)) with
// g_q(x) = A^n_q(x - c_q) and C the node-local collision.  For
// lam^{n+1} = dL/dA^{n+1} the adjoint is
//   mu(x)  = lam^{n+1}(x)                    (local read),
//   l(x)   = J_C(g(x))^T mu(x),              (node-local reverse pass)
//   lam^n_q(x - c_q) = l_q(x)                (scatter: the transpose of the
//                                             gather, a permutation),
//   dtheta += sum_x (dC/dtheta)^T mu(x).
// The reverse pass through C goes, in reverse order, through
//   post = g + P(Omega + k y) + f^ext,   Omega = (f^eq(rho, j) - g)/tau,
//   y = W3 h2 + b3, h2 = tanh(W2 h1 + b2), h1 = tanh(W1 g + b1),
// with P the symmetric projector of the kappa layer, k = s_out/tau, and
// tanh' = 1 - tanh^2.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels_fwd.hpp"

namespace lbm {

// Reverse pass through everything except the network.  Given g and
// mu = dL/dpost, returns nu = P mu and l = dL/dg without the network's
// input gradient.
template <class L>
__device__ inline void collide_adjoint(const float g[L::Q], const float mu[L::Q], float rho0,
                                       float omega, const float F[3], bool forced,
                                       float nu[L::Q], float lam[L::Q]) {
  constexpr int Q = L::Q;
  float drho, j[3];
  moments<L>(g, drho, j);
  const float rho = rho0 + drho, inv = __builtin_amdgcn_rcpf(rho);
  const float u[3] = {j[0] * inv, j[1] * inv, j[2] * inv};
  const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
  for (int q = 0; q < Q; ++q) nu[q] = mu[q];
  project<L>(nu);
  // d f^eq_q / d drho = w_q (1 - 9/2 (c.u)^2 + 3/2 |u|^2)
  // d f^eq_q / d j_a  = w_q (3 c_a + 9 (c.u) c_a - 3 u_a)
  float Gr = 0.f, Gj[3] = {0.f, 0.f, 0.f};
  auto accum = [&](int q, float cu, float a) {
    float wa = L::w[q] * a;
    Gr += wa * (1.f - 4.5f * cu * cu + 1.5f * uu);
    float s = wa * (3.f + 9.f * cu);
    Gj[0] += (L::cx[q] > 0 ? s : (L::cx[q] < 0 ? -s : 0.f)) - 3.f * wa * u[0];
    Gj[1] += (L::cy[q] > 0 ? s : (L::cy[q] < 0 ? -s : 0.f)) - 3.f * wa * u[1];
    Gj[2] += (L::cz[q] > 0 ? s : (L::cz[q] < 0 ? -s : 0.f)) - 3.f * wa * u[2];
  };
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    float cu = 0.f;
    if (L::cx[q] > 0) cu += u[0];
    if (L::cx[q] < 0) cu -= u[0];
    if (L::cy[q] > 0) cu += u[1];
    if (L::cy[q] < 0) cu -= u[1];
    if (L::cz[q] > 0) cu += u[2];
    if (L::cz[q] < 0) cu -= u[2];
    accum(q, cu, omega * nu[q]);
  }
  if (forced) {
    // f^ext_q = w_q rho [3 c.du + 9/2 c.du (2 c.u + c.du) - 3/2 du.(2u + du)],
    // du = F/rho:  d/d drho = -w_q [9/2 c.du (2 c.u + c.du) - 3/2 du.(2u+du)],
    //              d/d j_a  =  w_q (9 (c.du) c_a - 3 du_a).
    const float du[3] = {F[0] * inv, F[1] * inv, F[2] * inv};
    const float dd =
        du[0] * (2.f * u[0] + du[0]) + du[1] * (2.f * u[1] + du[1]) + du[2] * (2.f * u[2] + du[2]);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      float cu = 0.f, cd = 0.f;
      if (L::cx[q] > 0) { cu += u[0]; cd += du[0]; }
      if (L::cx[q] < 0) { cu -= u[0]; cd -= du[0]; }
      if (L::cy[q] > 0) { cu += u[1]; cd += du[1]; }
      if (L::cy[q] < 0) { cu -= u[1]; cd -= du[1]; }
      if (L::cz[q] > 0) { cu += u[2]; cd += du[2]; }
      if (L::cz[q] < 0) { cu -= u[2]; cd -= du[2]; }
      float wm = L::w[q] * mu[q];
      Gr -= wm * (4.5f * cd * (2.f * cu + cd) - 1.5f * dd);
      float s = 9.f * wm * cd;
      Gj[0] += (L::cx[q] > 0 ? s : (L::cx[q] < 0 ? -s : 0.f)) - 3.f * wm * du[0];
      Gj[1] += (L::cy[q] > 0 ? s : (L::cy[q] < 0 ? -s : 0.f)) - 3.f * wm * du[1];
      Gj[2] += (L::cz[q] > 0 ? s : (L::cz[q] < 0 ? -s : 0.f)) - 3.f * wm * du[2];
    }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    float d = Gr;
    if (L::cx[q] > 0) d += Gj[0];
    if (L::cx[q] < 0) d -= Gj[0];
    if (L::cy[q] > 0) d += Gj[1];
    if (L::cy[q] < 0) d -= Gj[1];
    if (L::cz[q] > 0) d += Gj[2];
    if (L::cz[q] < 0) d -= Gj[2];
    lam[q] = mu[q] - omega * nu[q] + d;
  }
}

// ---------------------------------------------------------------------------
// Adjoint of the BGK step (no network), one node per thread.
// ---------------------------------------------------------------------------
template <class L>
__global__ __launch_bounds__(256) void bgk_backward_kernel(const float* __restrict__ A,
                                                           const float* __restrict__ lam1,
                                                           float* __restrict__ lam0, Grid G,
                                                           Force Fc, float rho0, float omega,
                                                           int nxc) {
  const Item t = locate_item(blockIdx.x, nxc, G, threadIdx.x, 256);
  if (!t.active) return;
  const unsigned bytes = (unsigned)G.plane * (unsigned)(G.batch * L::Q) * 4u;
  float g[L::Q], mu[L::Q], nu[L::Q], lam[L::Q], F[3];
  gather_item<L>(make_rsrc(A, bytes), G, t, g);
  load_local<L>(make_rsrc(lam1, bytes), G, t, mu);
  body_force(Fc, G, t.x, t.y, t.z, F);
  collide_adjoint<L>(g, mu, rho0, omega, F, Fc.kind != 0, nu, lam);
  scatter_item<L>(make_rsrc(lam0, bytes), G, t, lam);
}

// ---------------------------------------------------------------------------
// Adjoint of the learned-collision step.
//
// Persistent wavefronts walk contiguous ranges of 64-node items as in the
// forward kernel.  Per item: node layout gathers g, reads mu, and runs the
// non-network part of the reverse pass; the network is recomputed and
// differentiated on the matrix cores per 16-node group:
//   forward   a1 = W1 x0 + b1, t1 = tanh a1;  a2 = W2 h1 + b2, t2 = tanh a2
//   backward  dy = k nu;  d2 = (W3^T dy) (1 - t2^2);  d1 = (W2^T d2) (1 - t1^2);
//             dx = W1^T d1
//   weights   dW3 += dy h2^T, dW2 += d2 h1^T, dW1|db1 += d1 [x0|1]^T (MFMA with
//             the node index as the contraction, operands transposed through
//             LDS), db2 += sum d2, db3 += sum dy (lane sums).
// Each wavefront writes its parameter-gradient partials (every entry, zeros
// if it had no work) to part[wave][param]; grad_reduce_kernel sums them in a
// fixed order.
// ---------------------------------------------------------------------------

// 16-node groups differentiated together (two wherever their transpose
// tiles fit in the LDS; the D3Q19 instances fall back to one)
#ifndef LBM_BWD_GROUPS
#define LBM_BWD_GROUPS 2
#endif

template <class L, int H, int P>
struct BwdLayout {
  using S = Shape<L::Q, H>;
  static constexpr int NF3 = S::HB * S::QB;   // W3^T fragments
  static constexpr int NF2 = S::HB * S::HB;   // W2^T fragments
  static constexpr int NF1 = S::KX * S::HB;   // W1^T fragments
  static constexpr int NF = NF3 + NF2 + NF1;
  static constexpr int SX = 16 * S::KX + 4;   // node-major tile stride (input / input grad)
  static constexpr int SD = 16 * (S::QB > S::KX ? S::QB : S::KX) + 4;
  static constexpr int ST = 20;               // feature-major transpose tile stride
  // two feature-major transpose tiles: h2 then d2 in the first, h1 then d1
  // in the second (a wave's LDS accesses complete in issue order, so a tile
  // can be rewritten once its previous contents have been read)
  // 16-node groups a wavefront differentiates at once (independent chains
  // the scheduler can interleave), each with its own transpose tiles
  static constexpr int wave_floats(int ngp) { return 64 * SX + 64 * SD + ngp * 2 * H * ST; }
  static constexpr int frag_bytes = (P == P_F32 ? 16 : 8) * 64;
  static constexpr bool fits(int ngp) {
    return 4 * 4 * wave_floats(ngp) + NF * frag_bytes <= 160 * 1024;
  }
  static constexpr int NGP = fits(LBM_BWD_GROUPS) ? LBM_BWD_GROUPS : 1;
  static constexpr int per_wave = wave_floats(NGP);
};

// Block-shared transposed weight fragments for the backward contractions,
// fragment-major (fragment f of lane l at w[64 f + l]): W3^T (HB x QB
// fragments), W2^T (HB x HB), W1^T (KX x HB).  W2 and W1 are the tanh
// layers: for bf16 / fp16 their fragments hold c W rounded, like the
// forward's, and the products are scaled back by 1/c.
template <class L, int H, int P>
__device__ inline void load_transposed_weights(typename Frag<P>::T* w,
                                               const float* __restrict__ theta) {
  using S = Shape<L::Q, H>;
  constexpr int Q = L::Q;
  constexpr int NF3 = S::HB * S::QB, NF2 = S::HB * S::HB, NF = NF3 + NF2 + S::KX * S::HB;
  constexpr float sc = tanh_weight_scale<P>();
  for (int e = threadIdx.x; e < NF * 64; e += blockDim.x) {
    const int f = e >> 6, l = e & 63, g = l >> 4, i = l & 15;
    f4 v;
    if (f < NF3) {  // W3^T: row h = 16 ob + i, k = q = 16 qc + 4 g + r
      const int ob = f / S::QB, qc = f % S::QB;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int q = 16 * qc + 4 * g + r, h = 16 * ob + i;
        v[r] = q < Q ? theta[S::oW3 + q * H + h] : 0.f;
      }
    } else if (f < NF3 + NF2) {  // W2^T: row h = 16 ob + i, k = o = 16 c + 4 g + r
      const int ff = f - NF3, ob = ff / S::HB, c = ff % S::HB;
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = sc * theta[S::oW2 + (16 * c + 4 * g + r) * H + 16 * ob + i];
    } else {  // W1^T: row k = 16 c + i (input index), k' = o = 16 ob + 4 g + r
      const int ff = f - NF3 - NF2, c = ff / S::HB, ob = ff % S::HB;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int k = 16 * c + i, o = 16 * ob + 4 * g + r;
        v[r] = k < Q ? sc * theta[S::oW1 + o * Q + k] : 0.f;
      }
    }
    w[e] = to_frag<P>(v);
  }
}

template <class L, int H, int P>
__global__ __launch_bounds__(256) void nlbm_backward_kernel(
    const float* __restrict__ A, const float* __restrict__ theta, const float* __restrict__ lam1,
    float* __restrict__ lam0, float* __restrict__ part, Grid G, Force Fc, float rho0,
    float omega, float knn, int nitems, int nxc, int accum) {
  using S = Shape<L::Q, H>;
  using BL = BwdLayout<L, H, P>;
  using Fr = typename Frag<P>::T;
  constexpr int Q = L::Q;
  __shared__ Fr wbk[BL::NF * 64];
  __shared__ float lds[4 * BL::per_wave];

  const int lane = threadIdx.x & 63, lg = lane >> 4, li = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  constexpr float sc = tanh_weight_scale<P>();
  load_transposed_weights<L, H, P>(wbk, theta);
  __syncthreads();

  float* X = lds + wave * BL::per_wave;  // [64][SX] network input x0
  float* D = X + 64 * BL::SX;            // [64][SD] dy, then overwritten by dx
  float* T = D + 64 * BL::SD;            // [H][ST] transpose scratch

  const int nb = gridDim.x, bid = blockIdx.x;
  const int lb = (nb % 8 == 0) ? (bid % 8) * (nb / 8) + bid / 8 : bid;
  const int nw = nb * 4, wv = lb * 4 + wave;
  const int per = (nitems + nw - 1) / nw;
  const int it0 = wv * per, it1 = min(it0 + per, nitems);

  Weights<P, S> W;
  W.load(theta);
  const Fr* W3T = wbk;
  const Fr* W2T = wbk + BL::NF3 * 64;
  const Fr* W1T = wbk + (BL::NF3 + BL::NF2) * 64;

  f4 dW1[S::HB][S::KX], dW2[S::HB][S::HB], dW3[S::QB][S::HB], db2[S::HB];
#pragma unroll
  for (int a = 0; a < S::HB; ++a) {
    db2[a] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < S::KX; ++c) dW1[a][c] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < S::HB; ++c) dW2[a][c] = f4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int a = 0; a < S::QB; ++a)
#pragma unroll
    for (int c = 0; c < S::HB; ++c) dW3[a][c] = f4{0.f, 0.f, 0.f, 0.f};
  float db3[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) db3[q] = 0.f;

  const unsigned bytes = (unsigned)G.plane * (unsigned)(G.batch * Q) * 4u;
  const rsrc_t rA = make_rsrc(A, bytes), rL1 = make_rsrc(lam1, bytes),
               rL0 = make_rsrc(lam0, bytes);
  auto load = [&](int it, float g[Q], float mu[Q]) {
    const Item t = locate_item(it, nxc, G, lane);
    if (t.active) {
      gather_item<L>(rA, G, t, g);
      load_local<L>(rL1, G, t, mu);
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q) g[q] = mu[q] = 0.f;
    }
  };

  float gc[Q], mc[Q];
  if (it0 < it1) load(it0, gc, mc);
  for (int it = it0; it < it1; ++it) {
    float gn[Q], mn[Q];
    if (it + 1 < it1) load(it + 1, gn, mn);
    const Item t = locate_item(it, nxc, G, lane);
    float F3[3] = {0.f, 0.f, 0.f};
    if (Fc.kind != 0) body_force(Fc, G, t.x, t.y, t.z, F3);
    float nu[Q], lam[Q];
    collide_adjoint<L>(gc, mc, rho0, omega, F3, Fc.kind != 0, nu, lam);

    // stage x0 and dy = k nu in node-major rows (zero padding)
#pragma unroll
    for (int c = 0; c < 4 * S::KX; ++c) {
      f4 v;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int k = 4 * c + r;
        v[r] = k < Q ? gc[k] : (k == Q ? 1.f : 0.f);
      }
      *reinterpret_cast<f4*>(X + lane * BL::SX + 4 * c) = v;
    }
#pragma unroll
    for (int c = 0; c < 4 * S::QB; ++c) {
      f4 v;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int q = 4 * c + r;
        float d = q < Q ? knn * nu[q] : 0.f;
        v[r] = d;
        if (q < Q) db3[q] += d;
      }
      *reinterpret_cast<f4*>(D + lane * BL::SD + 4 * c) = v;
    }
    wave_lds_sync();

    // NG consecutive 16-node groups at a time, stage by stage, so that the
    // scheduler has NG independent chains between the LDS ordering points;
    // the weight gradients contract over all 16 NG nodes at once.
    constexpr int NG = BL::NGP;
    auto groups = [&](const int jg0) {
      Fr xin[NG][S::KX], h1[NG][S::HB], h2[NG][S::HB], dyf[NG][S::QB], dyT[NG][S::QB];
      f4 t1[NG][S::HB], t2[NG][S::HB], d2[NG][S::HB], d1[NG][S::HB];
      Fr d2f[NG][S::HB], d1f[NG][S::HB];
      // forward recompute
#pragma unroll
      for (int e = 0; e < NG; ++e)
#pragma unroll
        for (int c = 0; c < S::KX; ++c)
          xin[e][c] = to_frag<P>(*reinterpret_cast<const f4*>(X + (16 * (jg0 + e) + li) * BL::SX + 16 * c + 4 * lg));
#pragma unroll
      for (int ob = 0; ob < S::HB; ++ob)
#pragma unroll
        for (int e = 0; e < NG; ++e) {
          t1[e][ob] = tanh4<P>(mma_row<P, S::KX>(f4{0.f, 0.f, 0.f, 0.f}, W.w1[ob], xin[e]));
          h1[e][ob] = to_frag<P>(t1[e][ob]);
        }
#pragma unroll
      for (int ob = 0; ob < S::HB; ++ob)
#pragma unroll
        for (int e = 0; e < NG; ++e) {
          t2[e][ob] = tanh4<P>(mma_row<P, S::HB>(W.b2[ob], W.w2[ob], h1[e]));
          h2[e][ob] = to_frag<P>(t2[e][ob]);
        }
      // dy in both operand layouts
#pragma unroll
      for (int e = 0; e < NG; ++e)
#pragma unroll
        for (int qc = 0; qc < S::QB; ++qc) {
          const int jg = jg0 + e;
          dyf[e][qc] = to_frag<P>(*reinterpret_cast<const f4*>(D + (16 * jg + li) * BL::SD + 16 * qc + 4 * lg));
          f4 v;
#pragma unroll
          for (int r = 0; r < 4; ++r) v[r] = D[(16 * jg + 4 * lg + r) * BL::SD + 16 * qc + li];
          dyT[e][qc] = to_frag<P>(v);
        }
      // d2 = (W3^T dy) (1 - t2^2)
#pragma unroll
      for (int ob = 0; ob < S::HB; ++ob)
#pragma unroll
        for (int e = 0; e < NG; ++e) {
          f4 a = mma_row_lds<P, S::QB>(f4{0.f, 0.f, 0.f, 0.f}, W3T + ob * S::QB * 64 + lane, dyf[e]);
          d2[e][ob] = a * (1.f - t2[e][ob] * t2[e][ob]);
          db2[ob] += d2[e][ob];
          d2f[e][ob] = to_frag<P>(d2[e][ob]);
        }
      // d1 = (W2^T d2) (1 - t1^2)
#pragma unroll
      for (int ob = 0; ob < S::HB; ++ob)
#pragma unroll
        for (int e = 0; e < NG; ++e) {
          f4 a = mma_row_lds<P, S::HB>(f4{0.f, 0.f, 0.f, 0.f}, W2T + ob * S::HB * 64 + lane, d2f[e]);
          if constexpr (sc != 1.f) a = a * (1.f / sc);
          d1[e][ob] = a * (1.f - t1[e][ob] * t1[e][ob]);
          d1f[e][ob] = to_frag<P>(d1[e][ob]);
        }
      // weight gradients, contraction over the 16 NG nodes of the groups;
      // group e's transpose tiles are T_e and T_e + H ST
      auto Te = [&](int e, int k) { return T + (2 * e + k) * H * BL::ST; };
      auto wgrad = [&](f4& acc, const Fr (&a)[NG], const Fr (&b)[NG]) {
        if constexpr (NG == 2)
          acc = mma_pair<P>(acc, a[0], a[1], b[0], b[1]);
        else
          acc = mma_chunk<P>(acc, a[0], b[0]);
      };
      {
        Fr h2T[S::HB][NG], dyTT[S::QB][NG];
#pragma unroll
        for (int e = 0; e < NG; ++e) {
#pragma unroll
          for (int blk = 0; blk < S::HB; ++blk)
#pragma unroll
            for (int r = 0; r < 4; ++r) Te(e, 0)[(16 * blk + 4 * lg + r) * BL::ST + li] = t2[e][blk][r];
        }
        wave_lds_sync();
#pragma unroll
        for (int e = 0; e < NG; ++e) {
#pragma unroll
          for (int blk = 0; blk < S::HB; ++blk)
            h2T[blk][e] = to_frag<P>(*reinterpret_cast<const f4*>(Te(e, 0) + (16 * blk + li) * BL::ST + 4 * lg));
#pragma unroll
          for (int qc = 0; qc < S::QB; ++qc) dyTT[qc][e] = dyT[e][qc];
        }
#pragma unroll
        for (int qc = 0; qc < S::QB; ++qc)
#pragma unroll
          for (int ib = 0; ib < S::HB; ++ib) wgrad(dW3[qc][ib], dyTT[qc], h2T[ib]);
      }
      {
        Fr h1T[S::HB][NG], d2T[S::HB][NG];
#pragma unroll
        for (int e = 0; e < NG; ++e)
#pragma unroll
          for (int blk = 0; blk < S::HB; ++blk)
#pragma unroll
            for (int r = 0; r < 4; ++r) Te(e, 1)[(16 * blk + 4 * lg + r) * BL::ST + li] = t1[e][blk][r];
        wave_lds_sync();
#pragma unroll
        for (int e = 0; e < NG; ++e)
#pragma unroll
          for (int blk = 0; blk < S::HB; ++blk)
            h1T[blk][e] = to_frag<P>(*reinterpret_cast<const f4*>(Te(e, 1) + (16 * blk + li) * BL::ST + 4 * lg));
        // the h2 tile has been read: reuse it for d2
        wave_lds_sync();
#pragma unroll
        for (int e = 0; e < NG; ++e)
#pragma unroll
          for (int blk = 0; blk < S::HB; ++blk)
#pragma unroll
            for (int r = 0; r < 4; ++r) Te(e, 0)[(16 * blk + 4 * lg + r) * BL::ST + li] = d2[e][blk][r];
        wave_lds_sync();
#pragma unroll
        for (int e = 0; e < NG; ++e)
#pragma unroll
          for (int blk = 0; blk < S::HB; ++blk)
            d2T[blk][e] = to_frag<P>(*reinterpret_cast<const f4*>(Te(e, 0) + (16 * blk + li) * BL::ST + 4 * lg));
#pragma unroll
        for (int ob = 0; ob < S::HB; ++ob)
#pragma unroll
          for (int ib = 0; ib < S::HB; ++ib) wgrad(dW2[ob][ib], d2T[ob], h1T[ib]);
      }
      {
        Fr d1T[S::HB][NG], x0T[S::KX][NG];
        wave_lds_sync();
#pragma unroll
        for (int e = 0; e < NG; ++e)
#pragma unroll
          for (int blk = 0; blk < S::HB; ++blk)
#pragma unroll
            for (int r = 0; r < 4; ++r) Te(e, 1)[(16 * blk + 4 * lg + r) * BL::ST + li] = d1[e][blk][r];
        wave_lds_sync();
#pragma unroll
        for (int e = 0; e < NG; ++e) {
#pragma unroll
          for (int blk = 0; blk < S::HB; ++blk)
            d1T[blk][e] = to_frag<P>(*reinterpret_cast<const f4*>(Te(e, 1) + (16 * blk + li) * BL::ST + 4 * lg));
#pragma unroll
          for (int c = 0; c < S::KX; ++c) {
            f4 v;
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = X[(16 * (jg0 + e) + 4 * lg + r) * BL::SX + 16 * c + li];
            x0T[c][e] = to_frag<P>(v);
          }
        }
#pragma unroll
        for (int ob = 0; ob < S::HB; ++ob)
#pragma unroll
          for (int c = 0; c < S::KX; ++c) wgrad(dW1[ob][c], d1T[ob], x0T[c]);
      }
      // dx = W1^T d1, over the input rows of these groups (overwrites the
      // groups' own dy rows, which are no longer read)
#pragma unroll
      for (int c = 0; c < S::KX; ++c)
#pragma unroll
        for (int e = 0; e < NG; ++e) {
          f4 a = mma_row_lds<P, S::HB>(f4{0.f, 0.f, 0.f, 0.f}, W1T + c * S::HB * 64 + lane, d1f[e]);
          if constexpr (sc != 1.f) a = a * (1.f / sc);
          *reinterpret_cast<f4*>(D + (16 * (jg0 + e) + li) * BL::SD + 16 * c + 4 * lg) = a;
        }
      // the transpose tiles are rewritten by the next groups
      wave_lds_sync();
    };
#pragma unroll 1
    for (int jp = 0; jp < 4; jp += NG) groups(jp);
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < Q; ++q) lam[q] += D[lane * BL::SD + q];
    if (t.active) scatter_item<L>(rL0, G, t, lam);
    wave_lds_sync();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      gc[q] = gn[q];
      mc[q] = mn[q];
    }
  }

  // Parameter-gradient partials: every wave writes its full vector to its
  // own LDS row (the tiles are free once every wave has left the item loop),
  // then the block sums the four rows in wave order and writes one partial
  // vector part[block][param].
  __syncthreads();
  static_assert(4 * S::n <= 4 * BL::per_wave, "reduction buffer");
  {
    float* red = lds + wave * S::n;
#pragma unroll
    for (int ob = 0; ob < S::HB; ++ob) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = 16 * ob + 4 * lg + r;
#pragma unroll
        for (int c = 0; c < S::KX; ++c) {
          const int k = 16 * c + li;
          if (k < Q) red[S::oW1 + o * Q + k] = dW1[ob][c][r];
          else if (k == Q) red[S::ob1 + o] = dW1[ob][c][r];
        }
#pragma unroll
        for (int c = 0; c < S::HB; ++c) red[S::oW2 + o * H + 16 * c + li] = dW2[ob][c][r];
        float sb = db2[ob][r];
        sb += __shfl_xor(sb, 8);
        sb += __shfl_xor(sb, 4);
        sb += __shfl_xor(sb, 2);
        sb += __shfl_xor(sb, 1);
        if (li == 0) red[S::ob2 + o] = sb;
      }
    }
#pragma unroll
    for (int qc = 0; qc < S::QB; ++qc)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = 16 * qc + 4 * lg + r;
#pragma unroll
        for (int c = 0; c < S::HB; ++c)
          if (q < Q) red[S::oW3 + q * H + 16 * c + li] = dW3[qc][c][r];
      }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      float sq = db3[q];
      sq += __shfl_xor(sq, 32);
      sq += __shfl_xor(sq, 16);
      sq += __shfl_xor(sq, 8);
      sq += __shfl_xor(sq, 4);
      sq += __shfl_xor(sq, 2);
      sq += __shfl_xor(sq, 1);
      if (lane == 0) red[S::ob3 + q] = sq;
    }
  }
  __syncthreads();
  float* pb = part + (size_t)blockIdx.x * S::n;
  for (int i = threadIdx.x; i < S::n; i += 256) {
    const float v = ((lds[i] + lds[S::n + i]) + lds[2 * S::n + i]) + lds[3 * S::n + i];
    pb[i] = accum ? pb[i] + v : v;
  }
}

// ---------------------------------------------------------------------------
// Cooperative adjoint of the learned-collision step (16-bit D2Q9 networks).
//
// The kernel above keeps all parameter-gradient accumulators of the network
// and the forward weights in every wavefront (about 150 registers at
// H = 64) and fits one wavefront per SIMD.  Here the eight wavefronts of a
// workgroup (two per SIMD) take one 16-node group each per step and split
// the 16 x 16 weight-gradient tiles between them.  After the forward
// recompute and the backward data path of its group, a wavefront writes the
// group's gradient operands (16-bit, as the products leave them) to its LDS
// slot; after a workgroup barrier each wavefront reads them back in
// contraction layout (the node index as K) and accumulates its own TPW
// tiles over the 128 nodes of the eight slots.  The network weights are
// staged in LDS once per workgroup and read from there into registers.  The
// contraction order is fixed, so the result is reproducible.
//
// Slot fragment layout: fragment f is 512 bytes of 64 rows of 8 bytes; lane
// l writes its four 16-bit values of the D-layout tile (features 4 (l / 16)
// + r of node l % 16) to row slot_row(l) = l ^ 4 (l / 16) with one 8-byte
// store.  The contraction reads it back transposed with ds_read_b64_tr_b16:
// within each block of 16 lanes, lane 4 a + e of the reading wavefront
// receives element e of the rows that lanes a, a + 4, a + 8 and a + 12 of
// its block address.  A reading lane L = 16 b + m (a = m % 4, k = m / 4)
// addresses the row of writer lane 16 a + 4 b + k, and so receives
// features 4 a + e of node 4 b + k: operand lane L then holds feature L % 16
// of nodes 4 (L / 16) + r, the layout the products over the nodes take.
// The XOR puts the 16 rows that one 16-lane block reads, and those that 16
// consecutive lanes write, on 16 different bank pairs.
__device__ __host__ constexpr int slot_row(int l) { return l ^ (4 * (l >> 4)); }
__device__ __host__ constexpr int tr_row(int L) {
  return slot_row(16 * ((L & 15) & 3) + 4 * (L >> 4) + ((L & 15) >> 2));
}
// The identity above, checked at compile time: with the transposing read's
// lane rule for 16-bit elements (within a 16-lane block, lane 4 a + e takes
// element e of the rows that lanes a + 4 j, j = 0..3, address), lane L's
// value j is element e of the row written by the lane w with slot_row(w) =
// tr_row(16 (L / 16) + a + 4 j), i.e. feature 4 (w / 16) + e of node w % 16;
// it must be feature L % 16 of node 4 (L / 16) + j.
__device__ __host__ constexpr bool slot_layout_ok() {
  for (int L = 0; L < 64; ++L) {
    const int blk = L >> 4, m = L & 15, a = m >> 2, e = m & 3;
    for (int j = 0; j < 4; ++j) {
      const int row = tr_row(16 * blk + a + 4 * j);
      int w = -1;
      for (int l = 0; l < 64; ++l)
        if (slot_row(l) == row) w = l;
      if (w < 0 || 4 * (w >> 4) + e != m || (w & 15) != 4 * blk + j) return false;
    }
  }
  return true;
}
static_assert(slot_layout_ok(), "slot rows and transposing reads");
// and the swizzle's purpose: an 8-byte row sits on bank pair row % 16, so
// the 16 rows that a 16-lane block reads, and those that 16 consecutive
// lanes write, must fall on 16 different pairs
__device__ __host__ constexpr bool slot_banks_ok() {
  for (int blk = 0; blk < 4; ++blk) {
    int rd = 0, wr = 0;
    for (int i = 0; i < 16; ++i) {
      rd |= 1 << (tr_row(16 * blk + i) & 15);
      wr |= 1 << (slot_row(16 * blk + i) & 15);
    }
    if (rd != 0xffff || wr != 0xffff) return false;
  }
  return true;
}
static_assert(slot_banks_ok(), "slot rows on distinct bank pairs");

template <int P>
__device__ inline typename Frag<P>::T read_tr(const unsigned char* p) {
  typedef short v4s __attribute__((ext_vector_type(4)));
  const v4s v = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
      (__attribute__((address_space(3))) v4s*)(p));
  return __builtin_bit_cast(typename Frag<P>::T, v);
}
template <class L, int H, int P>
struct CoopLayout {
  using S = Shape<L::Q, H>;
  static constexpr int NW = 8;  // wavefronts per workgroup
  // 16 x 16 gradient tiles: per hidden row block ob the HB tiles of dW2 and
  // the bias tile of b2; the tiles of dW1 with b1 as input column Q; per
  // output row block qc the HB tiles of dW3 and the bias tile of b3.  A
  // bias tile contracts its operand with a ones fragment (every column
  // holds the sum); like b1, the biases of layers 2 and 3 are thus formed
  // from the operand-format d2 and dy of the weight gradients.
  static constexpr int R = S::HB + 1;
  static constexpr int NT2 = S::HB * R, NT1 = S::HB * S::KX, NT3 = S::QB * R;
  static constexpr int NT = NT2 + NT1 + NT3, TPW = (NT + NW - 1) / NW;
  // Tile j of wavefront W (-1: none).  At H = 64 a wavefront's tiles share
  // their operands: 2 x 2 blocks of dW2 (D3Q19: with the b2 tile of one of
  // the block's rows), the b2 tiles together (D2Q9), blocks of dW1 and of
  // dW3 with b3.  Per 16-node step the eight wavefronts then read 248
  // (D2Q9) or 256 (D3Q19) operand fragments from the slots instead of the
  // 280 and 328 of consecutive tiles.  Other shapes take consecutive tiles.
  static constexpr int tile(int W, int j) {
    if constexpr (S::HB == 4 && S::KX == 1 && S::QB == 1 && TPW == 4) {
      constexpr int m[8][4] = {{0, 1, 5, 6},     {2, 3, 7, 8},     {10, 11, 15, 16},
                               {12, 13, 17, 18}, {4, 9, 14, 19},   {20, 21, 22, 23},
                               {24, 25, 26, 28}, {27, -1, -1, -1}};
      return m[W][j];
    } else if constexpr (S::HB == 4 && S::KX == 2 && S::QB == 2 && TPW == 5) {
      constexpr int m[8][5] = {{0, 1, 5, 6, 4},       {2, 3, 7, 8, 9},
                               {10, 11, 15, 16, 14},  {12, 13, 17, 18, 19},
                               {20, 21, 22, 23, -1},  {24, 25, 26, 27, -1},
                               {28, 29, 33, 34, 32},  {30, 31, 35, 36, 37}};
      return m[W][j];
    } else {
      return W * TPW + j < NT ? W * TPW + j : -1;
    }
  }
  // loop order of the tile products: slot pairs outer for D3Q19, tiles
  // outer for D2Q9 (the other order spills registers in each)
  static constexpr bool PAIRS_OUTER = L::Q != 9;
  // every tile belongs to exactly one wavefront
  static constexpr bool tiles_ok() {
    int seen[NT] = {};
    for (int W = 0; W < NW; ++W)
      for (int j = 0; j < TPW; ++j) {
        const int t = tile(W, j);
        if (t >= NT || t < -1) return false;
        if (t >= 0 && seen[t]++) return false;
      }
    for (int t = 0; t < NT; ++t)
      if (!seen[t]) return false;
    return true;
  }
  // fragments of one group, in slot order
  static constexpr int FDY = 0, FH2 = FDY + S::QB, FD2 = FH2 + S::HB, FH1 = FD2 + S::HB,
                       FD1 = FH1 + S::HB, FX0 = FD1 + S::HB, NFR = FX0 + S::KX;
  // weight fragments: transposed for the backward products, then W1 and W2
  static constexpr int NFB = S::HB * S::QB + S::HB * S::HB + S::KX * S::HB;
  static constexpr int NFF = S::HB * S::KX + S::HB * S::HB;
  static constexpr int wts_bytes = (NFB + NFF) * 512 + H * 4;
  static constexpr int slot_bytes = NFR * 512;
  // Per-wavefront staging, one of two layouts.
  // Item layout: the 64 nodes' x0 rows (16-bit) and dy rows (float32,
  // overwritten by dx group by group), padded to whole 16-wide chunks.
  static constexpr int XS = 16 * S::KX + 4;                             // x0 row (16-bit elements)
  static constexpr int SD = 16 * (S::QB > S::KX ? S::QB : S::KX) + 4;  // dy / dx row (floats)
  static constexpr int item_wave_bytes = 64 * XS * 2 + 64 * SD * 4 + slot_bytes;
  // Compact layout, where the item layout does not fit (D3Q19): x0 and dy
  // as 16-bit rows of exactly the features in use (Q + 1 and Q, rounded up
  // to 4; the operand reads past them are zeros), dx as float32 rows of one
  // 16-node group.
  static constexpr int NXF = (S::Q + 1 + 3) / 4 * 4, NQF = (S::Q + 3) / 4 * 4;
  static constexpr int compact_wave_bytes = 64 * NXF * 2 + 64 * NQF * 2 + 16 * NXF * 4 + slot_bytes;
  static constexpr bool COMPACT = wts_bytes + NW * item_wave_bytes > 160 * 1024;
  static constexpr int wave_bytes = COMPACT ? compact_wave_bytes : item_wave_bytes;
  // byte offsets within a wavefront's region: x0 rows, dy rows, dx rows, slot
  static constexpr int xoff = 0;
  static constexpr int doff = COMPACT ? 64 * NXF * 2 : 64 * XS * 2;
  static constexpr int dxoff = COMPACT ? doff + 64 * NQF * 2 : doff;
  static constexpr int soff = COMPACT ? dxoff + 16 * NXF * 4 : doff + 64 * SD * 4;
  static constexpr int bytes = wts_bytes + NW * wave_bytes;
  static constexpr bool ok = P != P_F32 && bytes <= 160 * 1024 && S::n * 4 <= NW * wave_bytes &&
                             wave_bytes % 16 == 0;
  // tile t: kind 2 = dW2, 4 = b2, 1 = dW1|b1, 3 = dW3, 5 = b3; its row and
  // column block; the slot fragments of its A and B operands (-1: ones)
  static constexpr int kind(int t) {
    return t < NT2 ? (t % R < S::HB ? 2 : 4)
                   : (t < NT2 + NT1 ? 1 : ((t - NT2 - NT1) % R < S::HB ? 3 : 5));
  }
  static constexpr int row(int t) {
    return t < NT2 ? t / R : (t < NT2 + NT1 ? (t - NT2) / S::KX : (t - NT2 - NT1) / R);
  }
  static constexpr int col(int t) {
    return t < NT2 ? t % R : (t < NT2 + NT1 ? (t - NT2) % S::KX : (t - NT2 - NT1) % R);
  }
  static constexpr int fa(int t) {
    return kind(t) == 2 || kind(t) == 4 ? FD2 + row(t) : (kind(t) == 1 ? FD1 : FDY) + row(t);
  }
  static constexpr int fb(int t) {
    return kind(t) == 2 ? FH1 + col(t)
                        : (kind(t) == 1 ? FX0 + col(t) : (kind(t) == 3 ? FH2 + col(t) : -1));
  }
};

// Workgroups of the adjoint launch (one per compute unit); the workspace
// holds one partial gradient vector per workgroup.
constexpr unsigned bwd_blocks(int ncu) { return (unsigned)ncu; }

// All weights of the cooperative kernel in LDS, from one pass over theta by
// the NT threads of the workgroup (consecutive threads on consecutive
// parameters, every read issued before any is used).  Each value goes to its
// positions in the fragment-major arrays: bwd = W3^T (HB x QB fragments),
// W2^T (HB x HB), W1^T (KX x HB), as load_transposed_weights builds them;
// fwd = W1 with b1 as input column Q (HB x KX), then W2 (HB x HB), scaled
// like the forward's; b2s = c b2.  Padding entries are zero.
// Ends with a workgroup barrier.
template <class L, int H, int P, int NT>
__device__ inline void stage_adjoint_weights(typename Frag<P>::T* bwd, typename Frag<P>::T* fwd,
                                             float* b2s, const float* __restrict__ th) {
  using S = Shape<L::Q, H>;
  using F = typename Frag<P>::T;
  constexpr int Q = L::Q;
  constexpr int NF3 = S::HB * S::QB, NF2 = S::HB * S::HB, NFB = NF3 + NF2 + S::KX * S::HB;
  constexpr int N1 = S::HB * S::KX, NFF = N1 + S::HB * S::HB;
  constexpr float sc = tanh_weight_scale<P>();
  constexpr int C1 = (H * Q + NT - 1) / NT, CB = (H + NT - 1) / NT, C2 = (H * H + NT - 1) / NT,
                C3 = (Q * H + NT - 1) / NT;
  const int tid = threadIdx.x;
  float v1[C1], vb[CB], vb2[CB], v2[C2], v3[C3];
#pragma unroll
  for (int i = 0; i < C1; ++i) {
    const int j = tid + i * NT;
    v1[i] = j < H * Q ? th[S::oW1 + j] : 0.f;
  }
#pragma unroll
  for (int i = 0; i < CB; ++i) {
    const int j = tid + i * NT;
    vb[i] = j < H ? th[S::ob1 + j] : 0.f;
    vb2[i] = j < H ? th[S::ob2 + j] : 0.f;
  }
#pragma unroll
  for (int i = 0; i < C2; ++i) {
    const int j = tid + i * NT;
    v2[i] = j < H * H ? th[S::oW2 + j] : 0.f;
  }
#pragma unroll
  for (int i = 0; i < C3; ++i) {
    const int j = tid + i * NT;
    v3[i] = j < Q * H ? th[S::oW3 + j] : 0.f;
  }
  for (int e = tid; e < NFB * 64; e += NT) bwd[e] = F{};
  for (int e = tid; e < NFF * 64; e += NT) fwd[e] = F{};
  __syncthreads();
  // element r of fragment f, lane l = row % 16 + 16 ((k % 16) / 4), r = k % 4
  auto put = [&](F* fr, int f, int row, int k, float v) {
    const int e = 64 * f + (row & 15) + 16 * ((k & 15) >> 2);
    const unsigned w = pack2<P>(v, 0.f);
    reinterpret_cast<unsigned short*>(fr)[4 * e + (k & 3)] = (unsigned short)w;
  };
#pragma unroll
  for (int i = 0; i < C1; ++i) {
    const int j = tid + i * NT, o = j / Q, k = j - o * Q;
    if (j < H * Q) {
      put(fwd, (o >> 4) * S::KX + (k >> 4), o, k, sc * v1[i]);             // W1 (o, k)
      put(bwd, NF3 + NF2 + (k >> 4) * S::HB + (o >> 4), k, o, sc * v1[i]);  // W1^T (k, o)
    }
  }
#pragma unroll
  for (int i = 0; i < CB; ++i) {
    const int o = tid + i * NT;
    if (o < H) {
      put(fwd, (o >> 4) * S::KX + (Q >> 4), o, Q, sc * vb[i]);
      b2s[o] = sc * vb2[i];
    }
  }
#pragma unroll
  for (int i = 0; i < C2; ++i) {
    const int j = tid + i * NT, o = j / H, k = j - o * H;
    if (j < H * H) {
      put(fwd, N1 + (o >> 4) * S::HB + (k >> 4), o, k, sc * v2[i]);   // W2 (o, k)
      put(bwd, NF3 + (k >> 4) * S::HB + (o >> 4), k, o, sc * v2[i]);  // W2^T (k, o)
    }
  }
#pragma unroll
  for (int i = 0; i < C3; ++i) {
    const int j = tid + i * NT, q = j / H, h = j - q * H;
    if (j < Q * H) put(bwd, (h >> 4) * S::QB + (q >> 4), h, q, v3[i]);  // W3^T (h, q)
  }
  __syncthreads();
}

// acc[j] += the product of tile CL::tile(W, j) over the slots (the nodes of
// slots 2p and 2p + 1 form the K = 32 of one matrix-core instruction).  An
// operand fragment that several of the wavefront's tiles use is read once
// per pair (with CL::PAIRS_OUTER the pairs are the outer loop, else the
// compiler shares the reads); each tile sums the pairs in slot order.
template <class CL, int P, int W>
__device__ inline void coop_tiles(f4 (&acc)[CL::TPW], const unsigned char* slots, int rdo) {
  using Fr = typename Frag<P>::T;
  constexpr unsigned one2 = P == P_BF16 ? 0x3F803F80u : 0x3C003C00u;  // two 16-bit 1.0
  const Fr ones = {one2, one2};
  auto frag = [&](int w, int f) {
    return f < 0 ? ones : read_tr<P>(slots + w * CL::wave_bytes + f * 512 + rdo);
  };
  auto pair = [&](int j, int p) {
    const int t = CL::tile(W, j);
    if (t >= 0)
      acc[j] = mma_pair<P>(acc[j], frag(p, CL::fa(t)), frag(p + 1, CL::fa(t)),
                           frag(p, CL::fb(t)), frag(p + 1, CL::fb(t)));
  };
  if constexpr (CL::PAIRS_OUTER) {
#pragma unroll
    for (int p = 0; p < CL::NW; p += 2)
#pragma unroll
      for (int j = 0; j < CL::TPW; ++j) pair(j, p);
  } else {
#pragma unroll
    for (int j = 0; j < CL::TPW; ++j)
#pragma unroll
      for (int p = 0; p < CL::NW; p += 2) pair(j, p);
  }
}

// Tiles of wavefront W to their parameter entries (D layout: lane l holds
// rows 4 (l / 16) + r of column l % 16).
template <class CL, int W>
__device__ inline void coop_put(const f4 (&acc)[CL::TPW], float* red, int lg, int li) {
  using S = typename CL::S;
#pragma unroll
  for (int j = 0; j < CL::TPW; ++j) {
    const int t = CL::tile(W, j);
    if (t < 0) continue;
    const int a = 16 * CL::row(t) + 4 * lg, b = 16 * CL::col(t) + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float v = acc[j][r];
      switch (CL::kind(t)) {
        case 2: red[S::oW2 + (a + r) * S::H + b] = v; break;
        case 4: if (li == 0) red[S::ob2 + a + r] = v; break;
        case 1:
          if (b < S::Q) red[S::oW1 + (a + r) * S::Q + b] = v;
          else if (b == S::Q) red[S::ob1 + a + r] = v;
          break;
        case 3: if (a + r < S::Q) red[S::oW3 + (a + r) * S::H + b] = v; break;
        default: if (li == 0 && a + r < S::Q) red[S::ob3 + a + r] = v; break;
      }
    }
  }
}

// Dispatch on the (wave-uniform) wavefront index.
template <class CL, int P, int W = 0>
__device__ inline void coop_tiles_of(int wave, f4 (&acc)[CL::TPW], const unsigned char* slots,
                                     int rdo) {
  if constexpr (W + 1 < CL::NW) {
    if (wave == W) coop_tiles<CL, P, W>(acc, slots, rdo);
    else coop_tiles_of<CL, P, W + 1>(wave, acc, slots, rdo);
  } else {
    coop_tiles<CL, P, W>(acc, slots, rdo);
  }
}
template <class CL, int W = 0>
__device__ inline void coop_put_of(int wave, const f4 (&acc)[CL::TPW], float* red, int lg, int li) {
  if constexpr (W + 1 < CL::NW) {
    if (wave == W) coop_put<CL, W>(acc, red, lg, li);
    else coop_put_of<CL, W + 1>(wave, acc, red, lg, li);
  } else {
    coop_put<CL, W>(acc, red, lg, li);
  }
}

template <class L, int H, int P>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void
nlbm_backward_coop_kernel(const float* __restrict__ A, const float* __restrict__ theta,
                          const float* __restrict__ lam1, float* __restrict__ lam0,
                          float* __restrict__ part, Grid G, Force Fc, float rho0, float omega,
                          float knn, int nitems, int nxc, int accum) {
  using S = Shape<L::Q, H>;
  using CL = CoopLayout<L, H, P>;
  using Fr = typename Frag<P>::T;
  constexpr int Q = L::Q, NW = CL::NW;
  static_assert(CL::ok, "cooperative adjoint: precision or LDS budget");
  static_assert(CL::tiles_ok(), "cooperative adjoint: tile assignment");
  __shared__ Fr wts[(CL::NFB + CL::NFF) * 64];
  __shared__ __attribute__((aligned(16))) float b2s[H];  // c b2 (the layer-2 bias)
  __shared__ __attribute__((aligned(16))) unsigned char wl[NW * CL::wave_bytes];

  const int lane = threadIdx.x & 63, lg = lane >> 4, li = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  constexpr float sc = tanh_weight_scale<P>();
  stage_adjoint_weights<L, H, P, 64 * NW>(wts, wts + CL::NFB * 64, b2s, theta);
  const Fr* W3T = wts;
  const Fr* W2T = wts + S::HB * S::QB * 64;
  const Fr* W1T = wts + (S::HB * S::QB + S::HB * S::HB) * 64;
  const Fr* W1F = wts + CL::NFB * 64;
  const Fr* W2F = W1F + S::HB * S::KX * 64;

  unsigned char* mine = wl + wave * CL::wave_bytes;
  // item layout: X [64][XS] x0 (operand format), D [64][SD] dy then dx (float32);
  // compact layout: X [64][NXF] x0, Y [64][NQF] dy (operand format), DX [16][NXF] dx
  unsigned short* X = reinterpret_cast<unsigned short*>(mine + CL::xoff);
  float* D = reinterpret_cast<float*>(mine + CL::doff);
  unsigned short* Y = reinterpret_cast<unsigned short*>(mine + CL::doff);
  float* DX = reinterpret_cast<float*>(mine + CL::dxoff);
  unsigned char* slot = mine + CL::soff;
  const unsigned char* slots = wl + CL::soff;  // slot w at w * wave_bytes

  // Weight fragments in registers: all of them where two wavefronts per SIMD
  // hold them (the D2Q9 networks, 256 registers at H = 64); else all but W1,
  // which is then read from LDS per group (D3Q19 at H = 64: 256 registers;
  // W1 as well spills and runs slower, and of the four sets it gains least).
  constexpr bool RW1 = CL::NFB + CL::NFF <= 48;
  constexpr int N1 = S::HB * S::KX, N3 = S::HB * S::QB;
  Fr w2k[S::HB * S::HB], w2tk[S::HB * S::HB], w1tk[N1], w3tk[N3], w1k[RW1 ? N1 : 1];
#pragma unroll
  for (int i = 0; i < S::HB * S::HB; ++i) {
    w2k[i] = W2F[64 * i + lane];
    w2tk[i] = W2T[64 * i + lane];
  }
#pragma unroll
  for (int i = 0; i < N1; ++i) w1tk[i] = W1T[64 * i + lane];
#pragma unroll
  for (int i = 0; i < N3; ++i) w3tk[i] = W3T[64 * i + lane];
  if constexpr (RW1) {
#pragma unroll
    for (int i = 0; i < N1; ++i) w1k[i] = W1F[64 * i + lane];
  }
  // where all weights are in registers, the layer-2 bias c b2 is too
  f4 b2k[RW1 ? S::HB : 1];
  if constexpr (RW1) {
#pragma unroll
    for (int ob = 0; ob < S::HB; ++ob) b2k[ob] = *reinterpret_cast<const f4*>(b2s + 16 * ob + 4 * lg);
  }
  // this lane's rows of a slot fragment: written, and read transposed
  const int wro = 8 * slot_row(lane), rdo = 8 * tr_row(lane);

  // workgroup range of items; wavefront w takes item k + w of each step
  const int nb = gridDim.x, bid = blockIdx.x;
  const int lb = (nb % 8 == 0) ? (bid % 8) * (nb / 8) + bid / 8 : bid;
  const int per = (nitems + nb - 1) / nb;
  const int ib0 = min(lb * per, nitems), ib1 = min(ib0 + per, nitems);

  f4 acc[CL::TPW];
#pragma unroll
  for (int j = 0; j < CL::TPW; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};

  const unsigned bytes = (unsigned)G.plane * (unsigned)(G.batch * Q) * 4u;
  const rsrc_t rA = make_rsrc(A, bytes), rL1 = make_rsrc(lam1, bytes),
               rL0 = make_rsrc(lam0, bytes);
  // The next item's loads go out in two halves: the pulled populations
  // before the groups, lam^{n+1} with the second group (for D3Q19, with the
  // second or the third, odd and even wavefronts taking turns).  Issued at
  // once, the 2 Q loads of all the workgroup's wavefronts kept them waiting
  // for the address unit (1.5 us per item measured for D3Q19).
  // part 1: the pulled populations, 2: lam^{n+1}, 3: both.  Nodes past the
  // range enter as zeros (every product they feed is zero): mu is zeroed
  // where the item starts (zeroing it here, inside the group loop, made the
  // compiler wait there for the loads in flight), g there too for D2Q9 and
  // here for D3Q19, the faster placement for each in alternating runs.
  constexpr bool G_AT_START = L::Q == 9;
  auto load = [&](int it, const ItemWalk& w, float g[Q], float mu[Q], int part) {
    bool act = false;
    Item t;
    if (it < ib1) {
      t = w.item(G, lane);
      act = t.active;
    }
    if (act) {
      const ItemRows r(G, Q, t);
      if (part & 1) gather_rows<L>(rA, r, t, g);
      if (part & 2) load_rows<L>(rL1, r, t, mu);
    } else if (!G_AT_START && (part & 1)) {
#pragma unroll
      for (int q = 0; q < Q; ++q) g[q] = 0.f;
    }
  };

  // The wavefront's items are NW apart: they are walked without integer
  // division (one decode per launch; an item past the range keeps its walked
  // position and loads and stores nothing).
  ItemWalk wcur, wnxt;
  wcur.start(ib0 + wave, nxc, G);
  // The body force of an item is read before the stores of the previous
  // item (see wait_vmem): with the item's populations for D2Q9, at the end
  // of the previous item for D3Q19, whose registers (251 of 256) cannot hold
  // it across the groups without spilling.
  constexpr bool FORCE_EARLY = L::Q == 9;
  float gc[Q], mc[Q], F3[3] = {0.f, 0.f, 0.f};
  if (ib0 < ib1) {
    load(ib0 + wave, wcur, gc, mc, 3);
    if (Fc.kind != 0) {
      const Item t0 = wcur.item(G, lane);
      body_force(Fc, G, t0.x, t0.y, t0.z, F3);
    }
  }
  // no wait in the loop has to cover the loads issued before it
  wait_vmem();
  for (int k = ib0; k < ib1; k += NW) {
    const int it = k + wave;
    const Item t = wcur.item(G, lane);
    const bool act = it < ib1 && t.active;
    if (!act) {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        mc[q] = 0.f;
        if (G_AT_START) gc[q] = 0.f;
      }
    }
    float nu[Q], lam[Q];
    collide_adjoint<L>(gc, mc, rho0, omega, F3, Fc.kind != 0, nu, lam);

    // stage x0 (rounded to the operand format) and dy = k nu, node-major rows
    if constexpr (CL::COMPACT) {
#pragma unroll
      for (int c = 0; c < CL::NXF / 4; ++c) {
        f4 v;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int kk = 4 * c + r;
          v[r] = kk < Q ? gc[kk] : (kk == Q ? 1.f : 0.f);
        }
        *reinterpret_cast<Fr*>(X + lane * CL::NXF + 4 * c) = to_frag<P>(v);
      }
#pragma unroll
      for (int c = 0; c < CL::NQF / 4; ++c) {
        f4 v;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int q = 4 * c + r;
          v[r] = q < Q ? knn * nu[q] : 0.f;
        }
        *reinterpret_cast<Fr*>(Y + lane * CL::NQF + 4 * c) = to_frag<P>(v);
      }
    } else {
#pragma unroll
      for (int c = 0; c < 4 * S::KX; ++c) {
        f4 v;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int kk = 4 * c + r;
          v[r] = kk < Q ? gc[kk] : (kk == Q ? 1.f : 0.f);
        }
        *reinterpret_cast<Fr*>(X + lane * CL::XS + 4 * c) = to_frag<P>(v);
      }
#pragma unroll
      for (int c = 0; c < 4 * S::QB; ++c) {
        f4 v;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int q = 4 * c + r;
          v[r] = q < Q ? knn * nu[q] : 0.f;
        }
        *reinterpret_cast<f4*>(D + lane * CL::SD + 4 * c) = v;
      }
    }
    wave_lds_sync();
    // the next item's loads are in flight while this item's network runs
    wnxt = wcur;
    wnxt.advance(NW, nxc, G);
    if (k + NW < ib1) {
      load(it + NW, wnxt, gc, mc, 1);
      if (FORCE_EARLY && Fc.kind != 0) {
        const Item tn = wnxt.item(G, lane);
        body_force(Fc, G, tn.x, tn.y, tn.z, F3);
      }
    }

    // a D-layout fragment to the slot: lane l's four values to row slot_row(l)
    auto put_t = [&](int f, Fr v) { *reinterpret_cast<Fr*>(slot + f * 512 + wro) = v; };
#pragma unroll 1
    for (int jg = 0; jg < 4; ++jg) {
      const int nrow = 16 * jg + li;
      if (jg == (L::Q == 9 ? 1 : 1 + (wave & 1)) && k + NW < ib1) load(it + NW, wnxt, gc, mc, 2);
      // Weight fragments read from LDS come as one batch per layer, issued
      // before the VALU work of the previous layer so that their latency
      // overlaps it (the scheduling barriers keep the reads there).
      f4 t1[S::HB], t2[S::HB];
      {
        Fr xin[S::KX], w1l[RW1 ? 1 : N1], h1[S::HB], h2[S::HB];
        const Fr* w1 = w1k;
        if constexpr (!RW1) {
#pragma unroll
          for (int i = 0; i < N1; ++i) w1l[i] = W1F[64 * i + lane];
          w1 = w1l;
        }
#pragma unroll
        for (int c = 0; c < S::KX; ++c) {
          if constexpr (CL::COMPACT) {
            // features past NXF are zeros and are not stored
            xin[c] = 16 * c + 4 * lg < CL::NXF
                         ? *reinterpret_cast<const Fr*>(X + nrow * CL::NXF + 16 * c + 4 * lg)
                         : Fr{};
          } else {
            xin[c] = *reinterpret_cast<const Fr*>(X + nrow * CL::XS + 16 * c + 4 * lg);
          }
        }
        f4 a1[S::HB];
#pragma unroll
        for (int ob = 0; ob < S::HB; ++ob)
          a1[ob] = mma_row<P, S::KX>(f4{0.f, 0.f, 0.f, 0.f}, w1 + ob * S::KX, xin);
        const Fr* w2 = w2k;
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ob = 0; ob < S::HB; ++ob) {
          t1[ob] = tanh4<P>(a1[ob]);
          h1[ob] = to_frag<P>(t1[ob]);
        }
#pragma unroll
        for (int ob = 0; ob < S::HB; ++ob) {
          const f4 b2 = RW1 ? b2k[RW1 ? ob : 0] : *reinterpret_cast<const f4*>(b2s + 16 * ob + 4 * lg);
          t2[ob] = tanh4<P>(mma_row<P, S::HB>(b2, w2 + ob * S::HB, h1));
          h2[ob] = to_frag<P>(t2[ob]);
        }
        // every wavefront has finished reading the slots of the previous step
        __syncthreads();
        // x0, dy and the activations are all in D layout (feature 4 lg + r,
        // node li): each goes to the slot through the same transposing write
#pragma unroll
        for (int c = 0; c < S::KX; ++c) put_t(CL::FX0 + c, xin[c]);
#pragma unroll
        for (int ob = 0; ob < S::HB; ++ob) {
          put_t(CL::FH1 + ob, h1[ob]);
          put_t(CL::FH2 + ob, h2[ob]);
        }
      }
      {
        // dy in operand layout and in contraction layout
        Fr dyf[S::QB];
        const Fr* w3t = w3tk;
#pragma unroll
        for (int qc = 0; qc < S::QB; ++qc) {
          if constexpr (CL::COMPACT) {
            dyf[qc] = 16 * qc + 4 * lg < CL::NQF
                          ? *reinterpret_cast<const Fr*>(Y + nrow * CL::NQF + 16 * qc + 4 * lg)
                          : Fr{};
          } else {
            dyf[qc] = to_frag<P>(*reinterpret_cast<const f4*>(D + nrow * CL::SD + 16 * qc + 4 * lg));
          }
          put_t(CL::FDY + qc, dyf[qc]);
        }
        // d2 = (W3^T dy) (1 - t2^2),  d1 = (W2^T d2) (1 - t1^2)
        f4 a2[S::HB];
#pragma unroll
        for (int ob = 0; ob < S::HB; ++ob)
          a2[ob] = mma_row<P, S::QB>(f4{0.f, 0.f, 0.f, 0.f}, w3t + ob * S::QB, dyf);
        const Fr* w2t = w2tk;
        __builtin_amdgcn_sched_barrier(0);
        Fr d2f[S::HB], d1f[S::HB];
#pragma unroll
        for (int ob = 0; ob < S::HB; ++ob) {
          d2f[ob] = to_frag<P>(a2[ob] * (1.f - t2[ob] * t2[ob]));
          put_t(CL::FD2 + ob, d2f[ob]);
        }
        f4 a3[S::HB];
#pragma unroll
        for (int ob = 0; ob < S::HB; ++ob)
          a3[ob] = mma_row<P, S::HB>(f4{0.f, 0.f, 0.f, 0.f}, w2t + ob * S::HB, d2f);
        const Fr* w1t = w1tk;
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ob = 0; ob < S::HB; ++ob) {
          d1f[ob] = to_frag<P>(a3[ob] * (1.f / sc) * (1.f - t1[ob] * t1[ob]));
          put_t(CL::FD1 + ob, d1f[ob]);
        }
        // dx = W1^T d1 over this group's rows, whose dy has been read (item
        // layout), or into the group's dx rows (compact layout); the owner
        // lanes of the group's nodes add it to their lam
        wave_lds_sync();
#pragma unroll
        for (int c = 0; c < S::KX; ++c) {
          f4 a = mma_row<P, S::HB>(f4{0.f, 0.f, 0.f, 0.f}, w1t + c * S::HB, d1f);
          a = a * (1.f / sc);
          if constexpr (CL::COMPACT) {
            if (16 * c + 4 * lg < CL::NXF)
              *reinterpret_cast<f4*>(DX + li * CL::NXF + 16 * c + 4 * lg) = a;
          } else {
            *reinterpret_cast<f4*>(D + nrow * CL::SD + 16 * c + 4 * lg) = a;
          }
        }
        if constexpr (CL::COMPACT) {
          wave_lds_sync();
          if ((lane >> 4) == jg) {
#pragma unroll
            for (int q = 0; q < Q; ++q) lam[q] += DX[li * CL::NXF + q];
          }
        }
      }
      __syncthreads();
      // this wavefront's weight-gradient tiles over the nodes of the step
      coop_tiles_of<CL, P>(wave, acc, slots, rdo);
    }
    wave_lds_sync();
    if constexpr (!CL::COMPACT) {
#pragma unroll
      for (int q = 0; q < Q; ++q) lam[q] += D[lane * CL::SD + q];
    }
    if (!FORCE_EARLY && Fc.kind != 0 && k + NW < ib1) {
      const Item tn = wnxt.item(G, lane);
      body_force(Fc, G, tn.x, tn.y, tn.z, F3);
    }
    // the next item's loads arrived during the groups
    wait_vmem();
    if (act) scatter_rows<L>(rL0, ItemRows(G, Q, t), t, lam);
    wave_lds_sync();
    wcur = wnxt;
  }

  // Partial gradient of the workgroup: the tiles are disjoint between the
  // wavefronts and cover every parameter.
  __syncthreads();
  float* red = reinterpret_cast<float*>(wl);
  coop_put_of<CL>(wave, acc, red, lg, li);
  __syncthreads();
  float* pb = part + (size_t)blockIdx.x * S::n;
  for (int i = threadIdx.x; i < S::n; i += blockDim.x) pb[i] = accum ? pb[i] + red[i] : red[i];
}

// dtheta[p] += sum over the nb block partials part[b][p], in float64.
// Block = 64 parameters x 16 slices; slice s sums b = s, s + 16, ... with two
// independent accumulators; the sixteen slice sums are combined in slice
// order.  The order is fixed, so the result is bit-reproducible.
static __global__ __launch_bounds__(1024) void grad_reduce_kernel(const float* __restrict__ part,
                                                                 int nb, int np,
                                                                 float* __restrict__ dtheta) {
  const int pl = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const int p = blockIdx.x * 64 + pl;
  double a0 = 0.0, a1 = 0.0;
  if (p < np) {
    int b = sl;
    for (; b + 16 < nb; b += 32) {
      a0 += part[(size_t)b * np + p];
      a1 += part[(size_t)(b + 16) * np + p];
    }
    if (b < nb) a0 += part[(size_t)b * np + p];
  }
  __shared__ double red[16][64];
  red[sl][pl] = a0 + a1;
  __syncthreads();
  if (sl == 0 && p < np) {
    double t = red[0][pl];
    for (int k = 1; k < 16; ++k) t += red[k][pl];
    dtheta[p] += (float)t;
  }
}

// Launch of the adjoint kernel for (lattice, H, precision): the instances of
// each lattice are built in a translation unit of their own (nlbm_bwd.hip
// for D3Q19, nlbm_bwd_d2q9.hip for D2Q9), with their own scheduler options.
namespace bwd_detail {

template <class L, int H, int P>
hipError_t bwd_one(unsigned blocks, hipStream_t s, const float* A, const float* theta,
                   const float* lam1, float* lam0, float* part, Grid G, Force Fc, float rho0,
                   float omega, float knn, int nitems, int nxc, int accum) {
  if constexpr (CoopLayout<L, H, P>::ok)
    hipLaunchKernelGGL((nlbm_backward_coop_kernel<L, H, P>), dim3(blocks),
                       dim3(64 * CoopLayout<L, H, P>::NW), 0, s, A,
                       theta, lam1, lam0, part, G, Fc, rho0, omega, knn, nitems, nxc, accum);
  else
    hipLaunchKernelGGL((nlbm_backward_kernel<L, H, P>), dim3(blocks), dim3(256), 0, s, A, theta,
                       lam1, lam0, part, G, Fc, rho0, omega, knn, nitems, nxc, accum);
  return hipGetLastError();
}

template <class L, int H>
hipError_t bwd_prec(int prec, unsigned blocks, hipStream_t s, const float* A, const float* theta,
                    const float* lam1, float* lam0, float* part, Grid G, Force Fc, float rho0,
                    float omega, float knn, int nitems, int nxc, int accum) {
  switch (prec) {
    case P_F32:
      return bwd_one<L, H, P_F32>(blocks, s, A, theta, lam1, lam0, part, G, Fc, rho0, omega, knn, nitems, nxc, accum);
    case P_BF16:
      return bwd_one<L, H, P_BF16>(blocks, s, A, theta, lam1, lam0, part, G, Fc, rho0, omega, knn, nitems, nxc, accum);
    default:
      return bwd_one<L, H, P_F16>(blocks, s, A, theta, lam1, lam0, part, G, Fc, rho0, omega, knn, nitems, nxc, accum);
  }
}

template <class L>
hipError_t bwd_hidden(int hidden, int prec, unsigned blocks, hipStream_t s, const float* A,
                      const float* theta, const float* lam1, float* lam0, float* part, Grid G,
                      Force Fc, float rho0, float omega, float knn, int nitems, int nxc, int accum) {
  if (hidden == 32)
    return bwd_prec<L, 32>(prec, blocks, s, A, theta, lam1, lam0, part, G, Fc, rho0, omega, knn, nitems, nxc, accum);
  return bwd_prec<L, 64>(prec, blocks, s, A, theta, lam1, lam0, part, G, Fc, rho0, omega, knn, nitems, nxc, accum);
}

}  // namespace bwd_detail

hipError_t nlbm_bwd_launch_d2q9(int hidden, int prec, unsigned blocks, hipStream_t s,
                                const float* A, const float* theta, const float* lam1,
                                float* lam0, float* part, Grid G, Force Fc, float rho0,
                                float omega, float knn, int nitems, int nxc, int accum);

// Launch of the adjoint kernel for (lattice, H, precision), defined in
// nlbm_bwd.hip.  Each workgroup writes its partial gradient to its row of
// part (accum = 0) or adds it to what the row holds (accum = 1, for the
// steps of a sequence that share one reduction).
hipError_t nlbm_bwd_launch(bool d3q19, int hidden, int prec, unsigned blocks, hipStream_t s,
                           const float* A, const float* theta, const float* lam1, float* lam0,
                           float* part, Grid G, Force Fc, float rho0, float omega, float knn,
                           int nitems, int nxc, int accum);

}  // namespace lbm
