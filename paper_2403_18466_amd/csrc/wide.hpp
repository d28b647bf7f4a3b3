// wide.hpp -- stream-collide step with the collision network of the SI
// ("Neural Network Architecture and Optimization"): Q -> 300 -> 300 -> 100
// -> Q, LeakyReLU after the three hidden layers (negative slope 0.01), linear
// output, the kappa projection and eq. nn-model-full.
//
// At 255 200 multiply-add flops per node this network is the one variant of
// the step that the matrix cores bound, and its 128 k weights (256 KB in
// bf16) fit neither in registers nor in LDS.  The design:
//
//  * Activations stay in registers in MFMA "D layout" (see mlp.hpp): a
//    16-feature x 16-node chunk of one layer's output is directly a K = 16
//    slice of the next layer's B operand.  Layers are 300 -> 19 tiles of 16
//    rows (304), 100 -> 7 tiles (112), Q -> 1 or 2 tiles; padded rows have
//    zero weights and bias, so they stay zero through LeakyReLU.
//  * The weights stream through LDS.  Before a launch they are packed (once
//    per lbm_step call) into the A-operand fragment order of the kernel,
//    grouped into "steps": layer 1; then, for each group of RG layer-2
//    tiles, those rows of W2 together with the matching K columns of W3 (the
//    layer-3 contraction is accumulated group by group, so layer-2 outputs
//    never need to be held in full); then layer 4.  A block of 8 wavefronts
//    walks the steps in lockstep: while the matrix cores work on step s from
//    one LDS buffer, every thread's global loads of step s + 1 are in flight
//    and are written to the other buffer at the end of the step; one
//    barrier per step.
//  * Each wavefront owns work items of 64 nodes (one x-row segment, one node
//    per lane) for the gather, the BGK part and the store, and runs the
//    network over them in sweeps of NT 16-node tiles (NT = 2 for 16-bit
//    operands, 1 for float32, to stay within 256 registers so that two
//    wavefronts share each SIMD).
//  * A per-wavefront LDS tile holds, per node (row), the item's deviations g
//    and the constant 1 of the layer-1 bias column, then the network output
//    y in columns of its own, so g is still there when the item ends: the
//    BGK part, the projection of the whole update and the force are then
//    computed in node layout exactly as in the small network's kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "kernels_fwd.hpp"

namespace lbm {

// f(integral_constant<int, 0>), ..., f(integral_constant<int, N - 1>): a loop
// whose index is a compile-time constant in the body (the register arrays
// of the network are indexed by it).
template <class Fn, int... I>
__device__ __forceinline__ void static_for_impl(Fn&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class Fn>
__device__ __forceinline__ void static_for(Fn&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

constexpr float kLeakySlope = 0.01f;

__device__ inline f4 leaky4(f4 v) {
  f4 r;
#pragma unroll
  for (int k = 0; k < 4; ++k) r[k] = __builtin_fmaxf(v[k], kLeakySlope * v[k]);
  return r;
}

// Fragment layout of the packed weights (host and device agree on it).
//   chunk fragment: tile t (rows 16 t .. 16 t + 15), K chunk c; lane l holds
//     W[16 t + (l % 16)][16 c + 4 (l / 16) + r], r = 0..3,
//   a "pair" unit interleaves the fragments of chunks c and c + 1 per lane
//   (lane l: 4 values of chunk c, then 4 of chunk c + 1), a "single" unit
//   is one chunk fragment.  Units are consecutive in the order a step uses
//   them.  Bias vectors follow the weights as float32.
template <int Q_, int P>
struct WideLayout {
  static constexpr int Q = Q_;
  static constexpr int N1 = 300, N2 = 300, N3 = 100;
  static constexpr int T1 = 19, T2 = 19, T3 = 7, T4 = (Q + 15) / 16;  // output tiles
  static constexpr int K1 = (Q + 1 + 15) / 16, K2 = 19, K3 = 19, K4 = 7;  // input chunks
  static constexpr int EB = P == P_F32 ? 4 : 2;   // bytes per operand
  static constexpr int CHUNK = 64 * 4 * EB;      // bytes of one chunk fragment
  static constexpr int RG = P == P_F32 ? 1 : 2;  // layer-2 tiles per step
  static constexpr int NG = (T2 + RG - 1) / RG;  // layer-2/3 steps
  static constexpr int S1 = P == P_F32 ? 2 : 1;  // layer-1 steps
  static constexpr int TP1 = (T1 + S1 - 1) / S1; // layer-1 tiles per step
  static constexpr int NSTEP = S1 + NG + 1;      // S1 x layer 1, NG x layers 2/3, layer 4

  static constexpr int l1_tiles(int i) { return T1 - i * TP1 < TP1 ? T1 - i * TP1 : TP1; }
  static constexpr int group_tiles(int g) { return T2 - g * RG < RG ? T2 - g * RG : RG; }
  static constexpr int step_bytes(int s) {
    return s < S1 ? l1_tiles(s) * K1 * CHUNK
                  : (s < S1 + NG ? group_tiles(s - S1) * (K2 + T3) * CHUNK : T4 * K4 * CHUNK);
  }
  static constexpr int step_offset(int s) {
    int o = 0;
    for (int i = 0; i < s; ++i) o += step_bytes(i);
    return o;
  }
  static constexpr int max_step_bytes() {
    int m = 0;
    for (int i = 0; i < NSTEP; ++i) m = step_bytes(i) > m ? step_bytes(i) : m;
    return m;
  }
  static constexpr int weight_bytes = step_offset(NSTEP);
  // float32 bias region: b2 (T2 tiles), b3 (T3), b4 (T4), zero-padded
  static constexpr int fb2 = 0, fb3 = 16 * T2, fb4 = fb3 + 16 * T3, nbias = fb4 + 16 * T4;
  static constexpr int packed_bytes = weight_bytes + 4 * nbias;
  // offsets in the caller's packed parameter vector (W then b per layer)
  static constexpr int oW1 = 0, ob1 = N1 * Q, oW2 = ob1 + N1, ob2 = oW2 + N2 * N1,
                       oW3 = ob2 + N2, ob3 = oW3 + N3 * N2, oW4 = ob3 + N3, ob4 = oW4 + Q * N3,
                       nparam = ob4 + Q;
};

// packed[i] = theta[idx[i]] (0 where idx < 0), rounded to the operand type
// for the nw weight entries, float32 for the nb bias entries after them.
template <int P>
__global__ __launch_bounds__(256) void wide_pack_kernel(const float* __restrict__ theta,
                                                        const int* __restrict__ idx,
                                                        unsigned char* __restrict__ packed,
                                                        int nw, int nb) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nw + nb) return;
  const int j = idx[i];
  const float v = j >= 0 ? theta[j] : 0.f;
  if (i < nw) {
    if constexpr (P == P_F32) {
      reinterpret_cast<float*>(packed)[i] = v;
    } else if constexpr (P == P_BF16) {
      reinterpret_cast<__bf16*>(packed)[i] = (__bf16)v;
    } else {
      reinterpret_cast<_Float16*>(packed)[i] = (_Float16)v;
    }
  } else {
    reinterpret_cast<float*>(packed + (size_t)nw * (P == P_F32 ? 4 : 2))[i - nw] = v;
  }
}

// A-operand reads from a staged unit (p = unit base in LDS).
template <int P>
__device__ inline void lds_pair(const unsigned char* p, int lane, typename Frag<P>::T& a0,
                                typename Frag<P>::T& a1) {
  if constexpr (P == P_F32) {
    a0 = *reinterpret_cast<const f4*>(p + lane * 32);
    a1 = *reinterpret_cast<const f4*>(p + lane * 32 + 16);
  } else {
    const u4 v = *reinterpret_cast<const u4*>(p + lane * 16);
    a0 = u2{v[0], v[1]};
    a1 = u2{v[2], v[3]};
  }
}
template <int P>
__device__ inline typename Frag<P>::T lds_single(const unsigned char* p, int lane) {
  if constexpr (P == P_F32)
    return *reinterpret_cast<const f4*>(p + lane * 16);
  else
    return *reinterpret_cast<const u2*>(p + lane * 8);
}

// The A fragments of one staged unit: a chunk pair (a0, a1) or a single
// chunk (a0).
template <int P>
struct Unit {
  typename Frag<P>::T a0, a1;
};

template <int P, bool PAIR>
__device__ inline void lds_unit(const unsigned char* p, int lane, Unit<P>& f) {
  if constexpr (PAIR)
    lds_pair<P>(p, lane, f.a0, f.a1);
  else
    f.a0 = lds_single<P>(p, lane);
}

// Software pipeline over the U units of one step: the LDS reads run D units
// ahead of the matrix-core work that consumes them, in a ring of D + 1
// fragment sets.  rd(u, slot) reads unit u; pre() runs once the first reads
// are in flight (the VALU work that the step starts with); cs(u, slot)
// issues unit u's MFMAs.
template <int P, int U, int D, class Rd, class Pre, class Cs>
__device__ __forceinline__ void lds_pipeline(Rd&& rd, Pre&& pre, Cs&& cs) {
  constexpr int D0 = D < U ? D : U;
  Unit<P> ring[D + 1];
  static_for<D0>([&](auto ic) { rd(ic, ring[decltype(ic)::value]); });
  pre();
  static_for<U>([&](auto uc) {
    constexpr int u = decltype(uc)::value;
    if constexpr (u + D < U) rd(std::integral_constant<int, u + D>{}, ring[(u + D) % (D + 1)]);
    cs(uc, ring[u % (D + 1)]);
    // keeps the scheduler from sinking the reads back to their first use
    __builtin_amdgcn_sched_barrier(0);
  });
}

// Wave-uniform byte offsets of the rows one 64-node item reads and writes:
// the start of field b, the plane stride, and the rows y - c_y, z - c_z for
// c in {-1, 0, 1} (periodic); every population's row is a sum of these.
struct RowOffsets {
  unsigned field, plane;
  unsigned yo[3], zo[3];  // index c + 1
};

__device__ inline RowOffsets row_offsets(const Grid& G, int Q, int b, int y, int z) {
  RowOffsets r;
  b = __builtin_amdgcn_readfirstlane(b);
  y = __builtin_amdgcn_readfirstlane(y);
  z = __builtin_amdgcn_readfirstlane(z);
  const unsigned rowb = (unsigned)G.nx * 4u;
  r.plane = (unsigned)G.plane * 4u;
  r.field = (unsigned)(b * Q) * r.plane;
#pragma unroll
  for (int c = -1; c <= 1; ++c) {
    r.yo[c + 1] = (unsigned)wrap_sub(y, c, G.ny) * rowb;
    r.zo[c + 1] = (unsigned)wrap_sub(z, c, G.nz) * rowb * (unsigned)G.ny;
  }
  return r;
}

// g_q = A_q(x - c_q) for this lane's node.
template <class L, int q = 0>
__device__ inline void gather_rows(rsrc_t src, const RowOffsets& r, const Item& t, float g[L::Q]) {
  if constexpr (q < L::Q) {
    const unsigned so = r.field + q * r.plane + r.zo[L::cz[q] + 1] + r.yo[L::cy[q] + 1];
    const int vo = L::cx[q] > 0 ? t.vm : (L::cx[q] < 0 ? t.vp : t.vx);
    g[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(src, vo, (int)so, 0));
    gather_rows<L, q + 1>(src, r, t, g);
  }
}

template <class L>
__device__ inline void store_rows(rsrc_t dst, const RowOffsets& r, const Item& t, const float v[L::Q]) {
#pragma unroll
  for (int q = 0; q < L::Q; ++q)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v[q]), dst, t.vx,
                                          (int)(r.field + q * r.plane + r.zo[1] + r.yo[1]), 0);
}

template <class L, int P>
struct WideCfg {
  using WL = WideLayout<L::Q, P>;
  static constexpr int NT = P == P_F32 ? 1 : 2;  // 16-node tiles per sweep
  static constexpr int NS = 4 / NT;              // sweeps per 64-node item
  static constexpr int WAVES = 8;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int SB = WL::max_step_bytes();
  static constexpr int NLD = (SB / 16 + THREADS - 1) / THREADS;  // 16-byte loads per thread
  static constexpr int PD = P == P_F32 ? 2 : 3;  // LDS read distance of the step pipelines (units)
  // tile columns: g (Q), the bias input 1, zeros up to YC; y (Q, padded to 4)
  static constexpr int YC = (L::Q + 1 + 3) / 4 * 4;
  static constexpr int SX = YC + (L::Q + 3) / 4 * 4 + 4;  // row stride (floats)
  static constexpr int lds_bytes = 2 * SB + 4 * WL::nbias + 4 * WAVES * 64 * SX;
  static_assert(NLD * THREADS * 16 >= SB, "one pass of stage loads covers a step");
};

template <class L, int P>
__global__ __launch_bounds__(512) void wide_step_kernel(const float* __restrict__ Ain,
                                                        float* __restrict__ Aout,
                                                        const unsigned char* __restrict__ packed,
                                                        Grid G, Force Fc, float rho0,
                                                        float omega, float knn, int per,
                                                        int nitems, int nxc) {
  using C = WideCfg<L, P>;
  using WL = typename C::WL;
  using F = typename Frag<P>::T;
  constexpr int Q = L::Q, NT = C::NT, NS = C::NS, SX = C::SX, SB = C::SB;
  constexpr int CH = WL::CHUNK;

  // step s is read from stage0 for even s, stage1 for odd s (NSTEP is even,
  // so the assignment is the same in every sweep)
  static_assert(WL::NSTEP % 2 == 0, "the stage buffers alternate by step parity");
  __shared__ __attribute__((aligned(16))) unsigned char stage0[SB];
  __shared__ __attribute__((aligned(16))) unsigned char stage1[SB];
  __shared__ __attribute__((aligned(16))) float bias[WL::nbias];
  __shared__ __attribute__((aligned(16))) float tiles[C::WAVES * 64 * SX];

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63, lg = lane >> 4, li = lane & 15;
  float* T = tiles + wave * 64 * SX;

  const int nb = gridDim.x, bid = blockIdx.x;
  const int lb = (nb % 8 == 0) ? (bid % 8) * (nb / 8) + bid / 8 : bid;
  const int it0 = (lb * C::WAVES + wave) * per;

  const rsrc_t wsrc = make_rsrc(reinterpret_cast<const float*>(packed), (unsigned)WL::packed_bytes);
  const unsigned bytes = (unsigned)G.plane * (unsigned)(G.batch * Q) * 4u;
  const rsrc_t src = make_rsrc(Ain, bytes), dst = make_rsrc(Aout, bytes);

  // loads of a step's packed weights straight into an LDS stage buffer
  // (16 bytes per lane, a wavefront's 64 lanes fill 1 KB in lane order); they
  // land while the matrix cores work on the other buffer, and the barrier at
  // the end of the step waits for them
  // (the lane part of the source offset is one register, tid * 16; the step
  // and pass parts go to the scalar offset, kept opaque so that the compiler
  // does not fold them into a vector register per load)
  const int voff = tid * 16;
  auto stage_issue = [&](unsigned char* dstbuf, int off, int nbytes) {
#pragma unroll
    for (int j = 0; j < C::NLD; ++j) {
      const int i = tid + j * C::THREADS;
      int so = off + j * C::THREADS * 16;
      asm volatile("" : "+s"(so));
      if (i * 16 < nbytes)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            wsrc, (__attribute__((address_space(3))) void*)(dstbuf + (j * C::THREADS + wave * 64) * 16),
            16, voff, so, 0, 0);
    }
  };

  // prologue: biases and step 0 into buffer 0
  for (int i = tid; i < WL::nbias; i += C::THREADS)
    bias[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(wsrc, WL::weight_bytes + 4 * i, 0, 0));
  stage_issue(stage0, WL::step_offset(0), WL::step_bytes(0));
  __syncthreads();

  // the walk state is wave-uniform: keep it in scalar registers
  auto uniform = [](ItemWalk& w) {
    w.xc = __builtin_amdgcn_readfirstlane(w.xc);
    w.y = __builtin_amdgcn_readfirstlane(w.y);
    w.z = __builtin_amdgcn_readfirstlane(w.z);
    w.b = __builtin_amdgcn_readfirstlane(w.b);
  };
  ItemWalk cur, nxt;
  cur.start(it0 < nitems ? it0 : nitems - 1, nxc, G);
  uniform(cur);
  float gn[Q];
  if (it0 < nitems) {
    const Item t0 = cur.item(G, lane);
    gather_rows<L>(src, row_offsets(G, Q, t0.b, t0.y, t0.z), t0, gn);
  }

  constexpr int YC = C::YC;
  for (int k = 0; k < per; ++k) {
    const bool valid = it0 + k < nitems;
    const bool more = k + 1 < per && it0 + k + 1 < nitems;
    // item start: the network input row of this lane's node
#pragma unroll
    for (int q = 0; q < Q; ++q) T[lane * SX + q] = gn[q];
#pragma unroll
    for (int q = Q; q < YC; ++q) T[lane * SX + q] = q == Q ? 1.f : 0.f;
    wave_lds_sync();
    nxt = cur;
    nxt.next(nxc, G);
    uniform(nxt);

    static_for<NS>([&](auto swc) {
      constexpr int sw = decltype(swc)::value;
      constexpr int row0 = sw * 16 * NT;
      F x[WL::K1][NT];
      F h1[WL::T1][NT];
      f4 acc3[WL::T3][NT];
      static_for<WL::NSTEP>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        constexpr int sn = (s + 1) % WL::NSTEP;
        stage_issue(s % 2 == 0 ? stage1 : stage0, WL::step_offset(sn), WL::step_bytes(sn));
        if constexpr (s == WL::NSTEP - 1 && sw == NS - 1) {
          if (more) {
            const Item tn = nxt.item(G, lane);
            gather_rows<L>(src, row_offsets(G, Q, tn.b, tn.y, tn.z), tn, gn);
          }
        }
        const unsigned char* S = s % 2 == 0 ? stage0 : stage1;
        if constexpr (s < WL::S1) {
          // layer 1: h1 = leaky(W1 [g, 1]); input columns past YC are zero.
          // Units: tile-major, chunk pairs then the odd chunk.
          if constexpr (s == 0) {
#pragma unroll
            for (int n = 0; n < NT; ++n)
#pragma unroll
              for (int c = 0; c < WL::K1; ++c) {
                const int col = 16 * c + 4 * lg;
                f4 v = *reinterpret_cast<const f4*>(T + (row0 + 16 * n + li) * SX +
                                                    (col < YC ? col : 0));
                if (col >= YC) v = f4{0.f, 0.f, 0.f, 0.f};
                x[c][n] = to_frag<P>(v);
              }
          }
          constexpr int NP = WL::K1 / 2, KU = NP + WL::K1 % 2, NTL = WL::l1_tiles(s);
          f4 acc[NT];
          lds_pipeline<P, NTL * KU, C::PD>(
              [&](auto uc, Unit<P>& f) {
                constexpr int u = decltype(uc)::value, j = u / KU, k = u % KU;
                lds_unit<P, (k < NP)>(S + j * WL::K1 * CH + 2 * k * CH, lane, f);
              },
              [&] {},
              [&](auto uc, const Unit<P>& f) {
                constexpr int u = decltype(uc)::value, j = u / KU, k = u % KU;
                constexpr int tt = s * WL::TP1 + j;
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                  const f4 a = k == 0 ? f4{0.f, 0.f, 0.f, 0.f} : acc[n];
                  if constexpr (k < NP)
                    acc[n] = mma_pair<P>(a, f.a0, f.a1, x[2 * k][n], x[2 * k + 1][n]);
                  else
                    acc[n] = mma_chunk<P>(a, f.a0, x[WL::K1 - 1][n]);
                }
                if constexpr (k == KU - 1) {
#pragma unroll
                  for (int n = 0; n < NT; ++n) h1[tt][n] = to_frag<P>(leaky4(acc[n]));
                }
              });
          if constexpr (s == WL::S1 - 1) {
#pragma unroll
            for (int t3 = 0; t3 < WL::T3; ++t3) {
              const f4 b = *reinterpret_cast<const f4*>(bias + WL::fb3 + 16 * t3 + 4 * lg);
#pragma unroll
              for (int n = 0; n < NT; ++n) acc3[t3][n] = b;
            }
          }
        } else if constexpr (s < WL::S1 + WL::NG) {
          // layer-2 tiles of group g, then their share of layer 3.  Units:
          // layer-2 chunk pairs (pair-major, tile-minor, so consecutive MFMAs
          // feed different accumulators), the odd layer-2 chunk of each
          // tile, then one unit per layer-3 tile; the layer-3 reads are in
          // flight while the last layer-2 MFMAs and the activation run.
          constexpr int g = s - WL::S1;
          constexpr int GT = WL::group_tiles(g);
          constexpr int NP = WL::K2 / 2, KU = NP + WL::K2 % 2, U2 = KU * GT;
          const unsigned char* S3 = S + GT * WL::K2 * CH;
          f4 acc[GT][NT];
          F h2[WL::RG][NT];
#pragma unroll
          for (int j = 0; j < GT; ++j) {
            const f4 b = *reinterpret_cast<const f4*>(bias + WL::fb2 + 16 * (g * WL::RG + j) + 4 * lg);
#pragma unroll
            for (int n = 0; n < NT; ++n) acc[j][n] = b;
          }
          lds_pipeline<P, U2 + WL::T3, C::PD>(
              [&](auto uc, Unit<P>& f) {
                constexpr int u = decltype(uc)::value;
                if constexpr (u < U2) {
                  constexpr int k = u / GT, j = u % GT;
                  lds_unit<P, (k < NP)>(S + j * WL::K2 * CH + 2 * k * CH, lane, f);
                } else {
                  lds_unit<P, (GT == 2)>(S3 + (u - U2) * GT * CH, lane, f);
                }
              },
              [&] {},
              [&](auto uc, const Unit<P>& f) {
                constexpr int u = decltype(uc)::value;
                if constexpr (u < U2) {
                  constexpr int k = u / GT, j = u % GT;
#pragma unroll
                  for (int n = 0; n < NT; ++n) {
                    if constexpr (k < NP)
                      acc[j][n] = mma_pair<P>(acc[j][n], f.a0, f.a1, h1[2 * k][n], h1[2 * k + 1][n]);
                    else
                      acc[j][n] = mma_chunk<P>(acc[j][n], f.a0, h1[WL::K2 - 1][n]);
                  }
                  if constexpr (u == U2 - 1) {
#pragma unroll
                    for (int jj = 0; jj < GT; ++jj)
#pragma unroll
                      for (int n = 0; n < NT; ++n) h2[jj][n] = to_frag<P>(leaky4(acc[jj][n]));
                  }
                } else {
                  constexpr int t3 = u - U2;
#pragma unroll
                  for (int n = 0; n < NT; ++n) {
                    if constexpr (GT == 2)
                      acc3[t3][n] = mma_pair<P>(acc3[t3][n], f.a0, f.a1, h2[0][n], h2[WL::RG - 1][n]);
                    else
                      acc3[t3][n] = mma_chunk<P>(acc3[t3][n], f.a0, h2[0][n]);
                  }
                }
              });
        } else {
          // layer 4: y = W4 leaky(acc3) + b4, rows < Q written to the tile.
          // Units: chunk-major, tile-minor.
          constexpr int NP = WL::K4 / 2, KU = NP + WL::K4 % 2;
          F h3[WL::T3][NT];
          f4 acc[WL::T4][NT];
          lds_pipeline<P, KU * WL::T4, C::PD>(
              [&](auto uc, Unit<P>& f) {
                constexpr int u = decltype(uc)::value, k = u / WL::T4, t4 = u % WL::T4;
                lds_unit<P, (k < NP)>(S + t4 * WL::K4 * CH + 2 * k * CH, lane, f);
              },
              [&] {
#pragma unroll
                for (int t3 = 0; t3 < WL::T3; ++t3)
#pragma unroll
                  for (int n = 0; n < NT; ++n) h3[t3][n] = to_frag<P>(leaky4(acc3[t3][n]));
#pragma unroll
                for (int t4 = 0; t4 < WL::T4; ++t4) {
                  const f4 b = *reinterpret_cast<const f4*>(bias + WL::fb4 + 16 * t4 + 4 * lg);
#pragma unroll
                  for (int n = 0; n < NT; ++n) acc[t4][n] = b;
                }
              },
              [&](auto uc, const Unit<P>& f) {
                constexpr int u = decltype(uc)::value, k = u / WL::T4, t4 = u % WL::T4;
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                  if constexpr (k < NP)
                    acc[t4][n] = mma_pair<P>(acc[t4][n], f.a0, f.a1, h3[2 * k][n], h3[2 * k + 1][n]);
                  else
                    acc[t4][n] = mma_chunk<P>(acc[t4][n], f.a0, h3[WL::K4 - 1][n]);
                }
                if constexpr (k == KU - 1) {
                  const int row = 16 * t4 + 4 * lg;
                  if (row < Q) {
#pragma unroll
                    for (int n = 0; n < NT; ++n)
                      *reinterpret_cast<f4*>(T + (row0 + 16 * n + li) * SX + YC + row) = acc[t4][n];
                  }
                }
              });
        }
        __syncthreads();
      });
    });

    // item end (node layout): BGK, network term, projection, force, store
    {
      const Item t = cur.item(G, lane);
      float g[Q], upd[Q], rho, u[3];
#pragma unroll
      for (int q = 0; q < Q; ++q) g[q] = T[lane * SX + q];
      bgk_update<L>(g, rho0, omega, upd, rho, u);
#pragma unroll
      for (int q = 0; q < Q; ++q) upd[q] = __builtin_fmaf(knn, T[lane * SX + YC + q], upd[q]);
      float F3[3] = {0.f, 0.f, 0.f};
      if (Fc.kind != 0) body_force(Fc, G, t.x, t.y, t.z, F3);
      float post[Q];
      finish_collision<L>(g, upd, rho, u, F3, Fc.kind != 0, post);
      if (valid && t.active) store_rows<L>(dst, row_offsets(G, Q, t.b, t.y, t.z), t, post);
    }
    wave_lds_sync();
    cur = nxt;
  }
}

// Launches, defined in wide.hip (prec: a Prec value).
hipError_t wide_step_launch(bool d3q19, int prec, unsigned nb, hipStream_t s, const float* Ain,
                            float* Aout, const unsigned char* packed, Grid G, Force Fc,
                            float rho0, float omega, float knn, int per, int nitems, int nxc);
hipError_t wide_pack_launch(int prec, unsigned blocks, hipStream_t s, const float* theta,
                            const int* idx, unsigned char* packed, int nw, int nb);

}  // namespace lbm
