// mlp.hpp -- the per-node network Q -> H -> H -> Q (tanh, tanh, linear) of
// the collision correction (SI, "Neural Network Architecture and
// Optimization"; activation and widths per the workload), evaluated on the
// matrix cores of gfx950 for 16 nodes at a time.
//
// Orientation.  Every layer computes out[o][n] = sum_k W[o][k] in[k][n] for a
// group of 16 nodes n, with the weights as the MFMA A operand and the node
// activations as the B operand.  The MFMA result ("D layout") gives lane l
// the rows 4*(l/16) + r, r = 0..3, of column l % 16.  A block of 16
// features x 16 nodes in D layout is called a chunk.  Because the
// contraction index may be permuted freely as long as A and B agree, a chunk
// in D layout is directly a K = 16 slice of the next layer's B operand: lane
// group g = l/16 supplies k = 4g + r.  The weight fragments are loaded with
// the same k mapping, so activations never leave registers between layers.
//
// Precisions.
//   F32:  v_mfma_f32_16x16x4_f32, four per chunk (the r-th uses k = 4g + r).
//   BF16: v_mfma_f32_16x16x16_bf16 per chunk, or v_mfma_f32_16x16x32_bf16 per
//         pair of chunks (k = 8g + t maps to chunk c0 for t < 4, c1 for t >= 4).
//   F16:  the same with f16.
// Accumulation is float32 in all three.
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

enum Prec { P_F32 = 1, P_BF16 = 2, P_F16 = 3 };

typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned u2 __attribute__((ext_vector_type(2)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef _Float16 hf2 __attribute__((ext_vector_type(2)));

template <int P>
struct Frag;
template <>
struct Frag<P_F32> {
  using T = f4;
};
template <>
struct Frag<P_BF16> {
  using T = u2;
};
template <>
struct Frag<P_F16> {
  using T = u2;
};

// Round two float32 values to the operand format (round to nearest even) and
// pack them into one dword, first value in the low half.
template <int P>
__device__ inline unsigned pack2(float a, float b);
template <>
__device__ inline unsigned pack2<P_BF16>(float a, float b) {
  bf2 r = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(unsigned, r);
}
template <>
__device__ inline unsigned pack2<P_F16>(float a, float b) {
  // The empty asm keeps the compiler from fusing a preceding fma with the
  // conversion into v_fma_mix{lo,hi}_f16: their half-register writes ran the
  // fp16 step 5% slower than fma + v_cvt_pk_f16_f32 (the bf16 pattern).
  asm("" : "+v"(a), "+v"(b));
  hf2 r = {(_Float16)a, (_Float16)b};
  return __builtin_bit_cast(unsigned, r);
}

template <int P>
__device__ inline typename Frag<P>::T to_frag(f4 v) {
  if constexpr (P == P_F32) {
    return v;
  } else {
    u2 r = {pack2<P>(v[0], v[1]), pack2<P>(v[2], v[3])};
    return r;
  }
}

// acc += A(16 x 16) * B(16 x 16) for one K = 16 chunk.
template <int P>
__device__ inline f4 mma_chunk(f4 acc, typename Frag<P>::T a, typename Frag<P>::T b) {
  if constexpr (P == P_F32) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], acc, 0, 0, 0);
    return acc;
  } else if constexpr (P == P_BF16) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a),
                                                     __builtin_bit_cast(s4, b), acc, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(h4, a),
                                                 __builtin_bit_cast(h4, b), acc, 0, 0, 0);
  }
}

// acc += A * B for two K chunks at once.
template <int P>
__device__ inline f4 mma_pair(f4 acc, typename Frag<P>::T a0, typename Frag<P>::T a1,
                              typename Frag<P>::T b0, typename Frag<P>::T b1) {
  if constexpr (P == P_F32) {
    return mma_chunk<P>(mma_chunk<P>(acc, a0, b0), a1, b1);
  } else {
    u4 a = {a0[0], a0[1], a1[0], a1[1]};
    u4 b = {b0[0], b0[1], b1[0], b1[1]};
    if constexpr (P == P_BF16)
      return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, a),
                                                     __builtin_bit_cast(b8, b), acc, 0, 0, 0);
    else
      return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a),
                                                    __builtin_bit_cast(h8, b), acc, 0, 0, 0);
  }
}

// acc += sum over NC input chunks.
template <int P, int NC>
__device__ inline f4 mma_row(f4 acc, const typename Frag<P>::T* w, const typename Frag<P>::T* x) {
  int c = 0;
#pragma unroll
  for (; c + 1 < NC; c += 2) acc = mma_pair<P>(acc, w[c], w[c + 1], x[c], x[c + 1]);
  if constexpr (NC % 2 == 1) acc = mma_chunk<P>(acc, w[NC - 1], x[NC - 1]);
  return acc;
}

// The same with the weight fragments in LDS, fragment-major (fragment c of
// this lane at w[64 c]).
template <int P, int NC>
__device__ inline f4 mma_row_lds(f4 acc, const typename Frag<P>::T* w,
                                 const typename Frag<P>::T* x) {
  int c = 0;
#pragma unroll
  for (; c + 1 < NC; c += 2) acc = mma_pair<P>(acc, w[64 * c], w[64 * (c + 1)], x[c], x[c + 1]);
  if constexpr (NC % 2 == 1) acc = mma_chunk<P>(acc, w[64 * (NC - 1)], x[NC - 1]);
  return acc;
}

// tanh(z) = 1 - 2 / (1 + e^{2z}), with e^{2z} = 2^{2 z log2(e)} on the
// hardware exp2 and the hardware reciprocal.  Saturates to +-1 without a
// clamp: e^{2z} overflows to +inf (reciprocal 0) or underflows to 0.
__device__ inline float tanh_fast(float z) {
  float e = __builtin_amdgcn_exp2f(z * 2.8853900817779268f);
  return __builtin_fmaf(-2.f, __builtin_amdgcn_rcpf(1.f + e), 1.f);
}

// The float32 network's tanh is accurate to a few float32 ulps everywhere:
// the exp form above for |z| >= 0.55, and below it (where 1 - 2r cancels and
// loses all relative accuracy)
//   tanh z = z + z^3 P(z^2),
// with P the degree-4 least-squares fit of (tanh z - z) / z^3 in s = z^2,
// weighted by s, on 4000 Chebyshev nodes of s in [0, 0.55^2] (max relative
// error 6.4e-8 in float32); above it the exp form is within 2.9e-7.
__device__ inline float tanh_small(float z) {
  const float s = z * z;
  float p = __builtin_fmaf(-0.006272607482969761f, s, 0.02107025310397148f);
  p = __builtin_fmaf(p, s, -0.053851865231990814f);
  p = __builtin_fmaf(p, s, 0.13332580029964447f);
  p = __builtin_fmaf(p, s, -0.33333316445350647f);
  return __builtin_fmaf(z * s, p, z);
}

// Scale of the tanh argument on the hardware exp2: e^{2z} = 2^{c z},
// c = 2 log2(e).  The bf16 / fp16 networks carry it in the weights and the
// bias of the two tanh layers (the operand then holds c W rounded to the
// format), so their activation starts at exp2 of the accumulator.
constexpr float kTanhScale = 2.8853900817779268f;

// tanh(z) from v = c z: 1 - 2 / (1 + 2^v).
__device__ inline float tanh_prescaled(float v) {
  return __builtin_fmaf(-2.f, __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(v)), 1.f);
}

// Scale applied to the tanh layers' weights for precision P.
template <int P>
__device__ constexpr float tanh_weight_scale() {
  return P == P_F32 ? 1.f : kTanhScale;
}

// Activation of the precision, from the accumulator of a tanh layer: the
// float32 network needs the accurate tanh to stay within 1e-5 of float64
// over hundreds of steps; the bf16 / fp16 networks round the activation to
// 8 / 11 bits, far above the fast form's ~1e-7 absolute error, and their
// accumulator is already c z.
template <int P>
__device__ inline f4 tanh4(f4 v) {
  f4 r;
  if constexpr (P == P_F32) {
    // |v| < 0.55 ? tanh_small(v) : tanh_fast(v) per value, with one
    // wave-wide decision for the four values instead of a branch per value:
    // where every lane's four values fall on one side of 0.55 only that
    // side's form is evaluated, else both are and one is selected per value
    bool small = true, big = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool s = __builtin_fabsf(v[k]) < 0.55f;
      small = small && s;
      big = big && !s;
    }
    if (__builtin_amdgcn_ballot_w64(!small) == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) r[k] = tanh_small(v[k]);
    } else if (__builtin_amdgcn_ballot_w64(!big) == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) r[k] = tanh_fast(v[k]);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float a = tanh_small(v[k]), b = tanh_fast(v[k]);
        r[k] = __builtin_fabsf(v[k]) < 0.55f ? a : b;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = tanh_prescaled(v[k]);
  }
  return r;
}

// Network shape for Q populations and H hidden units.
template <int Q_, int H_>
struct Shape {
  static constexpr int Q = Q_, H = H_;
  static constexpr int KX = (Q + 1 + 15) / 16;  // input chunks: Q populations + bias slot
  static constexpr int HB = H / 16;             // hidden chunks
  static constexpr int QB = (Q + 15) / 16;      // output chunks
  // offsets in the packed parameter vector [W1 b1 W2 b2 W3 b3]
  static constexpr int oW1 = 0, ob1 = H * Q, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H,
                       ob3 = oW3 + Q * H, n = ob3 + Q;
};

// Weight fragments of one wave, resident in registers for the whole kernel.
// Layer 1 carries its bias as an extra input column (index Q, fed by a
// constant 1 in the input), layers 2 and 3 start their accumulators at the
// bias.  For bf16 / fp16 the two tanh layers (weights, layer-1 bias column
// and b2) are scaled by c = 2 log2(e) before rounding, see tanh4.
template <int P, class S>
struct Weights {
  using F = typename Frag<P>::T;
  F w1[S::HB][S::KX];
  F w2[S::HB][S::HB];
  F w3[S::QB][S::HB];
  f4 b2[S::HB];
  f4 b3[S::QB];

  // b2 and b3 from theta (independent of the staging, so their reads can
  // be in flight while it runs)
  __device__ inline void load_biases(const float* __restrict__ th) {
    const int g = (threadIdx.x & 63) >> 4;
    constexpr float sc = tanh_weight_scale<P>();
#pragma unroll
    for (int ob = 0; ob < S::HB; ++ob)
#pragma unroll
      for (int r = 0; r < 4; ++r) b2[ob][r] = sc * th[S::ob2 + 16 * ob + 4 * g + r];
#pragma unroll
    for (int ob = 0; ob < S::QB; ++ob)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int q = 16 * ob + 4 * g + r;
        b3[ob][r] = q < S::Q ? th[S::ob3 + q] : 0.f;
      }
  }

  // the weight fragments, from those staged in LDS (stage_weight_fragments)
  __device__ inline void load_staged(const F* fr) {
    const int l = threadIdx.x & 63;
    constexpr int N1 = S::HB * S::KX, N2 = S::HB * S::HB;
#pragma unroll
    for (int ob = 0; ob < S::HB; ++ob) {
#pragma unroll
      for (int c = 0; c < S::KX; ++c) w1[ob][c] = fr[64 * (ob * S::KX + c) + l];
#pragma unroll
      for (int c = 0; c < S::HB; ++c) w2[ob][c] = fr[64 * (N1 + ob * S::HB + c) + l];
    }
#pragma unroll
    for (int ob = 0; ob < S::QB; ++ob)
#pragma unroll
      for (int c = 0; c < S::HB; ++c) w3[ob][c] = fr[64 * (N1 + N2 + ob * S::HB + c) + l];
  }

  // lane-local A-operand entry: row o, k = 16 c + 4 g + r
  __device__ inline void load(const float* __restrict__ th) {
    const int l = threadIdx.x & 63, g = l >> 4, i = l & 15;
    constexpr float sc = tanh_weight_scale<P>();
#pragma unroll
    for (int ob = 0; ob < S::HB; ++ob) {
      const int o = 16 * ob + i;
#pragma unroll
      for (int c = 0; c < S::KX; ++c) {
        f4 v;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int k = 16 * c + 4 * g + r;
          v[r] = sc * (k < S::Q ? th[S::oW1 + o * S::Q + k] : (k == S::Q ? th[S::ob1 + o] : 0.f));
        }
        w1[ob][c] = to_frag<P>(v);
      }
#pragma unroll
      for (int c = 0; c < S::HB; ++c) {
        f4 v;
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = sc * th[S::oW2 + o * S::H + 16 * c + 4 * g + r];
        w2[ob][c] = to_frag<P>(v);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) b2[ob][r] = sc * th[S::ob2 + 16 * ob + 4 * g + r];
    }
#pragma unroll
    for (int ob = 0; ob < S::QB; ++ob) {
      const int o = 16 * ob + i;
#pragma unroll
      for (int c = 0; c < S::HB; ++c) {
        f4 v;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          v[r] = o < S::Q ? th[S::oW3 + o * S::H + 16 * c + 4 * g + r] : 0.f;
        w3[ob][c] = to_frag<P>(v);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int q = 16 * ob + 4 * g + r;
        b3[ob][r] = q < S::Q ? th[S::ob3 + q] : 0.f;
      }
    }
  }
};

// Block-cooperative staging of the fragments Weights::load builds, into a
// fragment-major LDS array fr (fragment f of lane l at fr[64 f + l]): W1
// with b1 as input column Q (HB x KX fragments), W2 (HB x HB), W3 (QB x HB),
// the two tanh layers scaled.  The NT threads of the workgroup read theta
// once, consecutive threads on consecutive parameters, all reads issued
// before any is used; every value is then stored at its fragment position.
// The padding entries are zero.  Ends with a workgroup barrier.
template <int P, class S, int NT>
__device__ inline void stage_weight_fragments(typename Frag<P>::T* fr,
                                              const float* __restrict__ th) {
  using F = typename Frag<P>::T;
  constexpr int N1 = S::HB * S::KX, N2 = S::HB * S::HB, N3 = S::QB * S::HB;
  constexpr int NF = N1 + N2 + N3;
  constexpr float sc = tanh_weight_scale<P>();
  constexpr int C1 = (S::H * S::Q + NT - 1) / NT, CB = (S::H + NT - 1) / NT,
                C2 = (S::H * S::H + NT - 1) / NT, C3 = (S::Q * S::H + NT - 1) / NT;
  const int tid = threadIdx.x;
  float v1[C1], vb[CB], v2[C2], v3[C3];
#pragma unroll
  for (int i = 0; i < C1; ++i) {
    const int j = tid + i * NT;
    v1[i] = j < S::H * S::Q ? th[S::oW1 + j] : 0.f;
  }
#pragma unroll
  for (int i = 0; i < CB; ++i) {
    const int j = tid + i * NT;
    vb[i] = j < S::H ? th[S::ob1 + j] : 0.f;
  }
#pragma unroll
  for (int i = 0; i < C2; ++i) {
    const int j = tid + i * NT;
    v2[i] = j < S::H * S::H ? th[S::oW2 + j] : 0.f;
  }
#pragma unroll
  for (int i = 0; i < C3; ++i) {
    const int j = tid + i * NT;
    v3[i] = j < S::Q * S::H ? th[S::oW3 + j] : 0.f;
  }
  for (int e = tid; e < NF * 64; e += NT) fr[e] = F{};
  __syncthreads();
  // element r of fragment f, lane l; l = row % 16 + 16 ((k % 16) / 4), r = k % 4
  auto put = [&](int f, int row, int k, float v) {
    const int e = 64 * f + (row & 15) + 16 * ((k & 15) >> 2);
    if constexpr (P == P_F32) {
      reinterpret_cast<float*>(fr)[4 * e + (k & 3)] = v;
    } else {
      const unsigned w = pack2<P>(v, 0.f);
      reinterpret_cast<unsigned short*>(fr)[4 * e + (k & 3)] = (unsigned short)w;
    }
  };
#pragma unroll
  for (int i = 0; i < C1; ++i) {
    const int j = tid + i * NT, o = j / S::Q, k = j - o * S::Q;
    if (j < S::H * S::Q) put((o >> 4) * S::KX + (k >> 4), o, k, sc * v1[i]);
  }
#pragma unroll
  for (int i = 0; i < CB; ++i) {
    const int o = tid + i * NT;
    if (o < S::H) put((o >> 4) * S::KX + (S::Q >> 4), o, S::Q, sc * vb[i]);
  }
#pragma unroll
  for (int i = 0; i < C2; ++i) {
    const int j = tid + i * NT, o = j / S::H, k = j - o * S::H;
    if (j < S::H * S::H) put(N1 + (o >> 4) * S::HB + (k >> 4), o, k, sc * v2[i]);
  }
#pragma unroll
  for (int i = 0; i < C3; ++i) {
    const int j = tid + i * NT, q = j / S::H, k = j - q * S::H;
    if (j < S::Q * S::H) put(N1 + N2 + (q >> 4) * S::HB + (k >> 4), q, k, v3[i]);
  }
  __syncthreads();
}

}  // namespace lbm
