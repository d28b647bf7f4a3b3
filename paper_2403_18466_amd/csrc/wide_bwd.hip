// wide_bwd.hip -- host sequence of the wide network's adjoint (wide_bwd.hpp).
#include <hip/hip_runtime.h>

#include "wide_bwd.hpp"

namespace lbm {

namespace {

struct WsLayout {
  long long Np;         // nodes padded to a multiple of 64
  int nsplit;           // K ranges of the weight-gradient products
  long long kc;         // nodes per range
  size_t X0, X0t, H1, H1t, H2, H2t, H3, H3t, dY, dYt, dZ3, dZ3t, dZ2, dZ2t, dZ1, dZ1t;
  size_t dX0, part, total;
};

template <int Q>
WsLayout ws_layout(long long nodes, size_t es) {
  using W = WideBwd<Q>;
  WsLayout l;
  l.Np = (nodes + 63) / 64 * 64;
  long long ns = l.Np / 512;
  if (ns < 1) ns = 1;
  if (ns > 128) ns = 128;
  l.kc = ((l.Np + ns - 1) / ns + 31) / 32 * 32;
  l.nsplit = (int)((l.Np + l.kc - 1) / l.kc);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += (bytes + 255) / 256 * 256;
    return at;
  };
  const size_t N = (size_t)l.Np;
  l.X0 = take(N * W::D0 * es);
  l.X0t = take(N * W::D0 * es);
  l.H1 = take(N * W::D1 * es);
  l.H1t = take(N * W::D1 * es);
  l.H2 = take(N * W::D2 * es);
  l.H2t = take(N * W::D2 * es);
  l.H3 = take(N * W::D3 * es);
  l.H3t = take(N * W::D3 * es);
  l.dY = take(N * W::D4 * es);
  l.dYt = take(N * W::D4 * es);
  l.dZ3 = take(N * W::D3 * es);
  l.dZ3t = take(N * W::D3 * es);
  l.dZ2 = take(N * W::D2 * es);
  l.dZ2t = take(N * W::D2 * es);
  l.dZ1 = take(N * W::D1 * es);
  l.dZ1t = take(N * W::D1 * es);
  l.dX0 = take(N * W::D0 * sizeof(float));
  l.part = take((size_t)l.nsplit * W::ngrad * sizeof(float));
  l.total = o;
  return l;
}

template <int P, int EPI>
hipError_t gemm(hipStream_t s, const GemmArgs& a, long long M, int N, int splits) {
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)splits);
  if constexpr (P == P_F32)
    hipLaunchKernelGGL((gemm_nt_kernel<P, EPI>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((gemm_nt16_kernel<P, EPI>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

GemmArgs args(const void* A, long long lda, const void* B, long long ldb, int M, int N,
              long long K, void* C, long long ldc) {
  GemmArgs a{};
  a.A = A;
  a.B = B;
  a.lda = lda;
  a.ldb = ldb;
  a.M = M;
  a.N = N;
  a.K = K;
  a.kc = K;
  a.C = C;
  a.ldc = ldc;
  return a;
}

#define WB_CHECK(x)                  \
  do {                               \
    hipError_t e_ = (x);             \
    if (e_ != hipSuccess) return e_; \
  } while (0)

template <class L, int P>
hipError_t run(hipStream_t s, const float* A, const float* theta, const float* lam1, float* lam0,
               float* dtheta, void* ws, const int* idx, unsigned char* packed, Grid G, Force Fc,
               float rho0, float omega, float knn) {
  using W = WideBwd<L::Q>;
  using T = typename OpT<P>::T;
  const long long nodes = (long long)G.plane * G.batch;
  const WsLayout l = ws_layout<L::Q>(nodes, sizeof(T));
  unsigned char* base = static_cast<unsigned char*>(ws);
  auto at = [&](size_t off) { return reinterpret_cast<T*>(base + off); };
  const T* Wp = reinterpret_cast<const T*>(packed);
  const float* vec = reinterpret_cast<const float*>(packed + (size_t)W::nw * sizeof(T));
  const unsigned nb_nodes = (unsigned)((l.Np + 255) / 256);

  hipLaunchKernelGGL(wide_bwd_pack_kernel<P>, dim3((W::nw + W::nb + 255) / 256), dim3(256), 0, s,
                     theta, idx, packed, W::nw, W::nb);
  WB_CHECK(hipGetLastError());
  hipLaunchKernelGGL((wide_prep_kernel<L, P>), dim3(nb_nodes), dim3(256), 0, s, A, G, l.Np,
                     at(l.X0), at(l.X0t));
  WB_CHECK(hipGetLastError());
  const int M = (int)l.Np;
  // forward recompute of the hidden layers
  {
    GemmArgs a = args(at(l.X0), W::D0, Wp + W::oW1, W::D0, M, W::D1, W::D0, at(l.H1), W::D1);
    a.Ct = at(l.H1t);
    a.ldct = l.Np;
    a.bias = vec + W::fE1;
    WB_CHECK((gemm<P, EPI_LEAKY>(s, a, M, W::D1, 1)));
  }
  {
    GemmArgs a = args(at(l.H1), W::D1, Wp + W::oW2, W::D1, M, W::D2, W::D1, at(l.H2), W::D2);
    a.Ct = at(l.H2t);
    a.ldct = l.Np;
    a.bias = vec + W::fB2;
    WB_CHECK((gemm<P, EPI_LEAKY>(s, a, M, W::D2, 1)));
  }
  {
    GemmArgs a = args(at(l.H2), W::D2, Wp + W::oW3, W::D2, M, W::D3, W::D2, at(l.H3), W::D3);
    a.Ct = at(l.H3t);
    a.ldct = l.Np;
    a.bias = vec + W::fB3;
    WB_CHECK((gemm<P, EPI_LEAKY>(s, a, M, W::D3, 1)));
  }
  hipLaunchKernelGGL((wide_dy_kernel<L, P>), dim3(nb_nodes), dim3(256), 0, s, A, lam1, G, Fc, rho0,
                     omega, knn, l.Np, at(l.dY), at(l.dYt));
  WB_CHECK(hipGetLastError());
  // input gradients of the layers, masked by the LeakyReLU derivative
  {
    GemmArgs a = args(at(l.dY), W::D4, Wp + W::oT4, W::D4, M, W::D3, W::D4, at(l.dZ3), W::D3);
    a.Ct = at(l.dZ3t);
    a.ldct = l.Np;
    a.mask = at(l.H3);
    WB_CHECK((gemm<P, EPI_MASK>(s, a, M, W::D3, 1)));
  }
  {
    GemmArgs a = args(at(l.dZ3), W::D3, Wp + W::oT3, W::D3, M, W::D2, W::D3, at(l.dZ2), W::D2);
    a.Ct = at(l.dZ2t);
    a.ldct = l.Np;
    a.mask = at(l.H2);
    WB_CHECK((gemm<P, EPI_MASK>(s, a, M, W::D2, 1)));
  }
  {
    GemmArgs a = args(at(l.dZ2), W::D2, Wp + W::oT2, W::D2, M, W::D1, W::D2, at(l.dZ1), W::D1);
    a.Ct = at(l.dZ1t);
    a.ldct = l.Np;
    a.mask = at(l.H1);
    WB_CHECK((gemm<P, EPI_MASK>(s, a, M, W::D1, 1)));
  }
  float* dX0 = reinterpret_cast<float*>(base + l.dX0);
  {
    GemmArgs a = args(at(l.dZ1), W::D1, Wp + W::oT1, W::D1, M, W::D0, W::D1, dX0, W::D0);
    WB_CHECK((gemm<P, EPI_F32>(s, a, M, W::D0, 1)));
  }
  // weight gradients: contractions over the nodes, one slab per node range
  float* part = reinterpret_cast<float*>(base + l.part);
  struct Wg {
    size_t a, b;
    int m, n, off;
  } wg[4] = {{l.dYt, l.H3t, W::D4, W::D3, W::gW4},
             {l.dZ3t, l.H2t, W::D3, W::D2, W::gW3},
             {l.dZ2t, l.H1t, W::D2, W::D1, W::gW2},
             {l.dZ1t, l.X0t, W::D1, W::D0, W::gW1}};
  for (const Wg& w : wg) {
    GemmArgs a = args(at(w.a), l.Np, at(w.b), l.Np, w.m, w.n, l.Np, part + w.off, w.n);
    a.kc = l.kc;
    a.slab = W::ngrad;
    WB_CHECK((gemm<P, EPI_PARTIAL>(s, a, w.m, w.n, l.nsplit)));
  }
  hipLaunchKernelGGL(wide_grad_reduce_kernel<L::Q>, dim3((W::nparam + 255) / 256), dim3(256), 0,
                     s, part, l.nsplit, dtheta);
  WB_CHECK(hipGetLastError());
  hipLaunchKernelGGL(wide_post_kernel<L>, dim3((unsigned)((nodes + 255) / 256)), dim3(256), 0, s,
                     A, lam1, dX0, lam0, G, Fc, rho0, omega);
  return hipGetLastError();
}

template <class L>
hipError_t run_prec(int prec, hipStream_t s, const float* A, const float* theta, const float* lam1,
                    float* lam0, float* dtheta, void* ws, const int* idx, unsigned char* packed,
                    Grid G, Force Fc, float rho0, float omega, float knn) {
  switch (prec) {
    case P_F32: return run<L, P_F32>(s, A, theta, lam1, lam0, dtheta, ws, idx, packed, G, Fc, rho0, omega, knn);
    case P_BF16: return run<L, P_BF16>(s, A, theta, lam1, lam0, dtheta, ws, idx, packed, G, Fc, rho0, omega, knn);
    default: return run<L, P_F16>(s, A, theta, lam1, lam0, dtheta, ws, idx, packed, G, Fc, rho0, omega, knn);
  }
}

}  // namespace

size_t wide_bwd_workspace_bytes(bool d3q19, int prec, long long nodes) {
  const size_t es = prec == P_F32 ? 4 : 2;
  return d3q19 ? ws_layout<19>(nodes, es).total : ws_layout<9>(nodes, es).total;
}

hipError_t wide_bwd_launch(bool d3q19, int prec, hipStream_t s, const float* A,
                           const float* theta, const float* lam1, float* lam0, float* dtheta,
                           void* ws, const int* idx, unsigned char* packed, Grid G, Force Fc,
                           float rho0, float omega, float knn) {
  if (d3q19)
    return run_prec<D3Q19>(prec, s, A, theta, lam1, lam0, dtheta, ws, idx, packed, G, Fc, rho0, omega, knn);
  return run_prec<D2Q9>(prec, s, A, theta, lam1, lam0, dtheta, ws, idx, packed, G, Fc, rho0, omega, knn);
}

}  // namespace lbm
