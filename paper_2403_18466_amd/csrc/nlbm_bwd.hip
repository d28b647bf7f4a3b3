// nlbm_bwd.hip -- instances and launch of the learned-collision adjoint
// kernel (kernels_bwd.hpp), in a translation unit of its own (the twelve
// instances are the largest kernels of the library; they compile in parallel
// with the rest).
#include <hip/hip_runtime.h>

#include "kernels_bwd.hpp"

namespace lbm {

namespace {

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

}  // namespace

hipError_t nlbm_bwd_launch(bool d3q19, int hidden, int prec, unsigned blocks, hipStream_t s,
                           const float* A, const float* theta, const float* lam1, float* lam0,
                           float* part, Grid G, Force Fc, float rho0, float omega, float knn,
                           int nitems, int nxc, int accum) {
  if (d3q19)
    return bwd_hidden<D3Q19>(hidden, prec, blocks, s, A, theta, lam1, lam0, part, G, Fc, rho0,
                             omega, knn, nitems, nxc, accum);
  return bwd_hidden<D2Q9>(hidden, prec, blocks, s, A, theta, lam1, lam0, part, G, Fc, rho0, omega,
                          knn, nitems, nxc, accum);
}

}  // namespace lbm
