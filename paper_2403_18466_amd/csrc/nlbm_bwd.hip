// nlbm_bwd.hip -- the D3Q19 instances and the launch of the learned-collision
// adjoint kernel (kernels_bwd.hpp), in a translation unit of their own (the
// adjoint instances are the largest kernels of the library; they compile in
// parallel with the rest).  The D2Q9 instances are in nlbm_bwd_d2q9.hip.
#include <hip/hip_runtime.h>

#include "kernels_bwd.hpp"

namespace lbm {

hipError_t nlbm_bwd_launch(bool d3q19, int hidden, int prec, unsigned blocks, hipStream_t s,
                           const float* A, const float* theta, const float* lam1, float* lam0,
                           float* part, Grid G, Force Fc, float rho0, float omega, float knn,
                           int nitems, int nxc, int accum) {
  if (d3q19)
    return bwd_detail::bwd_hidden<D3Q19>(hidden, prec, blocks, s, A, theta, lam1, lam0, part, G,
                                         Fc, rho0, omega, knn, nitems, nxc, accum);
  return nlbm_bwd_launch_d2q9(hidden, prec, blocks, s, A, theta, lam1, lam0, part, G, Fc, rho0,
                              omega, knn, nitems, nxc, accum);
}

}  // namespace lbm
