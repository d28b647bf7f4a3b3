// nlbm_bwd_d2q9.hip -- the D2Q9 instances of the learned-collision adjoint
// kernel (kernels_bwd.hpp), in a translation unit of their own so that they
// can be built with the max-ILP instruction scheduler (the D3Q19 instances
// run slower with it).
#include <hip/hip_runtime.h>

#include "kernels_bwd.hpp"

namespace lbm {

hipError_t nlbm_bwd_launch_d2q9(int hidden, int prec, unsigned blocks, hipStream_t s,
                                const float* A, const float* theta, const float* lam1,
                                float* lam0, float* part, Grid G, Force Fc, float rho0,
                                float omega, float knn, int nitems, int nxc, int accum) {
  return bwd_detail::bwd_hidden<D2Q9>(hidden, prec, blocks, s, A, theta, lam1, lam0, part, G, Fc,
                                      rho0, omega, knn, nitems, nxc, accum);
}

}  // namespace lbm
