// wide.hip -- instances and launches of the wide-network kernels (wide.hpp).
// A translation unit of its own so that it can be compiled with the
// instruction scheduler that keeps the weight-fragment reads from LDS ahead
// of the matrix-core instructions that consume them (max-ILP): the default,
// occupancy-first scheduler serialises every read with its two MFMAs.
#include <hip/hip_runtime.h>

#include "wide.hpp"

namespace lbm {

namespace {

template <class L, int P>
hipError_t step_one(unsigned nb, hipStream_t s, const float* Ain, float* Aout,
                    const unsigned char* packed, Grid G, Force Fc, float rho0, float omega,
                    float knn, int per, int nitems, int nxc) {
  hipLaunchKernelGGL((wide_step_kernel<L, P>), dim3(nb), dim3(WideCfg<L, P>::THREADS), 0, s, Ain,
                     Aout, packed, G, Fc, rho0, omega, knn, per, nitems, nxc);
  return hipGetLastError();
}

template <class L>
hipError_t step_prec(int prec, unsigned nb, hipStream_t s, const float* Ain, float* Aout,
                     const unsigned char* packed, Grid G, Force Fc, float rho0, float omega,
                     float knn, int per, int nitems, int nxc) {
  switch (prec) {
    case P_F32: return step_one<L, P_F32>(nb, s, Ain, Aout, packed, G, Fc, rho0, omega, knn, per, nitems, nxc);
    case P_BF16: return step_one<L, P_BF16>(nb, s, Ain, Aout, packed, G, Fc, rho0, omega, knn, per, nitems, nxc);
    default: return step_one<L, P_F16>(nb, s, Ain, Aout, packed, G, Fc, rho0, omega, knn, per, nitems, nxc);
  }
}

}  // namespace

hipError_t wide_step_launch(bool d3q19, int prec, unsigned nb, hipStream_t s, const float* Ain,
                            float* Aout, const unsigned char* packed, Grid G, Force Fc,
                            float rho0, float omega, float knn, int per, int nitems, int nxc) {
  if (d3q19)
    return step_prec<D3Q19>(prec, nb, s, Ain, Aout, packed, G, Fc, rho0, omega, knn, per, nitems, nxc);
  return step_prec<D2Q9>(prec, nb, s, Ain, Aout, packed, G, Fc, rho0, omega, knn, per, nitems, nxc);
}

hipError_t wide_pack_launch(int prec, unsigned blocks, hipStream_t s, const float* theta,
                            const int* idx, unsigned char* packed, int nw, int nb) {
  switch (prec) {
    case P_F32:
      hipLaunchKernelGGL(wide_pack_kernel<P_F32>, dim3(blocks), dim3(256), 0, s, theta, idx, packed, nw, nb);
      break;
    case P_BF16:
      hipLaunchKernelGGL(wide_pack_kernel<P_BF16>, dim3(blocks), dim3(256), 0, s, theta, idx, packed, nw, nb);
      break;
    default:
      hipLaunchKernelGGL(wide_pack_kernel<P_F16>, dim3(blocks), dim3(256), 0, s, theta, idx, packed, nw, nb);
  }
  return hipGetLastError();
}

}  // namespace lbm
