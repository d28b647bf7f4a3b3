// nlbm_fwd.hip -- instances and launch of the learned-collision step kernel
// (kernels_fwd.hpp), in a translation unit of its own: it is built with the
// max-ILP instruction scheduler, which the library's other kernels do not
// take (several of them need more registers with it).
#include <hip/hip_runtime.h>

#include "kernels_fwd.hpp"

namespace lbm {

namespace {

template <class L, int H, int P, bool FORCED>
hipError_t fwd_one(int ncu, hipStream_t s, const float* Ain, float* Aout, const float* theta,
                   Grid G, Force Fc, float rho0, float omega, float knn, int nitems, int nxc) {
  const auto kernel = nlbm_step_kernel<L, H, P, FORCED>;
  constexpr int wb = StepLds<L, H>::waves_per_block(P, FORCED);
  int occ = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, 64 * wb, 0);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kernel, dim3(persistent_grid(ncu, occ, wb, nitems)), dim3(64 * wb), 0, s,
                     Ain, Aout, theta, G, Fc, rho0, omega, knn, nitems, nxc);
  return hipGetLastError();
}

template <class L, int H, int P>
hipError_t fwd_forced(bool forced, int ncu, hipStream_t s, const float* Ain, float* Aout,
                      const float* theta, Grid G, Force Fc, float rho0, float omega, float knn,
                      int nitems, int nxc) {
  // forced and unforced instances: the unforced one needs fewer registers
  if (forced)
    return fwd_one<L, H, P, true>(ncu, s, Ain, Aout, theta, G, Fc, rho0, omega, knn, nitems, nxc);
  return fwd_one<L, H, P, false>(ncu, s, Ain, Aout, theta, G, Fc, rho0, omega, knn, nitems, nxc);
}

template <class L, int H>
hipError_t fwd_prec(int prec, bool forced, int ncu, hipStream_t s, const float* Ain, float* Aout,
                    const float* theta, Grid G, Force Fc, float rho0, float omega, float knn,
                    int nitems, int nxc) {
  switch (prec) {
    case P_F32:
      return fwd_forced<L, H, P_F32>(forced, ncu, s, Ain, Aout, theta, G, Fc, rho0, omega, knn, nitems, nxc);
    case P_BF16:
      return fwd_forced<L, H, P_BF16>(forced, ncu, s, Ain, Aout, theta, G, Fc, rho0, omega, knn, nitems, nxc);
    default:
      return fwd_forced<L, H, P_F16>(forced, ncu, s, Ain, Aout, theta, G, Fc, rho0, omega, knn, nitems, nxc);
  }
}

template <class L>
hipError_t fwd_hidden(int hidden, int prec, bool forced, int ncu, hipStream_t s,
                      const float* Ain, float* Aout, const float* theta, Grid G, Force Fc,
                      float rho0, float omega, float knn, int nitems, int nxc) {
  if (hidden == 32)
    return fwd_prec<L, 32>(prec, forced, ncu, s, Ain, Aout, theta, G, Fc, rho0, omega, knn, nitems, nxc);
  return fwd_prec<L, 64>(prec, forced, ncu, s, Ain, Aout, theta, G, Fc, rho0, omega, knn, nitems, nxc);
}

}  // namespace

hipError_t nlbm_fwd_launch(bool d3q19, int hidden, int prec, bool forced, int ncu, hipStream_t s,
                           const float* Ain, float* Aout, const float* theta, Grid G, Force Fc,
                           float rho0, float omega, float knn, int nitems, int nxc) {
  if (d3q19)
    return fwd_hidden<D3Q19>(hidden, prec, forced, ncu, s, Ain, Aout, theta, G, Fc, rho0, omega,
                             knn, nitems, nxc);
  return fwd_hidden<D2Q9>(hidden, prec, forced, ncu, s, Ain, Aout, theta, G, Fc, rho0, omega, knn,
                          nitems, nxc);
}

}  // namespace lbm
