// lbm_api.hip -- host implementation of the C ABI declared in include/lbm.h:
// argument validation, dispatch to the kernel instances and launches on the
// caller's stream.  No exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <string>

#include "kernels_aux.hpp"
#include "kernels_bwd.hpp"
#include "kernels_diag.hpp"
#include "kernels_fwd.hpp"
#include "kernels_ref.hpp"
#include "lbm.h"
#include "wide.hpp"
#include "wide_bwd.hpp"

#include <vector>

using namespace lbm;

// Scratch of lbm_step_backward_static: the adjoint's per-workgroup partial
// parameter gradients, in memory the library holds on every device it runs
// on until the process ends.  Host code never uses this name as a device
// address: lbm_create looks up each device's address of it once, with the
// device current, and the calls pass that address to the kernels.
constexpr size_t kStaticScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

struct lbm_ctx {
  lbm_config cfg;
  int device;
  int ncu;
  void* scratch;  // this device's address of `scratch` (null if the lookup failed)
  double* partial;  // float64 reduction partials, [batch][max(MOM_BLOCKS, MOMENT_BLOCKS)][3]
  // LBM_NET_LEAKY_300_300_100: theta -> fragment-order gather table and the
  // packed weights it fills
  int* wide_idx;
  unsigned char* wide_packed;
  int wide_nw, wide_nb;
  // its adjoint: gather table and packed padded W, W^T and bias vectors
  int* wide_bidx;
  unsigned char* wide_bpacked;
  // partial sums of the moment-space analysis (D3Q19 contexts)
  double* mrt;
  // body force tables F_x(y), F_y(z), F_z(x) (float32, from float64 on the host)
  float* force_tab;
};

namespace {

thread_local std::string g_err;

lbm_status fail(lbm_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define LBM_HIP(expr)                                                               \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) return fail(LBM_ERR_HIP, std::string(#expr) + ": " +      \
                                                       hipGetErrorString(e_));      \
  } while (0)

#define LBM_LAUNCHED(name)                                                          \
  do {                                                                              \
    hipError_t e_ = hipGetLastError();                                              \
    if (e_ != hipSuccess)                                                           \
      return fail(LBM_ERR_HIP, std::string("launch of ") + name + ": " +            \
                                   hipGetErrorString(e_));                          \
  } while (0)

int lattice_q(int lat) { return lat == LBM_D2Q9 ? 9 : 19; }
int lattice_d(int lat) { return lat == LBM_D2Q9 ? 2 : 3; }

Grid grid_of(const lbm_config& c) {
  Grid G;
  G.nx = c.nx;
  G.ny = c.ny;
  G.nz = c.nz;
  G.batch = c.batch;
  G.plane = c.nx * c.ny * c.nz;
  return G;
}

Force force_of(const lbm_ctx* ctx) {
  const lbm_config& c = ctx->cfg;
  Force f;
  f.kind = c.force_kind;
  f.fx_y = ctx->force_tab;
  f.fy_z = ctx->force_tab ? ctx->force_tab + c.ny : nullptr;
  f.fz_x = ctx->force_tab ? ctx->force_tab + c.ny + c.nz : nullptr;
  return f;
}

// amp sin(2 pi k s / n) for s = 0 .. n - 1, the argument reduced exactly in
// integers, in float64, rounded once to float32.
void force_table(double amp, int k, int n, float* out) {
  const double two_pi = 6.283185307179586476925286766559;
  for (int s = 0; s < n; ++s) {
    long long r = ((long long)k * s) % n;
    if (r < 0) r += n;
    out[s] = (float)(amp * std::sin(two_pi * (double)r / (double)n));
  }
}

size_t param_count(int lat, int H, int net) {
  if (H <= 0) return 0;
  if (net == LBM_NET_LEAKY_300_300_100)
    return lat == LBM_D2Q9 ? (size_t)WideLayout<9, P_BF16>::nparam
                           : (size_t)WideLayout<19, P_BF16>::nparam;
  size_t Q = (size_t)lattice_q(lat), h = (size_t)H;
  return h * Q + h + h * h + h + Q * h + Q;
}

size_t param_count(const lbm_config& c) { return param_count(c.lattice, c.hidden, c.net); }

// Gather table of the packed wide-network weights: entry e of the packed
// buffer takes theta[idx[e]] (0 where idx[e] < 0).  Follows the fragment
// layout described in wide.hpp.
template <int Q, int P>
std::vector<int> wide_index() {
  using WL = WideLayout<Q, P>;
  const int nw = WL::weight_bytes / WL::EB;
  std::vector<int> idx((size_t)nw + WL::nbias, -1);
  // units of tile t over K chunks [c0, c0 + kc), starting at byte offset off
  auto emit = [&](int off, int t, int c0, int kc, auto value) {
    for (int c = 0; c < kc; c += 2) {
      const int nc = c + 1 < kc ? 2 : 1;
      const int unit = off + c * WL::CHUNK;
      for (int l = 0; l < 64; ++l)
        for (int j = 0; j < nc; ++j)
          for (int r = 0; r < 4; ++r) {
            const int o = 16 * t + (l & 15), k = 16 * (c0 + c + j) + 4 * (l >> 4) + r;
            const int e = (unit + l * nc * 4 * WL::EB + (4 * j + r) * WL::EB) / WL::EB;
            idx[(size_t)e] = value(o, k);
          }
    }
  };
  auto v1 = [](int o, int k) {
    if (o >= WL::N1) return -1;
    return k < Q ? WL::oW1 + o * Q + k : (k == Q ? WL::ob1 + o : -1);
  };
  auto v2 = [](int o, int k) { return o < WL::N2 && k < WL::N1 ? WL::oW2 + o * WL::N1 + k : -1; };
  auto v3 = [](int o, int k) { return o < WL::N3 && k < WL::N2 ? WL::oW3 + o * WL::N2 + k : -1; };
  auto v4 = [](int o, int k) { return o < Q && k < WL::N3 ? WL::oW4 + o * WL::N3 + k : -1; };
  for (int t = 0; t < WL::T1; ++t)
    emit(WL::step_offset(t / WL::TP1) + (t % WL::TP1) * WL::K1 * WL::CHUNK, t, 0, WL::K1, v1);
  for (int g = 0; g < WL::NG; ++g) {
    const int off = WL::step_offset(WL::S1 + g), gt = WL::group_tiles(g);
    for (int j = 0; j < gt; ++j)
      emit(off + j * WL::K2 * WL::CHUNK, g * WL::RG + j, 0, WL::K2, v2);
    for (int t3 = 0; t3 < WL::T3; ++t3)
      emit(off + gt * WL::K2 * WL::CHUNK + t3 * gt * WL::CHUNK, t3, g * WL::RG, gt, v3);
  }
  for (int t4 = 0; t4 < WL::T4; ++t4)
    emit(WL::step_offset(WL::NSTEP - 1) + t4 * WL::K4 * WL::CHUNK, t4, 0, WL::K4, v4);
  int* b = idx.data() + nw;
  for (int i = 0; i < 16 * WL::T2; ++i) b[WL::fb2 + i] = i < WL::N2 ? WL::ob2 + i : -1;
  for (int i = 0; i < 16 * WL::T3; ++i) b[WL::fb3 + i] = i < WL::N3 ? WL::ob3 + i : -1;
  for (int i = 0; i < 16 * WL::T4; ++i) b[WL::fb4 + i] = i < Q ? WL::ob4 + i : -1;
  return idx;
}

// Gather table of the adjoint's padded matrices (see WideBwd): -1 is 0, -2
// is the constant 1 of the padded bias columns.
template <int Q>
std::vector<int> wide_bwd_index() {
  using W = WideBwd<Q>;
  std::vector<int> idx((size_t)W::nw + W::nb, -1);
  for (int o = 0; o < W::D1; ++o)
    for (int k = 0; k < W::D0; ++k) {
      const int v = o < W::N1 ? (k < Q ? W::pW1 + o * Q + k : (k == Q ? W::pb1 + o : -1)) : -1;
      idx[W::oW1 + o * W::D0 + k] = v;
      idx[W::oT1 + k * W::D1 + o] = v;
    }
  for (int o = 0; o < W::D2; ++o)
    for (int k = 0; k < W::D1; ++k) {
      const int v = o < W::N2 && k < W::N1 ? W::pW2 + o * W::N1 + k : -1;
      idx[W::oW2 + o * W::D1 + k] = v;
      idx[W::oT2 + k * W::D2 + o] = v;
    }
  for (int o = 0; o < W::D3; ++o)
    for (int k = 0; k < W::D2; ++k) {
      const int v = o < W::N3 && k < W::N2 ? W::pW3 + o * W::N2 + k : -1;
      idx[W::oW3 + o * W::D2 + k] = v;
      idx[W::oT3 + k * W::D3 + o] = v;
    }
  for (int o = 0; o < W::D4; ++o)
    for (int k = 0; k < W::D3; ++k) {
      const int v = o < Q && k < W::N3 ? W::pW4 + o * W::N3 + k : -1;
      idx[W::oW4 + o * W::D3 + k] = v;
      idx[W::oT4 + k * W::D4 + o] = v;
    }
  int* v = idx.data() + W::nw;
  for (int j = 0; j < W::D1; ++j) v[W::fE1 + j] = j == W::ONE1 ? -2 : -1;
  for (int j = 0; j < W::D2; ++j) v[W::fB2 + j] = j < W::N2 ? W::pb2 + j : (j == W::ONE1 ? -2 : -1);
  for (int j = 0; j < W::D3; ++j) v[W::fB3 + j] = j < W::N3 ? W::pb3 + j : (j == W::ONE3 ? -2 : -1);
  return idx;
}

template <int Q>
std::vector<int> wide_index_p(int prec, int& packed_bytes) {
  if (prec == LBM_MLP_FP32) {
    packed_bytes = WideLayout<Q, P_F32>::packed_bytes;
    return wide_index<Q, P_F32>();
  }
  packed_bytes = WideLayout<Q, P_BF16>::packed_bytes;
  return wide_index<Q, P_BF16>();  // bf16 and fp16 share the layout
}

lbm_status validate(const lbm_config* c) {
  if (!c) return fail(LBM_ERR_INVALID, "config is null");
  if (c->lattice != LBM_D2Q9 && c->lattice != LBM_D3Q19)
    return fail(LBM_ERR_INVALID, "lattice must be LBM_D2Q9 or LBM_D3Q19");
  if (c->nx < 1 || c->ny < 1 || c->nz < 1 || c->batch < 1)
    return fail(LBM_ERR_INVALID, "nx, ny, nz and batch must be >= 1");
  if (c->lattice == LBM_D2Q9 && c->nz != 1) return fail(LBM_ERR_INVALID, "D2Q9 needs nz == 1");
  double elems = (double)c->batch * lattice_q(c->lattice) * c->nx * (double)c->ny * c->nz;
  if (elems >= 1073741824.0)
    return fail(LBM_ERR_INVALID, "batch*Q*nx*ny*nz must stay below 2^30 elements (4 GiB)");
  if (!(c->tau > 0.5) || !std::isfinite(c->tau))
    return fail(LBM_ERR_INVALID, "tau must be finite and > 0.5");
  if (!(c->rho0 > 0.0) || !std::isfinite(c->rho0))
    return fail(LBM_ERR_INVALID, "rho0 must be finite and > 0");
  if (c->force_kind < LBM_FORCE_NONE || c->force_kind > LBM_FORCE_SINE3)
    return fail(LBM_ERR_INVALID, "unknown force_kind");
  if (c->force_kind == LBM_FORCE_SINE3 && c->lattice != LBM_D3Q19)
    return fail(LBM_ERR_INVALID, "the three-component sine force needs D3Q19");
  if (c->force_kind != LBM_FORCE_NONE && !std::isfinite(c->force_amp))
    return fail(LBM_ERR_INVALID, "force_amp must be finite");
  if (c->collision != LBM_COLLISION_BGK && c->collision != LBM_COLLISION_SMAGORINSKY)
    return fail(LBM_ERR_INVALID, "collision must be LBM_COLLISION_BGK or LBM_COLLISION_SMAGORINSKY");
  if (c->collision == LBM_COLLISION_SMAGORINSKY) {
    if (c->hidden != 0)
      return fail(LBM_ERR_INVALID, "the Smagorinsky collision takes no network (hidden must be 0)");
    if (!(c->smag_cs >= 0.0) || !std::isfinite(c->smag_cs))
      return fail(LBM_ERR_INVALID, "smag_cs must be finite and >= 0");
  }
  if (c->hidden != 0) {
    if (c->net != LBM_NET_TANH && c->net != LBM_NET_LEAKY_300_300_100)
      return fail(LBM_ERR_INVALID, "net must be LBM_NET_TANH or LBM_NET_LEAKY_300_300_100");
    if (c->net == LBM_NET_TANH && c->hidden != 32 && c->hidden != 64)
      return fail(LBM_ERR_UNSUPPORTED, "hidden must be 0, 32 or 64 for LBM_NET_TANH");
    if (c->net == LBM_NET_LEAKY_300_300_100 && c->hidden != 300)
      return fail(LBM_ERR_INVALID, "hidden must be 300 for LBM_NET_LEAKY_300_300_100");
    if (c->mlp_prec != LBM_MLP_FP32 && c->mlp_prec != LBM_MLP_BF16 &&
        c->mlp_prec != LBM_MLP_FP16)
      return fail(LBM_ERR_INVALID, "mlp_prec must be LBM_MLP_FP32, _BF16 or _FP16");
    if (!std::isfinite(c->out_scale)) return fail(LBM_ERR_INVALID, "out_scale must be finite");
  }
  return LBM_OK;
}

lbm_status check_ctx(const lbm_ctx* ctx) {
  if (!ctx) return fail(LBM_ERR_INVALID, "context is null");
  int dev = -1;
  LBM_HIP(hipGetDevice(&dev));
  if (dev != ctx->device)
    return fail(LBM_ERR_INVALID, "current device differs from the context's device");
  return LBM_OK;
}

// Device address of `scratch` on device dev (current), looked up once per
// device.  On failure the error is recorded and cleared, and null returned.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices];
std::string g_scratch_err[kMaxDevices];

void* static_scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev] && g_scratch_err[dev].empty()) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      g_scratch_err[dev] = std::string("hipGetSymbolAddress of the static scratch: ") +
                           hipGetErrorString(e);
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_addr[dev] = p;
  }
  return g_scratch_addr[dev];
}

unsigned blocks_for(long long n, int per_block = 256) {
  return (unsigned)((n + per_block - 1) / per_block);
}

// ------------------------------------------------------------------ forward
template <class L>
lbm_status run_init(lbm_ctx* ctx, const float* rho, const float* u, float* A, hipStream_t s) {
  Grid G = grid_of(ctx->cfg);
  long long total = (long long)G.plane * G.batch;
  hipLaunchKernelGGL(init_kernel<L>, dim3(blocks_for(total)), dim3(256), 0, s, rho, u, A, G,
                     (float)ctx->cfg.rho0);
  LBM_LAUNCHED("init_kernel");
  return LBM_OK;
}

template <class L>
lbm_status run_shift(lbm_ctx* ctx, const float* src, float* dst, int dir, hipStream_t s) {
  Grid G = grid_of(ctx->cfg);
  long long total = (long long)G.plane * G.batch;
  hipLaunchKernelGGL(shift_kernel<L>, dim3(blocks_for(total)), dim3(256), 0, s, src, dst, G,
                     dir);
  LBM_LAUNCHED("shift_kernel");
  return LBM_OK;
}

template <class L>
lbm_status run_moments(lbm_ctx* ctx, const float* A, float* rho, float* u, double* diag,
                       hipStream_t s) {
  Grid G = grid_of(ctx->cfg);
  const int nxc = (G.nx + 255) / 256;
  hipLaunchKernelGGL(moments_kernel<L>, dim3(MOMENT_BLOCKS, G.batch), dim3(256), 0, s, A, rho, u,
                     ctx->partial, G, (float)ctx->cfg.rho0, force_of(ctx), nxc);
  LBM_LAUNCHED("moments_kernel");
  if (diag) {
    hipLaunchKernelGGL(diag_reduce_kernel, dim3(G.batch), dim3(256), 0, s, ctx->partial, diag,
                       MOMENT_BLOCKS);
    LBM_LAUNCHED("diag_reduce_kernel");
  }
  return LBM_OK;
}

template <class L, int R, bool NT, bool SMAG>
lbm_status launch_bgk_v(lbm_ctx* ctx, const float* Ain, float* Aout, hipStream_t s) {
  Grid G = grid_of(ctx->cfg);
  const lbm_config& c = ctx->cfg;
  int nxc = (G.nx + 255) / 256;
  long long nblk = (long long)nxc * ((G.ny + R - 1) / R) * G.nz * G.batch;
  hipLaunchKernelGGL((bgk_step_kernel<L, R, NT, SMAG>), dim3((unsigned)nblk), dim3(256), 0, s,
                     Ain, Aout, G, force_of(ctx), (float)c.rho0, (float)(1.0 / c.tau), nxc,
                     (float)c.tau, (float)(1.5 / c.tau), (float)(3.0 * c.smag_cs * c.smag_cs));
  LBM_LAUNCHED("bgk_step_kernel");
  return LBM_OK;
}

template <class L>
lbm_status launch_bgk(lbm_ctx* ctx, const float* Ain, float* Aout, hipStream_t s) {
  // one node per thread with non-temporal stores measured fastest for both
  // lattices (D3Q19 256^3: 452 us; two rows per thread 459 us, default
  // stores 474 us)
  if (ctx->cfg.collision == LBM_COLLISION_SMAGORINSKY)
    return launch_bgk_v<L, 1, true, true>(ctx, Ain, Aout, s);
  return launch_bgk_v<L, 1, true, false>(ctx, Ain, Aout, s);
}

int prec_of(int mlp_prec) {
  return mlp_prec == LBM_MLP_FP32 ? P_F32 : (mlp_prec == LBM_MLP_BF16 ? P_BF16 : P_F16);
}

// The learned-collision step: its instances live in nlbm_fwd.hip.
template <class L, int H>
lbm_status launch_nlbm(lbm_ctx* ctx, const float* Ain, float* Aout, const float* theta,
                       hipStream_t s) {
  Grid G = grid_of(ctx->cfg);
  int nxc = (G.nx + 63) / 64;
  long long nitems = (long long)nxc * G.ny * G.nz * G.batch;
  if (nitems >= (1LL << 31)) return fail(LBM_ERR_INVALID, "too many work items");
  const lbm_config& c = ctx->cfg;
  hipError_t e = nlbm_fwd_launch(L::Q == 19, H, prec_of(c.mlp_prec),
                                 c.force_kind != LBM_FORCE_NONE, ctx->ncu, s, Ain, Aout, theta, G,
                                 force_of(ctx), (float)c.rho0, (float)(1.0 / c.tau),
                                 (float)(c.out_scale / c.tau), (int)nitems, nxc);
  if (e != hipSuccess)
    return fail(LBM_ERR_HIP, std::string("launch of nlbm_step_kernel: ") + hipGetErrorString(e));
  return LBM_OK;
}

// The wide network: weights into fragment order, then the persistent step.
lbm_status wide_pack(lbm_ctx* ctx, const float* theta, hipStream_t s) {
  const int n = ctx->wide_nw + ctx->wide_nb;
  hipError_t e = wide_pack_launch(prec_of(ctx->cfg.mlp_prec), blocks_for(n), s, theta,
                                  ctx->wide_idx, ctx->wide_packed, ctx->wide_nw, ctx->wide_nb);
  if (e != hipSuccess)
    return fail(LBM_ERR_HIP, std::string("launch of wide_pack_kernel: ") + hipGetErrorString(e));
  return LBM_OK;
}

template <class L, int P>
lbm_status launch_wide(lbm_ctx* ctx, const float* Ain, float* Aout, hipStream_t s) {
  using C = WideCfg<L, P>;
  Grid G = grid_of(ctx->cfg);
  int nxc = (G.nx + 63) / 64;
  long long nitems = (long long)nxc * G.ny * G.nz * G.batch;
  if (nitems >= (1LL << 31)) return fail(LBM_ERR_INVALID, "too many work items");
  // one workgroup of 8 wavefronts per compute unit (the LDS holds one)
  long long nb = ctx->ncu;
  long long cap = (nitems + C::WAVES - 1) / C::WAVES;
  if (nb > cap) nb = cap;
  if (nb >= 16) nb -= nb % 8;
  const long long per = (nitems + nb * C::WAVES - 1) / (nb * C::WAVES);
  const lbm_config& c = ctx->cfg;
  hipError_t e = wide_step_launch(L::Q == 19, P, (unsigned)nb, s, Ain, Aout, ctx->wide_packed, G,
                                  force_of(ctx), (float)c.rho0, (float)(1.0 / c.tau),
                                  (float)(c.out_scale / c.tau), (int)per, (int)nitems, nxc);
  if (e != hipSuccess)
    return fail(LBM_ERR_HIP, std::string("launch of wide_step_kernel: ") + hipGetErrorString(e));
  return LBM_OK;
}

template <class L>
lbm_status one_step(lbm_ctx* ctx, const float* Ain, float* Aout, const float* theta,
                    hipStream_t s) {
  if (ctx->cfg.net == LBM_NET_LEAKY_300_300_100 && ctx->cfg.hidden != 0) {
    switch (ctx->cfg.mlp_prec) {
      case LBM_MLP_FP32: return launch_wide<L, P_F32>(ctx, Ain, Aout, s);
      case LBM_MLP_BF16: return launch_wide<L, P_BF16>(ctx, Ain, Aout, s);
      default: return launch_wide<L, P_F16>(ctx, Ain, Aout, s);
    }
  }
  switch (ctx->cfg.hidden) {
    case 0: return launch_bgk<L>(ctx, Ain, Aout, s);
    case 32: return launch_nlbm<L, 32>(ctx, Ain, Aout, theta, s);
    default: return launch_nlbm<L, 64>(ctx, Ain, Aout, theta, s);
  }
}

// ----------------------------------------------------------------- backward
// accum: add this step's per-workgroup partials to those in ws instead of
// overwriting them; reduce: sum the partials into dtheta after the step.
template <class L, int H, int P>
lbm_status launch_bwd(lbm_ctx* ctx, const float* A, const float* theta, const float* lam1,
                      float* lam0, float* dtheta, void* ws, hipStream_t s, int accum,
                      bool reduce) {
  Grid G = grid_of(ctx->cfg);
  int nxc = (G.nx + 63) / 64;
  long long nitems = (long long)nxc * G.ny * G.nz * G.batch;
  if (nitems >= (1LL << 31)) return fail(LBM_ERR_INVALID, "too many work items");
  const lbm_config& c = ctx->cfg;
  const int nparam = (int)param_count(c);
  float* part = static_cast<float*>(ws);
  const unsigned blocks = bwd_blocks(ctx->ncu);
  hipError_t e = nlbm_bwd_launch(L::Q == 19, H, P, blocks, s, A, theta, lam1, lam0, part, G,
                                 force_of(ctx), (float)c.rho0, (float)(1.0 / c.tau),
                                 (float)(c.out_scale / c.tau), (int)nitems, nxc, accum);
  if (e != hipSuccess)
    return fail(LBM_ERR_HIP, std::string("launch of nlbm_backward_kernel: ") + hipGetErrorString(e));
  if (!reduce) return LBM_OK;
  hipLaunchKernelGGL(grad_reduce_kernel, dim3(blocks_for(nparam, 64)), dim3(1024), 0, s, part,
                     (int)blocks, nparam, dtheta);
  LBM_LAUNCHED("grad_reduce_kernel");
  return LBM_OK;
}

template <class L, int H>
lbm_status launch_bwd_p(lbm_ctx* ctx, const float* A, const float* theta, const float* lam1,
                        float* lam0, float* dtheta, void* ws, hipStream_t s, int accum,
                        bool reduce) {
  switch (ctx->cfg.mlp_prec) {
    case LBM_MLP_FP32:
      return launch_bwd<L, H, P_F32>(ctx, A, theta, lam1, lam0, dtheta, ws, s, accum, reduce);
    case LBM_MLP_BF16:
      return launch_bwd<L, H, P_BF16>(ctx, A, theta, lam1, lam0, dtheta, ws, s, accum, reduce);
    default:
      return launch_bwd<L, H, P_F16>(ctx, A, theta, lam1, lam0, dtheta, ws, s, accum, reduce);
  }
}

template <class L>
lbm_status run_backward(lbm_ctx* ctx, const float* A, const float* theta, const float* lam1,
                        float* lam0, float* dtheta, void* ws, hipStream_t s, int accum = 0,
                        bool reduce = true) {
  const lbm_config& c = ctx->cfg;
  if (c.hidden == 0) {
    Grid G = grid_of(c);
    int nxc = (G.nx + 255) / 256;
    long long nblk = (long long)nxc * G.ny * G.nz * G.batch;
    hipLaunchKernelGGL(bgk_backward_kernel<L>, dim3((unsigned)nblk), dim3(256), 0, s, A, lam1,
                       lam0, G, force_of(ctx), (float)c.rho0, (float)(1.0 / c.tau), nxc);
    LBM_LAUNCHED("bgk_backward_kernel");
    return LBM_OK;
  }
  if (c.hidden == 32)
    return launch_bwd_p<L, 32>(ctx, A, theta, lam1, lam0, dtheta, ws, s, accum, reduce);
  return launch_bwd_p<L, 64>(ctx, A, theta, lam1, lam0, dtheta, ws, s, accum, reduce);
}

template <class L>
lbm_status run_loss(lbm_ctx* ctx, const float* A, const float* ut, double* loss, float* dLdA,
                    hipStream_t s) {
  Grid G = grid_of(ctx->cfg);
  const int nblk = MOM_BLOCKS;
  double count = (double)G.plane * G.batch * L::D;
  hipLaunchKernelGGL(loss_kernel<L>, dim3(nblk), dim3(256), 0, s, A, ut, dLdA, ctx->partial, G,
                     (float)ctx->cfg.rho0, force_of(ctx), 1.0 / count);
  LBM_LAUNCHED("loss_kernel");
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, ctx->partial, nblk,
                     1.0 / count, loss);
  LBM_LAUNCHED("sum_partials_kernel");
  return LBM_OK;
}

// ---------------------------------------------------- float64 reference
template <class L, int H>
lbm_status launch_ref(lbm_ctx* ctx, const double* Ain, double* Aout, const double* theta,
                      hipStream_t s) {
  Grid G = grid_of(ctx->cfg);
  const lbm_config& c = ctx->cfg;
  RefParams p;
  p.force_kind = c.force_kind;
  p.force_k = c.force_k;
  p.force_amp = c.force_amp;
  p.rho0 = c.rho0;
  p.tau = c.tau;
  p.knn = c.out_scale / c.tau;
  hipLaunchKernelGGL((ref_step_f64_kernel<L, H>), dim3(blocks_for((long long)G.plane * G.batch, 128)),
                     dim3(128), 0, s, Ain, Aout, theta, G, p);
  LBM_LAUNCHED("ref_step_f64_kernel");
  return LBM_OK;
}

template <class L>
lbm_status ref_step(lbm_ctx* ctx, const double* Ain, double* Aout, const double* theta,
                    hipStream_t s) {
  switch (ctx->cfg.hidden) {
    case 0: return launch_ref<L, 0>(ctx, Ain, Aout, theta, s);
    case 32: return launch_ref<L, 32>(ctx, Ain, Aout, theta, s);
    default: return launch_ref<L, 64>(ctx, Ain, Aout, theta, s);
  }
}
}  // namespace

#define LBM_GUARD_BEGIN try {
#define LBM_GUARD_END                                                        \
  }                                                                          \
  catch (const std::exception& e) {                                          \
    return fail(LBM_ERR_HIP, std::string("internal error: ") + e.what());    \
  }                                                                          \
  catch (...) {                                                              \
    return fail(LBM_ERR_HIP, "internal error");                              \
  }

extern "C" {

lbm_status lbm_create(const lbm_config* cfg, lbm_ctx** out) {
  LBM_GUARD_BEGIN
  if (!out) return fail(LBM_ERR_INVALID, "out is null");
  *out = nullptr;
  lbm_status st = validate(cfg);
  if (st != LBM_OK) return st;
  int dev = 0;
  LBM_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  LBM_HIP(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(LBM_ERR_UNSUPPORTED, std::string("built for gfx950, device is ") +
                                         prop.gcnArchName);
  lbm_ctx* ctx = new (std::nothrow) lbm_ctx;
  if (!ctx) return fail(LBM_ERR_INVALID, "out of host memory");
  ctx->cfg = *cfg;
  ctx->device = dev;
  ctx->ncu = prop.multiProcessorCount;
  ctx->scratch = static_scratch_address(dev);
  ctx->partial = nullptr;
  ctx->wide_idx = nullptr;
  ctx->wide_packed = nullptr;
  ctx->wide_nw = ctx->wide_nb = 0;
  ctx->wide_bidx = nullptr;
  ctx->wide_bpacked = nullptr;
  ctx->mrt = nullptr;
  ctx->force_tab = nullptr;
  size_t bytes = sizeof(double) * 3 * (size_t)(MOM_BLOCKS > MOMENT_BLOCKS ? MOM_BLOCKS : MOMENT_BLOCKS) *
                 (size_t)cfg->batch;
  hipError_t e = hipMalloc(&ctx->partial, bytes);
  if (e != hipSuccess) {
    delete ctx;
    return fail(LBM_ERR_HIP, std::string("hipMalloc of the reduction buffer: ") +
                                 hipGetErrorString(e));
  }
  if (cfg->force_kind != LBM_FORCE_NONE) {
    std::vector<float> tab((size_t)cfg->ny + cfg->nz + cfg->nx, 0.f);
    force_table(cfg->force_amp, cfg->force_k, cfg->ny, tab.data());
    if (cfg->force_kind == LBM_FORCE_SINE3) {
      force_table(cfg->force_amp, cfg->force_k, cfg->nz, tab.data() + cfg->ny);
      force_table(cfg->force_amp, cfg->force_k, cfg->nx, tab.data() + cfg->ny + cfg->nz);
    }
    e = hipMalloc(&ctx->force_tab, sizeof(float) * tab.size());
    if (e == hipSuccess)
      e = hipMemcpy(ctx->force_tab, tab.data(), sizeof(float) * tab.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      lbm_destroy(ctx);
      return fail(LBM_ERR_HIP, std::string("the body-force table: ") + hipGetErrorString(e));
    }
  }
  if (cfg->lattice == LBM_D3Q19) {
    e = hipMalloc(&ctx->mrt, sizeof(double) * 19 * DIAG_BLOCKS * 5);
    if (e != hipSuccess) {
      lbm_destroy(ctx);
      return fail(LBM_ERR_HIP, std::string("hipMalloc of the moment-analysis buffer: ") +
                                   hipGetErrorString(e));
    }
  }
  if (cfg->hidden != 0 && cfg->net == LBM_NET_LEAKY_300_300_100) {
    int pbytes = 0;
    std::vector<int> idx = cfg->lattice == LBM_D2Q9 ? wide_index_p<9>(cfg->mlp_prec, pbytes)
                                                     : wide_index_p<19>(cfg->mlp_prec, pbytes);
    const int eb = cfg->mlp_prec == LBM_MLP_FP32 ? 4 : 2;
    ctx->wide_nb = cfg->lattice == LBM_D2Q9 ? WideLayout<9, P_BF16>::nbias
                                            : WideLayout<19, P_BF16>::nbias;
    ctx->wide_nw = (int)idx.size() - ctx->wide_nb;
    if ((long long)ctx->wide_nw * eb + 4LL * ctx->wide_nb != pbytes) {
      lbm_destroy(ctx);
      return fail(LBM_ERR_HIP, "internal error: wide-network layout size mismatch");
    }
    e = hipMalloc(&ctx->wide_idx, sizeof(int) * idx.size());
    if (e == hipSuccess) e = hipMalloc(&ctx->wide_packed, (size_t)pbytes);
    if (e == hipSuccess)
      e = hipMemcpy(ctx->wide_idx, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice);
    std::vector<int> bidx = cfg->lattice == LBM_D2Q9 ? wide_bwd_index<9>() : wide_bwd_index<19>();
    const size_t bbytes = (size_t)WideBwd<9>::nw * eb + 4 * (size_t)WideBwd<9>::nb;
    if (e == hipSuccess) e = hipMalloc(&ctx->wide_bidx, sizeof(int) * bidx.size());
    if (e == hipSuccess) e = hipMalloc(&ctx->wide_bpacked, bbytes);
    if (e == hipSuccess)
      e = hipMemcpy(ctx->wide_bidx, bidx.data(), sizeof(int) * bidx.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      lbm_destroy(ctx);
      return fail(LBM_ERR_HIP, std::string("allocation of the wide-network buffers: ") +
                                   hipGetErrorString(e));
    }
  }
  *out = ctx;
  return LBM_OK;
  LBM_GUARD_END
}

lbm_status lbm_destroy(lbm_ctx* ctx) {
  LBM_GUARD_BEGIN
  if (!ctx) return LBM_OK;
  if (ctx->partial) (void)hipFree(ctx->partial);
  if (ctx->wide_idx) (void)hipFree(ctx->wide_idx);
  if (ctx->wide_packed) (void)hipFree(ctx->wide_packed);
  if (ctx->wide_bidx) (void)hipFree(ctx->wide_bidx);
  if (ctx->wide_bpacked) (void)hipFree(ctx->wide_bpacked);
  if (ctx->mrt) (void)hipFree(ctx->mrt);
  if (ctx->force_tab) (void)hipFree(ctx->force_tab);
  delete ctx;
  return LBM_OK;
  LBM_GUARD_END
}

size_t lbm_state_elems(const lbm_ctx* ctx) {
  if (!ctx) return 0;
  const lbm_config& c = ctx->cfg;
  return (size_t)c.batch * lattice_q(c.lattice) * c.nx * (size_t)c.ny * c.nz;
}

size_t lbm_param_elems(const lbm_ctx* ctx) {
  if (!ctx) return 0;
  return param_count(ctx->cfg);
}

size_t lbm_workspace_bytes(const lbm_ctx* ctx) {
  if (!ctx || ctx->cfg.hidden == 0) return 0;
  if (ctx->cfg.net == LBM_NET_LEAKY_300_300_100) {
    const lbm_config& c = ctx->cfg;
    return wide_bwd_workspace_bytes(c.lattice == LBM_D3Q19, prec_of(c.mlp_prec),
                                    (long long)c.batch * c.nx * c.ny * c.nz);
  }
  return sizeof(float) * (size_t)bwd_blocks(ctx->ncu) * param_count(ctx->cfg);
}

lbm_status lbm_lattice_tables(int32_t lattice, int32_t* q, int32_t* c, double* w) {
  LBM_GUARD_BEGIN
  if (!q || !c || !w) return fail(LBM_ERR_INVALID, "null output pointer");
  if (lattice == LBM_D2Q9) {
    *q = D2Q9::Q;
    for (int i = 0; i < D2Q9::Q; ++i) {
      c[3 * i] = D2Q9::cx[i];
      c[3 * i + 1] = D2Q9::cy[i];
      c[3 * i + 2] = D2Q9::cz[i];
      w[i] = D2Q9::wd[i];
    }
    return LBM_OK;
  }
  if (lattice == LBM_D3Q19) {
    *q = D3Q19::Q;
    for (int i = 0; i < D3Q19::Q; ++i) {
      c[3 * i] = D3Q19::cx[i];
      c[3 * i + 1] = D3Q19::cy[i];
      c[3 * i + 2] = D3Q19::cz[i];
      w[i] = D3Q19::wd[i];
    }
    return LBM_OK;
  }
  return fail(LBM_ERR_INVALID, "unknown lattice");
  LBM_GUARD_END
}

lbm_status lbm_init(lbm_ctx* ctx, const float* rho, const float* u, float* A0,
                    hipStream_t stream) {
  LBM_GUARD_BEGIN
  lbm_status st = check_ctx(ctx);
  if (st != LBM_OK) return st;
  if (!rho || !u || !A0) return fail(LBM_ERR_INVALID, "null array");
  if (ctx->cfg.lattice == LBM_D2Q9) return run_init<D2Q9>(ctx, rho, u, A0, stream);
  return run_init<D3Q19>(ctx, rho, u, A0, stream);
  LBM_GUARD_END
}

lbm_status lbm_step(lbm_ctx* ctx, float* A, float* B, const float* theta, int32_t nsteps,
                    hipStream_t stream) {
  LBM_GUARD_BEGIN
  lbm_status st = check_ctx(ctx);
  if (st != LBM_OK) return st;
  if (!A || !B) return fail(LBM_ERR_INVALID, "null state buffer");
  if (A == B) return fail(LBM_ERR_INVALID, "A and B must be different buffers");
  if (nsteps < 1) return fail(LBM_ERR_INVALID, "nsteps must be >= 1");
  if (ctx->cfg.hidden != 0 && !theta) return fail(LBM_ERR_INVALID, "theta is null");
  if (ctx->cfg.hidden != 0 && ctx->cfg.net == LBM_NET_LEAKY_300_300_100) {
    st = wide_pack(ctx, theta, stream);
    if (st != LBM_OK) return st;
  }
  float* buf[2] = {A, B};
  for (int s = 0; s < nsteps; ++s) {
    const float* in = buf[s & 1];
    float* out = buf[(s + 1) & 1];
    st = ctx->cfg.lattice == LBM_D2Q9 ? one_step<D2Q9>(ctx, in, out, theta, stream)
                                      : one_step<D3Q19>(ctx, in, out, theta, stream);
    if (st != LBM_OK) return st;
  }
  return LBM_OK;
  LBM_GUARD_END
}


lbm_status lbm_step_f64(lbm_ctx* ctx, double* A, double* B, const double* theta, int32_t nsteps,
                        hipStream_t stream) {
  LBM_GUARD_BEGIN
  lbm_status st = check_ctx(ctx);
  if (st != LBM_OK) return st;
  const lbm_config& c = ctx->cfg;
  if (c.collision != LBM_COLLISION_BGK)
    return fail(LBM_ERR_UNSUPPORTED, "the float64 reference step covers the BGK collision only");
  if (c.hidden != 0 && c.net != LBM_NET_TANH)
    return fail(LBM_ERR_UNSUPPORTED, "the float64 reference step covers the tanh networks only");
  if (!A || !B) return fail(LBM_ERR_INVALID, "null state buffer");
  if (A == B) return fail(LBM_ERR_INVALID, "A and B must be different buffers");
  if (nsteps < 1) return fail(LBM_ERR_INVALID, "nsteps must be >= 1");
  if (c.hidden != 0 && !theta) return fail(LBM_ERR_INVALID, "theta is null");
  double* buf[2] = {A, B};
  for (int k = 0; k < nsteps; ++k) {
    st = c.lattice == LBM_D2Q9 ? ref_step<D2Q9>(ctx, buf[k & 1], buf[(k + 1) & 1], theta, stream)
                               : ref_step<D3Q19>(ctx, buf[k & 1], buf[(k + 1) & 1], theta, stream);
    if (st != LBM_OK) return st;
  }
  return LBM_OK;
  LBM_GUARD_END
}

lbm_status lbm_moments(lbm_ctx* ctx, const float* A, float* rho, float* u, double* diag,
                       hipStream_t stream) {
  LBM_GUARD_BEGIN
  lbm_status st = check_ctx(ctx);
  if (st != LBM_OK) return st;
  if (!A) return fail(LBM_ERR_INVALID, "null state");
  if (ctx->cfg.lattice == LBM_D2Q9) return run_moments<D2Q9>(ctx, A, rho, u, diag, stream);
  return run_moments<D3Q19>(ctx, A, rho, u, diag, stream);
  LBM_GUARD_END
}

lbm_status lbm_shift(lbm_ctx* ctx, const float* src, float* dst, int32_t direction,
                     hipStream_t stream) {
  LBM_GUARD_BEGIN
  lbm_status st = check_ctx(ctx);
  if (st != LBM_OK) return st;
  if (!src || !dst) return fail(LBM_ERR_INVALID, "null array");
  if (src == dst) return fail(LBM_ERR_INVALID, "src and dst must differ");
  if (direction != 1 && direction != -1) return fail(LBM_ERR_INVALID, "direction must be +1 or -1");
  if (ctx->cfg.lattice == LBM_D2Q9) return run_shift<D2Q9>(ctx, src, dst, direction, stream);
  return run_shift<D3Q19>(ctx, src, dst, direction, stream);
  LBM_GUARD_END
}

lbm_status lbm_step_backward(lbm_ctx* ctx, const float* A_n, const float* theta,
                             const float* lam_n1, float* lam_n, float* dtheta, void* ws,
                             size_t ws_bytes, hipStream_t stream) {
  LBM_GUARD_BEGIN
  lbm_status st = check_ctx(ctx);
  if (st != LBM_OK) return st;
  if (!A_n || !lam_n1 || !lam_n) return fail(LBM_ERR_INVALID, "null array");
  if (lam_n == lam_n1 || lam_n == A_n)
    return fail(LBM_ERR_INVALID, "lam_n must not alias lam_n1 or A_n");
  if (ctx->cfg.collision != LBM_COLLISION_BGK)
    return fail(LBM_ERR_UNSUPPORTED, "the adjoint of the Smagorinsky collision is not implemented");
  if (ctx->cfg.hidden != 0) {
    if (!theta || !dtheta) return fail(LBM_ERR_INVALID, "theta and dtheta must be given");
    if (!ws) return fail(LBM_ERR_INVALID, "workspace is null");
    if (ws_bytes < lbm_workspace_bytes(ctx))
      return fail(LBM_ERR_WORKSPACE, "workspace smaller than lbm_workspace_bytes()");
  }
  if (ctx->cfg.hidden != 0 && ctx->cfg.net == LBM_NET_LEAKY_300_300_100) {
    const lbm_config& c = ctx->cfg;
    hipError_t e = wide_bwd_launch(c.lattice == LBM_D3Q19, prec_of(c.mlp_prec), stream, A_n, theta,
                                   lam_n1, lam_n, dtheta, ws, ctx->wide_bidx, ctx->wide_bpacked,
                                   grid_of(c), force_of(ctx), (float)c.rho0, (float)(1.0 / c.tau),
                                   (float)(c.out_scale / c.tau));
    if (e != hipSuccess)
      return fail(LBM_ERR_HIP, std::string("wide-network adjoint: ") + hipGetErrorString(e));
    return LBM_OK;
  }
  if (ctx->cfg.lattice == LBM_D2Q9)
    return run_backward<D2Q9>(ctx, A_n, theta, lam_n1, lam_n, dtheta, ws, stream);
  return run_backward<D3Q19>(ctx, A_n, theta, lam_n1, lam_n, dtheta, ws, stream);
  LBM_GUARD_END
}

lbm_status lbm_step_backward_static(lbm_ctx* ctx, const float* A_n, const float* theta,
                                    const float* lam_n1, float* lam_n, float* dtheta,
                                    hipStream_t stream) {
  LBM_GUARD_BEGIN
  lbm_status st = check_ctx(ctx);
  if (st != LBM_OK) return st;
  const size_t need = lbm_workspace_bytes(ctx);
  if (need > kStaticScratchBytes)
    return fail(LBM_ERR_WORKSPACE,
                "this configuration needs " + std::to_string(need) +
                    " bytes of adjoint scratch; the static buffer holds " +
                    std::to_string(kStaticScratchBytes) +
                    " (use lbm_step_backward with a workspace)");
  if (!ctx->scratch) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    const bool in_range = ctx->device >= 0 && ctx->device < kMaxDevices;
    return fail(LBM_ERR_HIP, in_range ? g_scratch_err[ctx->device]
                                      : std::string("device index out of range"));
  }
  return lbm_step_backward(ctx, A_n, theta, lam_n1, lam_n, dtheta, ctx->scratch,
                           kStaticScratchBytes, stream);
  LBM_GUARD_END
}

lbm_status lbm_step_backward_seq(lbm_ctx* ctx, const float* const* A, int32_t nsteps,
                                 const float* theta, float* lam_a, float* lam_b, float* dtheta,
                                 void* ws, size_t ws_bytes, hipStream_t stream) {
  LBM_GUARD_BEGIN
  lbm_status st = check_ctx(ctx);
  if (st != LBM_OK) return st;
  if (nsteps < 1) return fail(LBM_ERR_INVALID, "nsteps must be >= 1");
  if (!A || !lam_a || !lam_b) return fail(LBM_ERR_INVALID, "null array");
  if (lam_a == lam_b) return fail(LBM_ERR_INVALID, "lam_a and lam_b must differ");
  for (int m = 0; m < nsteps; ++m) {
    if (!A[m]) return fail(LBM_ERR_INVALID, "null state in A");
    if (A[m] == lam_a || A[m] == lam_b)
      return fail(LBM_ERR_INVALID, "lam_a and lam_b must not alias a state");
  }
  const lbm_config& c = ctx->cfg;
  // the kernels that leave one partial gradient per workgroup sum the
  // partials of all steps in ws and reduce them once; the others (plain
  // BGK, the SI's network) run lbm_step_backward step by step
  const bool shared = c.hidden != 0 && c.net != LBM_NET_LEAKY_300_300_100 &&
                      c.collision == LBM_COLLISION_BGK;
  if (shared) {
    if (!theta || !dtheta) return fail(LBM_ERR_INVALID, "theta and dtheta must be given");
    if (!ws) return fail(LBM_ERR_INVALID, "workspace is null");
    if (ws_bytes < lbm_workspace_bytes(ctx))
      return fail(LBM_ERR_WORKSPACE, "workspace smaller than lbm_workspace_bytes()");
  }
  float* in = lam_a;
  float* out = lam_b;
  for (int m = nsteps - 1; m >= 0; --m) {
    if (shared) {
      const int accum = m != nsteps - 1;
      const bool reduce = m == 0;
      st = c.lattice == LBM_D2Q9
               ? run_backward<D2Q9>(ctx, A[m], theta, in, out, dtheta, ws, stream, accum, reduce)
               : run_backward<D3Q19>(ctx, A[m], theta, in, out, dtheta, ws, stream, accum, reduce);
    } else {
      st = lbm_step_backward(ctx, A[m], theta, in, out, dtheta, ws, ws_bytes, stream);
    }
    if (st != LBM_OK) return st;
    float* t = in;
    in = out;
    out = t;
  }
  return LBM_OK;
  LBM_GUARD_END
}

lbm_status lbm_loss_velocity_mse(lbm_ctx* ctx, const float* A, const float* u_target,
                                 double* loss, float* dLdA, hipStream_t stream) {
  LBM_GUARD_BEGIN
  lbm_status st = check_ctx(ctx);
  if (st != LBM_OK) return st;
  if (!A || !u_target || !loss) return fail(LBM_ERR_INVALID, "null array");
  if (dLdA == A) return fail(LBM_ERR_INVALID, "dLdA must not alias A");
  if (ctx->cfg.lattice == LBM_D2Q9) return run_loss<D2Q9>(ctx, A, u_target, loss, dLdA, stream);
  return run_loss<D3Q19>(ctx, A, u_target, loss, dLdA, stream);
  LBM_GUARD_END
}

lbm_status lbm_adam(float* param, const float* grad, float* m, float* v, int64_t n, double lr,
                    double beta1, double beta2, double eps, double weight_decay, int32_t t,
                    hipStream_t stream) {
  LBM_GUARD_BEGIN
  if (!param || !grad || !m || !v) return fail(LBM_ERR_INVALID, "null array");
  if (n < 0) return fail(LBM_ERR_INVALID, "n must be >= 0");
  if (t < 1) return fail(LBM_ERR_INVALID, "t must be >= 1");
  if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
    return fail(LBM_ERR_INVALID, "betas must lie in [0, 1)");
  if (n == 0) return LBM_OK;
  float bc1 = (float)(1.0 - std::pow(beta1, t)), bc2 = (float)(1.0 - std::pow(beta2, t));
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(256), 0, stream, param, grad, m, v,
                     (long long)n, (float)lr, (float)beta1, (float)beta2, (float)(1.0 - beta1),
                     (float)(1.0 - beta2), (float)eps, (float)weight_decay, bc1, bc2);
  LBM_LAUNCHED("adam_kernel");
  return LBM_OK;
  LBM_GUARD_END
}

lbm_status lbm_box_filter(const float* src, float* dst, int32_t batch, int32_t channels,
                          int32_t nx, int32_t ny, int32_t nz, int32_t factor,
                          hipStream_t stream) {
  LBM_GUARD_BEGIN
  if (!src || !dst) return fail(LBM_ERR_INVALID, "null array");
  if (src == dst) return fail(LBM_ERR_INVALID, "src and dst must differ");
  if (batch < 1 || channels < 1 || nx < 1 || ny < 1 || nz < 1 || factor < 1)
    return fail(LBM_ERR_INVALID, "sizes must be >= 1");
  int fz = nz > 1 ? factor : 1;
  if (nx % factor || ny % factor || nz % fz)
    return fail(LBM_ERR_INVALID, "grid sizes must be multiples of factor");
  long long total = (long long)batch * channels * (nz / fz) * (ny / factor) * (nx / factor);
  hipLaunchKernelGGL(box_filter_kernel, dim3(blocks_for(total)), dim3(256), 0, stream, src, dst,
                     batch, channels, nx, ny, nz, factor, fz);
  LBM_LAUNCHED("box_filter_kernel");
  return LBM_OK;
  LBM_GUARD_END
}

lbm_status lbm_subsample(int32_t lattice, const float* src, float* dst, int32_t batch,
                         int32_t nx, int32_t ny, int32_t nz, int32_t factor, hipStream_t stream) {
  LBM_GUARD_BEGIN
  if (!src || !dst) return fail(LBM_ERR_INVALID, "null array");
  if (src == dst) return fail(LBM_ERR_INVALID, "src and dst must differ");
  if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19) return fail(LBM_ERR_INVALID, "unknown lattice");
  if (batch < 1 || nx < 1 || ny < 1 || nz < 1 || factor < 1)
    return fail(LBM_ERR_INVALID, "sizes must be >= 1");
  if (lattice == LBM_D2Q9 && nz != 1) return fail(LBM_ERR_INVALID, "D2Q9 needs nz == 1");
  const int fz = nz > 1 ? factor : 1;
  if (nx % factor || ny % factor || nz % fz)
    return fail(LBM_ERR_INVALID, "grid sizes must be multiples of factor");
  if ((double)batch * lattice_q(lattice) * nx * (double)ny * nz >= 1073741824.0)
    return fail(LBM_ERR_INVALID, "batch*Q*nx*ny*nz must stay below 2^30 elements");
  const long long total = (long long)batch * (nz / fz) * (ny / factor) * (nx / factor);
  if (lattice == LBM_D2Q9)
    hipLaunchKernelGGL(subsample_kernel<D2Q9>, dim3(blocks_for(total)), dim3(256), 0, stream, src,
                       dst, batch, nx, ny, nz, factor, fz);
  else
    hipLaunchKernelGGL(subsample_kernel<D3Q19>, dim3(blocks_for(total)), dim3(256), 0, stream, src,
                       dst, batch, nx, ny, nz, factor, fz);
  LBM_LAUNCHED("subsample_kernel");
  return LBM_OK;
  LBM_GUARD_END
}

lbm_status lbm_loss_population_sse(lbm_ctx* ctx, const float* A, const float* target,
                                   const int32_t* nodes, int32_t n_nodes, double* loss,
                                   float* dLdA, hipStream_t stream) {
  LBM_GUARD_BEGIN
  lbm_status st = check_ctx(ctx);
  if (st != LBM_OK) return st;
  if (!A || !target || !nodes || !loss) return fail(LBM_ERR_INVALID, "null array");
  if (n_nodes < 1) return fail(LBM_ERR_INVALID, "n_nodes must be >= 1");
  if (dLdA == A || dLdA == target) return fail(LBM_ERR_INVALID, "dLdA must not alias A or target");
  Grid G = grid_of(ctx->cfg);
  int nblk = (int)blocks_for(n_nodes);
  if (nblk > MOM_BLOCKS) nblk = MOM_BLOCKS;
  if (ctx->cfg.lattice == LBM_D2Q9)
    hipLaunchKernelGGL(population_sse_kernel<D2Q9>, dim3(nblk), dim3(256), 0, stream, A, target,
                       nodes, n_nodes, dLdA, ctx->partial, G);
  else
    hipLaunchKernelGGL(population_sse_kernel<D3Q19>, dim3(nblk), dim3(256), 0, stream, A, target,
                       nodes, n_nodes, dLdA, ctx->partial, G);
  LBM_LAUNCHED("population_sse_kernel");
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, stream, ctx->partial, nblk, 1.0,
                     loss);
  LBM_LAUNCHED("sum_partials_kernel");
  return LBM_OK;
  LBM_GUARD_END
}

size_t lbm_structure_functions_workspace_bytes(const lbm_ctx* ctx, int32_t lmax, int32_t pmax) {
  if (!ctx || lmax < 1 || pmax < 1 || pmax > SF_PMAX) return 0;
  return sizeof(double) * (size_t)lmax * DIAG_BLOCKS * 2 * (size_t)pmax;
}

lbm_status lbm_structure_functions(lbm_ctx* ctx, const float* u, int32_t lmax, int32_t pmax,
                                   double* S, double* S_abs, void* ws, size_t ws_bytes,
                                   hipStream_t stream) {
  LBM_GUARD_BEGIN
  lbm_status st = check_ctx(ctx);
  if (st != LBM_OK) return st;
  if (!u || !S || !S_abs) return fail(LBM_ERR_INVALID, "null array");
  if (pmax < 1 || pmax > SF_PMAX) return fail(LBM_ERR_INVALID, "pmax must be in 1..8");
  const lbm_config& c = ctx->cfg;
  int lim = c.nx < c.ny ? c.nx : c.ny;
  if (c.lattice == LBM_D3Q19 && c.nz < lim) lim = c.nz;
  if (lmax < 1 || lmax > lim) return fail(LBM_ERR_INVALID, "lmax must be in 1..min(grid sizes)");
  if (!ws) return fail(LBM_ERR_INVALID, "workspace is null");
  if (ws_bytes < lbm_structure_functions_workspace_bytes(ctx, lmax, pmax))
    return fail(LBM_ERR_WORKSPACE,
                "workspace smaller than lbm_structure_functions_workspace_bytes()");
  double* part = static_cast<double*>(ws);
  Grid G = grid_of(c);
  dim3 grid(DIAG_BLOCKS, (unsigned)lmax);
  if (c.lattice == LBM_D2Q9)
    hipLaunchKernelGGL(structure_kernel<2>, grid, dim3(256), 0, stream, u, G, pmax, part);
  else
    hipLaunchKernelGGL(structure_kernel<3>, grid, dim3(256), 0, stream, u, G, pmax, part);
  LBM_LAUNCHED("structure_kernel");
  const double count = (double)G.plane * G.batch * lattice_d(c.lattice);
  hipLaunchKernelGGL(structure_reduce_kernel, dim3(blocks_for((long long)lmax * 2 * pmax)), dim3(256),
                     0, stream, part, DIAG_BLOCKS, lmax, pmax, 1.0 / count, S, S_abs);
  LBM_LAUNCHED("structure_reduce_kernel");
  return LBM_OK;
  LBM_GUARD_END
}

lbm_status lbm_mrt_moment_sums(lbm_ctx* ctx, const float* A_n, const float* A_n1, double* stats,
                               hipStream_t stream) {
  LBM_GUARD_BEGIN
  lbm_status st = check_ctx(ctx);
  if (st != LBM_OK) return st;
  if (!A_n || !A_n1 || !stats) return fail(LBM_ERR_INVALID, "null array");
  if (ctx->cfg.lattice != LBM_D3Q19)
    return fail(LBM_ERR_UNSUPPORTED, "the moment matrix M is given for D3Q19 only");
  Grid G = grid_of(ctx->cfg);
  hipLaunchKernelGGL(mrt_sums_kernel, dim3(DIAG_BLOCKS, 19), dim3(256), 0, stream, A_n, A_n1, G,
                     force_of(ctx), (float)ctx->cfg.rho0, ctx->mrt);
  LBM_LAUNCHED("mrt_sums_kernel");
  hipLaunchKernelGGL(mrt_reduce_kernel, dim3(1), dim3(128), 0, stream, ctx->mrt, DIAG_BLOCKS, stats);
  LBM_LAUNCHED("mrt_reduce_kernel");
  return LBM_OK;
  LBM_GUARD_END
}

const char* lbm_status_str(lbm_status s) {
  switch (s) {
    case LBM_OK: return "LBM_OK";
    case LBM_ERR_INVALID: return "LBM_ERR_INVALID";
    case LBM_ERR_UNSUPPORTED: return "LBM_ERR_UNSUPPORTED";
    case LBM_ERR_HIP: return "LBM_ERR_HIP";
    case LBM_ERR_WORKSPACE: return "LBM_ERR_WORKSPACE";
  }
  return "unknown status";
}

const char* lbm_last_error(void) { return g_err.c_str(); }

}  // extern "C"
