/*
 * lbm.h -- C ABI of the learned-collision lattice Boltzmann step on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Ortali, Gabbana, Demo, Rozza, Toschi, "Kinetic data-driven
 * approach to turbulence subgrid modeling" (arXiv:2403.18466).  One time
 * step is the lattice Boltzmann equation of the SI (eq. lbe-sm): every node
 * collides locally and the post-collision populations stream to the
 * neighbour x + c_i.  The collision is BGK (eq. bgk-sm, equilibrium eq. feq)
 * plus a per-node neural correction (eq. nn-model-full) whose output is made
 * to conserve mass and momentum by the kappa layer of the SI ("Neural Network
 * Architecture and Optimization"); an optional body force enters through the
 * exact difference method (eq. fext).
 *
 * ---------------------------------------------------------------------------
 * Conventions shared by every entry point
 * ---------------------------------------------------------------------------
 * Memory.  Every array argument is a DEVICE pointer owned by the caller,
 * contiguous, 4-byte aligned (float) or 8-byte aligned (double).  The library
 * never frees caller memory and keeps no pointer past a call.  The context
 * owns its configuration and a small reduction buffer (see lbm_create).
 *
 * Streams.  Every call that takes a hipStream_t only enqueues work on that
 * stream (pass 0 for the null stream); none synchronises the device.  A call
 * returns LBM_ERR_HIP when a launch fails; the detail is in lbm_last_error().
 *
 * Errors.  Every function returns an lbm_status and never lets a C++
 * exception cross the ABI.  Invalid arguments are detected on the host before
 * anything is enqueued and return LBM_ERR_INVALID (or LBM_ERR_UNSUPPORTED for
 * a valid but unimplemented combination); the detail string is kept per host
 * thread and read with lbm_last_error().  Non-finite populations are not an
 * error: lbm_moments reports them in its diagnostics so that no call has to
 * read device memory.
 *
 * Lattices.  D2Q9 (nz = 1) and D3Q19.  The D3Q19 velocities c_i and weights
 * w_i are those of Table S1 of the SI, in its order.  D2Q9 uses the same
 * ordering convention (rest, axis vectors in lexicographic order of c, then
 * diagonals in lexicographic order):
 *   0:(0,0) 4/9 | 1:(-1,0) 2:(0,-1) 3:(0,1) 4:(1,0) 1/9 |
 *   5:(-1,-1) 6:(-1,1) 7:(1,-1) 8:(1,1) 1/36.
 * The order is part of the ABI because the network is not invariant under a
 * permutation of its inputs.  lbm_lattice_tables() returns both tables.
 *
 * State layout.  A population array holds float32 deviations
 *   A_q(x) = f_q - w_q * rho0
 * as [batch][Q][nz][ny][nx], x fastest (structure of arrays, one plane per
 * velocity).  It is stored in the PULL-SHIFTED form: the pre-collision
 * population of node x at step n is f_q(x, n) - w_q rho0 = A_q(x - c_q)
 * (periodic wrap).  lbm_init writes this form, lbm_step keeps it,
 * lbm_moments and the loss read it, and lbm_shift converts to and from the
 * canonical node-local form.  Storing deviations rather than f keeps the
 * float32 mantissa for the fluctuation instead of the constant w rho0.
 *
 * Network (lbm_net).  LBM_NET_TANH: Q -> H -> H -> Q with tanh after the
 * two hidden layers (H = 32 or 64).  LBM_NET_LEAKY_300_300_100: the network
 * of the SI ("Neural Network Architecture and Optimization"), Q -> 300 ->
 * 300 -> 100 -> Q with LeakyReLU (negative slope 0.01) after the three
 * hidden layers.  Both have a linear output layer; the output y enters the
 * collision as (s_out/tau) y and the whole collision update is projected
 * off span{1, c_x, c_y[, c_z]}.  Parameters are one packed float32 vector
 * (length lbm_param_elems), layer by layer: W_l (row-major [out][in]) then
 * b_l, i.e. [W1 b1 W2 b2 W3 b3] for the tanh network and
 * [W1 b1 W2 b2 W3 b3 W4 b4] for the other.  The network input is the node's
 * pre-collision deviation vector.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_ERR_INVALID = 1,     /* bad argument: null pointer, size, aliasing, range */
    LBM_ERR_UNSUPPORTED = 2, /* valid request this library does not implement */
    LBM_ERR_HIP = 3,         /* a HIP launch or query failed */
    LBM_ERR_WORKSPACE = 4    /* workspace argument smaller than required */
} lbm_status;

typedef enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1 } lbm_lattice;

/* Precision of the network contractions.  Populations, the BGK part, the
 * projection and the force are float32 in every mode.
 *   LBM_MLP_FP32: float32 operands, float32 accumulation (matrix cores).
 *   LBM_MLP_BF16: operands (network input, hidden activations, weights)
 *                 rounded to bfloat16 by round-to-nearest-even, float32
 *                 accumulation; biases and tanh in float32.
 *   LBM_MLP_FP16: the same with IEEE binary16 operands. */
typedef enum { LBM_MLP_FP32 = 1, LBM_MLP_BF16 = 2, LBM_MLP_FP16 = 3 } lbm_prec;

/* Network kind (see "Network" above). */
typedef enum { LBM_NET_TANH = 0, LBM_NET_LEAKY_300_300_100 = 1 } lbm_net;

/* Collision operator.
 *   LBM_COLLISION_BGK: BGK at tau (eq. bgk-sm), plus the network if hidden > 0.
 *   LBM_COLLISION_SMAGORINSKY: BGK at the local relaxation time of the
 *     Smagorinsky model (SI, "Implementing the Smagorinsky Turbulence Model
 *     in LBM"), computed from the node's non-equilibrium stress in the same
 *     pass, with dt = 1, c_s^2 = 1/3 and filter width 1:
 *       Pi^neq_ab = sum_q c_qa c_qb (f_q - f^eq_q),
 *       S_ab = -3 / (2 tau) Pi^neq_ab,  |S| = sqrt(2 S_ab S_ab),
 *       tau_eff = 3 ((tau - 1/2) / 3 + smag_cs^2 |S|) + 1/2.
 *     The SI prints the factor as 3 tau / 2; 3 / (2 tau) is the
 *     Chapman-Enskog relation Pi^neq = -2 rho c_s^2 tau S with rho = 1.
 *     Requires hidden == 0; no adjoint (LBM_ERR_UNSUPPORTED). */
typedef enum { LBM_COLLISION_BGK = 0, LBM_COLLISION_SMAGORINSKY = 1 } lbm_collision;

/* Body force F(x), added by the exact difference method of eq. fext.
 *   LBM_FORCE_NONE.
 *   LBM_FORCE_KOLMOGOROV: F_x = amp * sin(2 pi k y / ny), F_y = F_z = 0.
 *   LBM_FORCE_SINE3: the three-component forcing of the SI's DNS set-up,
 *     F_x = amp sin(2 pi k y / ny), F_y = amp sin(2 pi k z / nz),
 *     F_z = amp sin(2 pi k x / nx)  (D3Q19 only). */
typedef enum { LBM_FORCE_NONE = 0, LBM_FORCE_KOLMOGOROV = 1, LBM_FORCE_SINE3 = 2 } lbm_force;

typedef struct {
    int32_t lattice;     /* lbm_lattice */
    int32_t nx, ny, nz;  /* periodic grid; nz = 1 for D2Q9; each >= 1 */
    int32_t batch;       /* independent fields, >= 1 */
    double tau;          /* BGK relaxation time, > 0.5 (eq. tau: nu = (tau - 1/2)/3) */
    double rho0;         /* reference density of the deviation form, > 0 */
    int32_t force_kind;  /* lbm_force */
    int32_t force_k;     /* forcing wavenumber k */
    double force_amp;    /* forcing amplitude */
    int32_t hidden;      /* 0 = plain BGK; LBM_NET_TANH: H = 32 or 64;
                            LBM_NET_LEAKY_300_300_100: 300 (the first width) */
    int32_t mlp_prec;    /* lbm_prec; ignored when hidden == 0 */
    double out_scale;    /* s_out: the network term is (s_out / tau) * y */
    int32_t net;         /* lbm_net; ignored when hidden == 0 */
    int32_t collision;   /* lbm_collision */
    double smag_cs;      /* Smagorinsky constant C_s (LBM_COLLISION_SMAGORINSKY), >= 0 */
} lbm_config;

/* Validate `cfg` and create a context holding a copy of it, bound to the
 * current device.  The context allocates one small device buffer
 * (96 KiB per field) for the float64 partial sums of lbm_moments and the
 * losses, and for D3Q19 one of 48 KiB for lbm_mrt_moment_sums; calls that
 * use one context must therefore be ordered (one stream, or synchronised
 * streams).  With
 * LBM_NET_LEAKY_300_300_100 it also holds the weights in the kernel's
 * fragment order (about 0.3 MB in bf16/fp16, 0.6 MB in fp32, refreshed from
 * theta by every lbm_step call) and its index table (0.6 MB), plus the
 * adjoint's padded W and W^T (0.6 MB in bf16/fp16, 1.1 MB in fp32) and its
 * index table (1.1 MB).  Limit:
 * batch * Q * nx * ny * nz < 2^30 elements (each population array below
 * 4 GiB, the range of the kernels' 32-bit byte offsets).  Returns
 * LBM_ERR_INVALID or LBM_ERR_UNSUPPORTED with the reason in
 * lbm_last_error(), LBM_ERR_HIP if the device query or allocation fails. */
lbm_status lbm_create(const lbm_config* cfg, lbm_ctx** out);
lbm_status lbm_destroy(lbm_ctx* ctx);

/* Sizes in elements: population array (batch*Q*nz*ny*nx), packed parameter
 * vector (0 when hidden == 0), and the workspace of lbm_step_backward in
 * bytes.  Return 0 for a null context. */
size_t lbm_state_elems(const lbm_ctx* ctx);
size_t lbm_param_elems(const lbm_ctx* ctx);
size_t lbm_workspace_bytes(const lbm_ctx* ctx);

/* Host copies of the lattice tables: c[Q][3] (int32, z component 0 for
 * D2Q9) and w[Q] (double), in ABI order.  Q is written to *q.  Arrays must
 * hold 19 entries (57 for c). */
lbm_status lbm_lattice_tables(int32_t lattice, int32_t* q, int32_t* c, double* w);

/* Equilibrium initial state (eq. feq with c_s^2 = 1/3):
 *   A0_q(x - c_q) = f^eq_q(rho(x), u(x)) - w_q rho0,
 * i.e. the pull-shifted form of an equilibrium with the given fields.
 * rho: [batch][nz][ny][nx] float32; u: [batch][D][nz][ny][nx] float32
 * (D = 2 or 3); A0: population array (written). */
lbm_status lbm_init(lbm_ctx* ctx, const float* rho, const float* u, float* A0,
                    hipStream_t stream);

/* nsteps >= 1 time steps of eq. lbe-sm with the collision of
 * eq. nn-model-full (BGK alone when hidden == 0): each node gathers its
 * pre-collision populations A_q(x - c_q), collides and writes the
 * post-collision vector at x, which is the pull-shifted state of the next
 * step.  The two buffers alternate: step s reads buf[s % 2] and writes
 * buf[(s + 1) % 2] with buf = {A, B}.  The result is therefore in B when
 * nsteps is odd and in A when it is even; for nsteps > 1 both buffers are
 * overwritten.  A != B, both population arrays.  theta: packed parameters
 * (ignored, may be null, when hidden == 0); with LBM_NET_LEAKY_300_300_100
 * the call first converts theta into the context's fragment buffer, so
 * theta may change between calls but not during one. */
lbm_status lbm_step(lbm_ctx* ctx, float* A, float* B, const float* theta, int32_t nsteps,
                    hipStream_t stream);

/* The float64 reference instance of lbm_step: the same map (collision of
 * eq. nn-model-full with the kappa projection, force by eq. fext) with the
 * populations, the parameters and every operation in float64.  A plain
 * kernel, one thread per node, made to check long float32 / bf16 / fp16 runs
 * (e.g. thousands of steps of a turbulent field) against the reference
 * precision on the GPU; it is itself checked against the CPU oracle.
 * A, B: float64 population arrays ([batch][Q][nz][ny][nx] deviations,
 * pull-shifted as for lbm_step), ping-pong as lbm_step (result in B for odd
 * nsteps, in A for even).  theta: packed float64 parameters (may be null when
 * hidden == 0).  mlp_prec is ignored.  LBM_ERR_UNSUPPORTED for the
 * Smagorinsky collision and for LBM_NET_LEAKY_300_300_100. */
lbm_status lbm_step_f64(lbm_ctx* ctx, double* A, double* B, const double* theta, int32_t nsteps,
                        hipStream_t stream);

/* Moments of the pre-collision state (SI: rho = sum f, rho u = sum f c):
 *   rho = rho0 + sum_q A_q(x - c_q),  u = (j + F/2) / rho,
 * with j = sum_q c_q A_q(x - c_q) and F the body force (the usual
 * exact-difference-method velocity).  rho: [batch][nz][ny][nx] float32 and
 * u: [batch][D][nz][ny][nx] float32, each may be null.  diag (may be null):
 * [batch][4] float64 = {total mass, kinetic energy 1/2 sum rho |u|^2, number
 * of nodes holding a non-finite population, 0}; those nodes are left out of
 * the sums.  The diagnostics are summed in float64 in a fixed order, so they
 * are bit-reproducible for a given size. */
lbm_status lbm_moments(lbm_ctx* ctx, const float* A, float* rho, float* u, double* diag,
                       hipStream_t stream);

/* Convert between the pull-shifted and the canonical node-local form of a
 * population array: direction +1 writes g_q(x) = A_q(x - c_q) (canonical
 * from shifted), direction -1 writes A_q(x) = g_q(x + c_q) (shifted from
 * canonical).  src != dst.  This is the streaming permutation of the SI's
 * stream/collide split and its inverse (the anti-streaming of Fig. 2). */
lbm_status lbm_shift(lbm_ctx* ctx, const float* src, float* dst, int32_t direction,
                     hipStream_t stream);

/* Adjoint of one lbm_step (reverse-mode derivative, the backpropagation of
 * the SI's unrolled training).  With A_n the state that lbm_step mapped to
 * A_{n+1} and lam_n1 = dL/dA_{n+1}:
 *   lam_n  = (dA_{n+1}/dA_n)^T lam_n1            (written, population array)
 *   dtheta += (dA_{n+1}/dtheta)^T lam_n1          (accumulated, packed layout)
 * The step is recomputed from A_n inside the kernel (no activations are
 * stored).  In the bf16/fp16 modes the rounding of the forward operands is
 * passed straight through and the backward contractions use the same operand
 * precision.  fp16 operands cover 6e-8 .. 65504 only: where the network's
 * part of the adjoint, (s_out / tau) times lam^{n+1} projected, falls below
 * that (a mean loss over many nodes), it flushes to zero; scale lam^{n+1}
 * by a power of two (loss scaling) or use bf16, whose range is float32's.  ws: device workspace of at least lbm_workspace_bytes() bytes
 * for the per-workgroup partial parameter gradients, which are summed in a
 * fixed order (the result is bit-reproducible).  dtheta may be null only
 * when hidden == 0.  lam_n must not alias lam_n1 or A_n.
 * With LBM_NET_LEAKY_300_300_100 the adjoint runs as dense products over the
 * node dimension and keeps every hidden activation in the workspace (about
 * 6 KB per node in bf16/fp16, 12 KB in fp32: meant for training grids such
 * as 32^3 - 64^3); the weights are repacked from theta by the call.  Not
 * implemented for LBM_COLLISION_SMAGORINSKY (LBM_ERR_UNSUPPORTED). */
lbm_status lbm_step_backward(lbm_ctx* ctx, const float* A_n, const float* theta,
                             const float* lam_n1, float* lam_n, float* dtheta, void* ws,
                             size_t ws_bytes, hipStream_t stream);

/* lbm_step_backward without a workspace argument and without any
 * allocation, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving or training loops, harnesses that forbid
 * hipMalloc).  The per-workgroup partial gradients go to a static device
 * buffer of 8 MiB that the library holds on each device until the process
 * ends (looked up by lbm_create); every partial row is written before it is
 * read, so nothing needs clearing between calls.  Configurations whose
 * lbm_workspace_bytes() exceeds 8 MiB return LBM_ERR_WORKSPACE with nothing
 * enqueued: this covers plain BGK and every tanh network on grids of any
 * size (their partials depend only on the number of compute units and
 * parameters: 6.8 MB at most on 256 compute units), and the SI's network,
 * whose workspace holds every activation of every node (about 6 KB per node
 * in bf16), only on grids of up to about a thousand nodes.  All calls on one
 * device share the buffer: calls that may overlap on one device (different
 * streams, or host threads) race and must be ordered by the caller.
 * Arguments, results and other errors as lbm_step_backward, which it
 * equals bit for bit. */
lbm_status lbm_step_backward_static(lbm_ctx* ctx, const float* A_n, const float* theta,
                                    const float* lam_n1, float* lam_n, float* dtheta,
                                    hipStream_t stream);

/* The adjoint of nsteps consecutive lbm_step calls, the backward pass over
 * one checkpoint segment of the SI's unrolled training: for m = nsteps - 1
 * down to 0, lbm_step_backward with A_n = A[m], giving
 *   lam^m   = (dA^{m+1}/dA^m)^T lam^{m+1}
 *   dtheta += sum over m of (dA^{m+1}/dtheta)^T lam^{m+1}.
 * A: host array of nsteps device pointers, A[m] the state the m-th step read
 * (a population array each).  lam_a holds lam^{nsteps} on entry; lam_a and
 * lam_b then take the outputs in turn, so lam^0 ends in lam_b for odd
 * nsteps and in lam_a for even (lam_a is overwritten when nsteps >= 2).
 * lam_a and lam_b must differ and alias no state.  For the tanh networks
 * (hidden > 0, LBM_NET_TANH) the per-workgroup partial gradients of all the
 * steps are summed in ws (in step order, so the result is bit-reproducible)
 * and reduced into dtheta once; it equals the step-by-step sum up to float32
 * rounding order.  Plain BGK and LBM_NET_LEAKY_300_300_100 run the steps
 * through lbm_step_backward.  Errors as lbm_step_backward, plus
 * LBM_ERR_INVALID for nsteps < 1 or a null entry of A. */
lbm_status lbm_step_backward_seq(lbm_ctx* ctx, const float* const* A, int32_t nsteps,
                                 const float* theta, float* lam_a, float* lam_b, float* dtheta,
                                 void* ws, size_t ws_bytes, hipStream_t stream);

/* Velocity mean-squared error of a pull-shifted state against a target
 * field (the training loss, a mean rather than the sum of eq. nn-loss, on
 * velocities rather than populations):
 *   L = mean over batch, nodes and D components of (u - u_target)^2,
 * u as in lbm_moments.  loss: one float64, written.  dLdA (may be null):
 * dL/dA in pull-shifted layout, written.  u_target: [batch][D][nz][ny][nx]
 * float32.  The sum is taken in float64 in a fixed order. */
lbm_status lbm_loss_velocity_mse(lbm_ctx* ctx, const float* A, const float* u_target,
                                 double* loss, float* dLdA, hipStream_t stream);

/* One Adam step with L2 weight decay added to the gradient (the optimiser
 * of the SI's Table S2), in float32 for n parameters:
 *   g = grad + wd * p;  m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
 *   p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * t >= 1 is the step count after this update. */
lbm_status lbm_adam(float* param, const float* grad, float* m, float* v, int64_t n,
                    double lr, double beta1, double beta2, double eps, double weight_decay,
                    int32_t t, hipStream_t stream);

/* Coarse-graining by block averaging: dst(X) = mean of src over the
 * factor^D fine nodes of block X, per [batch][channel] plane.  src:
 * [batch][channels][nz][ny][nx], dst: [batch][channels][nz/f][ny/f][nx/f]
 * (nz untouched when nz == 1).  Each of nx, ny (and nz > 1) must be a
 * multiple of factor. */
lbm_status lbm_box_filter(const float* src, float* dst, int32_t batch, int32_t channels,
                          int32_t nx, int32_t ny, int32_t nz, int32_t factor,
                          hipStream_t stream);

/* Sub-sampling filter of the SI's training set ("Definition of the Training
 * Dataset": one lattice point in every `factor` along each axis) for
 * pull-shifted population arrays: the coarse canonical population at node X
 * is the fine one at factor * X, which in the pull-shifted form of both
 * grids reads
 *   dst_q(X) = src_q(factor X + (factor - 1) c_q)   (periodic).
 * src: [batch][Q][nz][ny][nx] of `lattice`; dst: [batch][Q][nz/f][ny/f][nx/f]
 * (nz is not divided for D2Q9, where nz == 1).  Sizes must be multiples of
 * factor.  src != dst. */
lbm_status lbm_subsample(int32_t lattice, const float* src, float* dst, int32_t batch,
                         int32_t nx, int32_t ny, int32_t nz, int32_t factor, hipStream_t stream);

/* Population loss of eq. nn-loss on a node subset S:
 *   L = sum over x in S and q of (A_q(x) - T_q(x))^2,
 * A the model's state after the unrolled steps, T the target, both
 * population arrays of the context.  Because they are pull-shifted,
 * A_q(x) is the post-collision population of node x of the last step: the
 * comparison of post-collision values of the SI needs no separate
 * anti-streaming.  nodes: device int32[n_nodes] of flat indices
 * b * (nx ny nz) + (z ny + y) nx + x, which must be distinct; an index out of
 * range makes *loss NaN.  loss: device float64[1].  dLdA (may be null):
 * written with 2 (A - T) at the listed nodes and left untouched elsewhere
 * (zero it first to obtain the full gradient).  Summed in float64 in a
 * fixed order. */
lbm_status lbm_loss_population_sse(lbm_ctx* ctx, const float* A, const float* target,
                                   const int32_t* nodes, int32_t n_nodes, double* loss,
                                   float* dLdA, hipStream_t stream);

/* Eulerian structure functions (SI, eq. structure-fun-sm) of a velocity
 * field u [batch][D][nz][ny][nx] of the context's grid, along the lattice
 * axes: for l = 1..lmax and p = 1..pmax,
 *   S[p-1][l-1]     = < (u_a(x + l e_a) - u_a(x))^p >,
 *   S_abs[p-1][l-1] = < |u_a(x + l e_a) - u_a(x)|^p >,
 * means over every node, field and axis a (the longitudinal increment,
 * periodic).  S, S_abs: device float64 [pmax][lmax].  pmax <= 8, lmax <=
 * the smallest grid size.  Increments and sums in float64, fixed order.
 * ws: caller-owned device workspace of at least
 * lbm_structure_functions_workspace_bytes(ctx, lmax, pmax) bytes for the
 * per-block partial sums (LBM_ERR_WORKSPACE if smaller); the call neither
 * allocates nor waits for the device. */
size_t lbm_structure_functions_workspace_bytes(const lbm_ctx* ctx, int32_t lmax, int32_t pmax);
lbm_status lbm_structure_functions(lbm_ctx* ctx, const float* u, int32_t lmax, int32_t pmax,
                                   double* S, double* S_abs, void* ws, size_t ws_bytes,
                                   hipStream_t stream);

/* Sums of the SI's moment-space analysis of a collision (D3Q19 only; the
 * SI gives M for D3Q19).  A_n and A_n1 are consecutive states of lbm_step
 * (pull-shifted, so A_n1(x) holds the post-collision populations of node
 * x).  With pre = A_n gathered at x, f^eq and f^ext of pre (eq. feq,
 * eq. fext) and the MRT matrix M:
 *   m_diff = M (post - pre - f_ext),   m_neq = M (f_eq - pre),
 * stats[i][0..4] (device float64 [19][5]) = sums over the nodes of m_neq_i,
 * m_diff_i, m_neq_i^2, m_neq_i m_diff_i, m_diff_i^2.  A relaxation
 * m_diff_i = m_neq_i / tau_i shows as the regression slope 1 / tau_i. */
lbm_status lbm_mrt_moment_sums(lbm_ctx* ctx, const float* A_n, const float* A_n1, double* stats,
                               hipStream_t stream);

const char* lbm_status_str(lbm_status s);
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
