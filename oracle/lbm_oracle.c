/*
 * lbm_oracle.c -- plain serial FP64 reference of the learned-collision
 * lattice Boltzmann step (Ortali, Gabbana, Demo, Rozza, Toschi,
 * "Kinetic data-driven approach to turbulence subgrid modeling",
 * arXiv:2403.18466).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.  It shares
 * no code, header, table or constant with the GPU library: every constant
 * below is typed here from the paper (or from the stated reading where the
 * paper is silent).
 *
 * State convention: canonical pre-collision populations stored as deviations
 *   g_q(x) = f_q^pre(x) - w_q * rho0,
 * layout [B][Q][nz][ny][nx], x fastest.  All arithmetic is double precision,
 * node by node, in the order the paper states the method.
 *
 * One step (SI, "Numerical Method" and "Neural Network Architecture"):
 *   moments      rho = sum f, rho u = sum f c                   (SI, moments)
 *   equilibrium  2nd-order polynomial f^eq(rho, u)              (eq. feq)
 *   BGK          Omega = -(1/tau)(f - f^eq), dt = 1             (eq. bgk-sm)
 *                (or with the local tau_eff of the Smagorinsky model, SI,
 *                "Implementing the Smagorinsky Turbulence Model in LBM")
 *   network      y = MLP(g): tanh net Q-H-H-Q, or the SI's net
 *                Q-300-300-100-Q with LeakyReLU                 (SI, MLP)
 *   update       Omega + (s_out/tau) y                          (eq. nn-model-full)
 *   projection   remove the components along 1 and c_alpha      (SI, kappa layer)
 *   forcing      f^eq(rho, u + F/rho) - f^eq(rho, u)            (eq. fext, EDM)
 *   collide      f^post = f^pre + update + f^ext                (eq. lbe-sm)
 *   stream       f^pre(x, t+1) = f^post(x - c, t), periodic     (stream/collide split)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Lattices                                                                  */
/* ------------------------------------------------------------------------ */

/* D3Q19, in the order and with the weights of Table S1. */
static const int D3Q19_C[19][3] = {
    {0, 0, 0},
    {-1, 0, 0}, {0, -1, 0}, {0, 0, -1}, {0, 0, 1}, {0, 1, 0}, {1, 0, 0},
    {-1, -1, 0}, {-1, 0, -1}, {-1, 0, 1}, {-1, 1, 0},
    {0, -1, -1}, {0, -1, 1}, {0, 1, -1}, {0, 1, 1},
    {1, -1, 0}, {1, 0, -1}, {1, 0, 1}, {1, 1, 0}};
static const double D3Q19_W[19] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* D2Q9.  The paper gives only D3Q19; this follows the same convention as
 * Table S1: rest vector, then the axis vectors in lexicographic order, then
 * the diagonals in lexicographic order.  Weights 4/9, 1/9, 1/36. */
static const int D2Q9_C[9][3] = {
    {0, 0, 0},
    {-1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {1, 0, 0},
    {-1, -1, 0}, {-1, 1, 0}, {1, -1, 0}, {1, 1, 0}};
static const double D2Q9_W[9] = {
    4.0 / 9.0,
    1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

#define QMAX 19
#define HMAX 512
#define NLMAX 4       /* linear layers of the largest network */
#define LEAKY_SLOPE 0.01

typedef struct {
    int32_t lattice; /* 0 = D2Q9, 1 = D3Q19 */
    int32_t nx, ny, nz, batch;
    double tau, rho0;
    int32_t force_kind; /* 0 none; 1 Kolmogorov Fx = A sin(2 pi k y / ny);
                           2 the SI's three-component sine forcing */
    double force_amp;
    int32_t force_k;
    int32_t hidden;     /* 0 = plain BGK */
    int32_t quant;      /* 0 exact; 1 bf16; 2 fp16 rounding at the MLP operands */
    double out_scale;   /* s_out: the network update is (s_out / tau) y */
    int32_t net;        /* 0: Q-H-H-Q, tanh; 1: the SI's Q-300-300-100-Q, LeakyReLU
                           (hidden must be 300) */
    int32_t collision;  /* 0: BGK at tau; 1: BGK at the Smagorinsky tau_eff (hidden
                           must be 0) */
    double smag_cs;     /* Smagorinsky constant C_s (filter width = 1 lattice unit) */
    int32_t quant_weights; /* with quant != 0: 1 rounds every weight to the format
                              (the rounding points of the reduced-precision network);
                              0 takes the weights as given, for a caller that
                              supplies the operand weights in effect itself */
} orc_config;

typedef struct {
    int Q, D;
    const int (*c)[3];
    const double *w;
} lattice_t;

static int get_lattice(int id, lattice_t *L) {
    if (id == 0) {
        L->Q = 9; L->D = 2; L->c = D2Q9_C; L->w = D2Q9_W;
        return 0;
    }
    if (id == 1) {
        L->Q = 19; L->D = 3; L->c = D3Q19_C; L->w = D3Q19_W;
        return 0;
    }
    return -1;
}

int orc_tables(int lattice, int *Q, int *D, int *c, double *w) {
    lattice_t L;
    if (get_lattice(lattice, &L)) return -1;
    *Q = L.Q;
    *D = L.D;
    for (int q = 0; q < L.Q; ++q) {
        for (int a = 0; a < 3; ++a) c[3 * q + a] = L.c[q][a];
        w[q] = L.w[q];
    }
    return 0;
}

/* Layer widths of the network.  net 0: Q -> H -> H -> Q with tanh after the
 * two hidden layers (the workload's small network).  net 1: the network of
 * the SI ("Neural Network Architecture and Optimization"): Q -> 300 -> 300 ->
 * 100 -> Q with LeakyReLU after the three hidden layers; the SI does not give
 * the negative slope, 0.01 is taken.  The output layer is linear in both. */
typedef struct {
    int nl;                 /* number of linear layers (0: no network) */
    int width[NLMAX + 1];   /* width[0] = width[nl] = Q */
    int leaky;              /* hidden activation: 0 tanh, 1 LeakyReLU */
} net_shape;

static int get_net(int Q, int hidden, int net, net_shape *n) {
    memset(n, 0, sizeof(*n));
    if (hidden == 0) return 0;
    if (net == 0) {
        if (hidden < 0 || hidden > HMAX) return -1;
        n->nl = 3;
        n->width[0] = Q; n->width[1] = hidden; n->width[2] = hidden; n->width[3] = Q;
        return 0;
    }
    if (net == 1) {
        if (hidden != 300) return -1;
        n->nl = 4; n->leaky = 1;
        n->width[0] = Q; n->width[1] = 300; n->width[2] = 300; n->width[3] = 100; n->width[4] = Q;
        return 0;
    }
    return -1;
}

/* Number of packed parameters: for each layer l in order, W_l (row-major
 * [out][in]) followed by b_l.  For net 0 this is [W1 b1 W2 b2 W3 b3]. */
int64_t orc_param_elems(int lattice, int hidden, int net) {
    lattice_t L;
    net_shape n;
    if (get_lattice(lattice, &L) || get_net(L.Q, hidden, net, &n)) return 0;
    int64_t tot = 0;
    for (int l = 0; l < n.nl; ++l) tot += (int64_t)n.width[l + 1] * (n.width[l] + 1);
    return tot;
}

/* ------------------------------------------------------------------------ */
/* Rounding to a reduced-precision format, round-to-nearest-even.            */
/* Used only in the emulated-quantisation mode: the value is rounded to the  */
/* nearest number representable with `bits` significant bits (including the */
/* implicit one) and the exponent range of the format, then kept in double. */
/* ------------------------------------------------------------------------ */
static double round_to_format(double v, int bits, int emin, double maxval) {
    if (v == 0.0 || !isfinite(v)) return v;
    int e;
    frexp(v, &e);                  /* v = m 2^e, 0.5 <= |m| < 1 */
    int ulp_exp = e - bits;        /* spacing of representable numbers */
    int min_ulp_exp = emin - bits; /* subnormal spacing: 2^(emin-1) / 2^(bits-1) */
    if (ulp_exp < min_ulp_exp) ulp_exp = min_ulp_exp;
    double r = ldexp(nearbyint(ldexp(v, -ulp_exp)), ulp_exp); /* RNE */
    if (fabs(r) > maxval) r = copysign(INFINITY, v);
    return r;
}

/* `emin` is the frexp exponent of the smallest normal number (frexp writes
 * v = m 2^e with 1/2 <= |m| < 1), so normal spacing is 2^(e - bits) and the
 * subnormal spacing is 2^(emin - bits).
 * bfloat16: 8 significant bits, smallest normal 2^-126 (emin = -125).
 * binary16: 11 significant bits, smallest normal 2^-14 (emin = -13), largest 65504. */
double orc_round_bf16(double v) { return round_to_format(v, 8, -125, 3.3895313892515355e38); }
double orc_round_fp16(double v) { return round_to_format(v, 11, -13, 65504.0); }

static double quantise(int quant, double v) {
    if (quant == 1) return orc_round_bf16(v);
    if (quant == 2) return orc_round_fp16(v);
    return v;
}

/* The weight a reduced-precision network reads: the stored float32 weight
 * rounded to the operand format.  Biases are not rounding points (they are
 * added to the float32 sums). */
static double qweight(const orc_config *cfg, double w) {
    if (!cfg->quant || !cfg->quant_weights) return w;
    return quantise(cfg->quant, w);
}

/* ------------------------------------------------------------------------ */
/* Per-node physics                                                          */
/* ------------------------------------------------------------------------ */

/* Body force at integer node (x, y, z) of a field with the given sizes. */
static void body_force(const orc_config *cfg, int x, int y, int z, double F[3]) {
    F[0] = F[1] = F[2] = 0.0;
    const double two_pi = 6.283185307179586476925286766559;
    if (cfg->force_kind == 1) {
        F[0] = cfg->force_amp * sin(two_pi * cfg->force_k * y / (double)cfg->ny);
    } else if (cfg->force_kind == 2) {
        /* SI, DNS set-up: Fx(y), Fy(z), Fz(x), each F sin(2 pi k s / L). */
        F[0] = cfg->force_amp * sin(two_pi * cfg->force_k * y / (double)cfg->ny);
        F[1] = cfg->force_amp * sin(two_pi * cfg->force_k * z / (double)cfg->nz);
        F[2] = cfg->force_amp * sin(two_pi * cfg->force_k * x / (double)cfg->nx);
    }
}

/* Equilibrium of eq. feq with c_s^2 = 1/3, written as a deviation from
 * w rho0 and as a function of (drho = rho - rho0, momentum j = rho u):
 *   f^eq_q - w_q rho0 = w_q [ drho + rho (3 c.u + 9/2 (c.u)^2 - 3/2 |u|^2) ]. */
static void equilibrium_dev(const lattice_t *L, double rho0, double drho,
                            const double j[3], double geq[]) {
    double rho = rho0 + drho;
    double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int q = 0; q < L->Q; ++q) {
        double cu = L->c[q][0] * u[0] + L->c[q][1] * u[1] + L->c[q][2] * u[2];
        geq[q] = L->w[q] * (drho + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    }
}

/* Per-node moments: drho = sum g, j = sum g c (the w rho0 part sums to 0). */
static void node_moments(const lattice_t *L, const double g[], double *drho, double j[3]) {
    double s = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int q = 0; q < L->Q; ++q) {
        s += g[q];
        jx += g[q] * L->c[q][0];
        jy += g[q] * L->c[q][1];
        jz += g[q] * L->c[q][2];
    }
    *drho = s;
    j[0] = jx; j[1] = jy; j[2] = jz;
}

/* Orthogonal projection onto the complement of span{1, c_x, c_y, c_z}
 * (SI, kappa layer): v <- v + k1 + k2 c_x + k3 c_y + k4 c_z with
 * k1 = -sum v / Q and k_{a+1} = -sum v c_a / sum c_a^2. */
static void project(const lattice_t *L, double v[]) {
    double s = 0.0, m[3] = {0, 0, 0}, n2[3] = {0, 0, 0};
    for (int q = 0; q < L->Q; ++q) {
        s += v[q];
        for (int a = 0; a < 3; ++a) {
            m[a] += v[q] * L->c[q][a];
            n2[a] += (double)(L->c[q][a] * L->c[q][a]);
        }
    }
    double k1 = -s / L->Q;
    double k[3];
    for (int a = 0; a < 3; ++a) k[a] = (n2[a] > 0) ? -m[a] / n2[a] : 0.0;
    for (int q = 0; q < L->Q; ++q)
        v[q] += k1 + k[0] * L->c[q][0] + k[1] * L->c[q][1] + k[2] * L->c[q][2];
}

/* Saved forward quantities of one node, needed by the adjoint. */
typedef struct {
    double g[QMAX];
    double drho, j[3], F[3];
    double x0[QMAX];
    double pre[NLMAX][HMAX];  /* hidden pre-activations */
    double t[NLMAX][HMAX];    /* activation values before rounding */
    double h[NLMAX][HMAX];    /* activations as the next layer reads them */
    double y[QMAX];
} node_fwd;

static double activation(int leaky, double a) {
    if (leaky) return a > 0.0 ? a : LEAKY_SLOPE * a;
    return tanh(a);
}

/* Derivative of the activation, from the pre-activation a and the value t. */
static double activation_slope(int leaky, double a, double t) {
    if (leaky) return a > 0.0 ? 1.0 : LEAKY_SLOPE;
    return 1.0 - t * t; /* tanh' = 1 - tanh^2 */
}

/* The MLP of the SI: linear layers with the hidden activation after every
 * layer but the last.  In the emulated reduced-precision mode the rounding
 * points are the network input, every weight and every hidden activation
 * (after the exact activation function); the biases and all sums stay
 * exact. */
static void mlp_forward(const orc_config *cfg, const net_shape *n, const double *theta,
                        node_fwd *s) {
    int qt = cfg->quant;
    for (int i = 0; i < n->width[0]; ++i) s->x0[i] = quantise(qt, s->g[i]);
    const double *in = s->x0;
    const double *W = theta;
    for (int l = 0; l < n->nl; ++l) {
        int nin = n->width[l], nout = n->width[l + 1];
        const double *b = W + (int64_t)nout * nin;
        for (int o = 0; o < nout; ++o) {
            double a = b[o];
            for (int i = 0; i < nin; ++i) a += qweight(cfg, W[(int64_t)o * nin + i]) * in[i];
            if (l + 1 < n->nl) {
                s->pre[l][o] = a;
                s->t[l][o] = activation(n->leaky, a);
                s->h[l][o] = quantise(qt, s->t[l][o]);
            } else {
                s->y[o] = a;
            }
        }
        in = s->h[l];
        W = b + nout;
    }
}

/* Relaxation time of the Smagorinsky model at one node (SI, "Implementing
 * the Smagorinsky Turbulence Model in LBM"), with dt = 1, c_s^2 = 1/3 and
 * filter width 1:
 *   Pi^neq_ab = sum_q c_qa c_qb (f_q - f^eq_q)
 *   S_ab      = -3 / (2 tau) Pi^neq_ab     (the printed factor 3 tau / 2 is
 *                                           taken as 3 / (2 tau), see below)
 *   |S|       = sqrt(2 S_ab S_ab)
 *   nu_eff    = (tau - 1/2) / 3 + C_s^2 |S|
 *   tau_eff   = 3 nu_eff + 1/2.
 * The strain rate follows from the Chapman-Enskog relation
 * Pi^neq = -2 rho c_s^2 tau S with rho taken as 1, as the SI does; tau is
 * the molecular relaxation time (explicit, not iterated). */
static double smagorinsky_tau(const orc_config *cfg, const lattice_t *L, const double g[],
                              const double geq[]) {
    double pi[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int q = 0; q < L->Q; ++q) {
        double d = g[q] - geq[q];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) pi[a][b] += L->c[q][a] * L->c[q][b] * d;
    }
    double ss = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double sab = -3.0 / (2.0 * cfg->tau) * pi[a][b];
            ss += sab * sab;
        }
    double smag = sqrt(2.0 * ss);
    double nu = (cfg->tau - 0.5) / 3.0 + cfg->smag_cs * cfg->smag_cs * smag;
    return 3.0 * nu + 0.5;
}

/* Collision of one node: post = g + P(Omega_BGK + (s_out/tau) y) + f^ext. */
static void collide_node(const orc_config *cfg, const lattice_t *L, const double *theta,
                         node_fwd *s, double post[]) {
    int Q = L->Q;
    double geq[QMAX], upd[QMAX];
    node_moments(L, s->g, &s->drho, s->j);
    equilibrium_dev(L, cfg->rho0, s->drho, s->j, geq);
    double tau = cfg->collision == 1 ? smagorinsky_tau(cfg, L, s->g, geq) : cfg->tau;
    for (int q = 0; q < Q; ++q) upd[q] = -(s->g[q] - geq[q]) / tau;
    if (cfg->hidden > 0) {
        net_shape n;
        get_net(Q, cfg->hidden, cfg->net, &n);
        mlp_forward(cfg, &n, theta, s);
        double k = cfg->out_scale / cfg->tau;
        for (int q = 0; q < Q; ++q) upd[q] += k * s->y[q];
    }
    project(L, upd);
    double fext[QMAX];
    for (int q = 0; q < Q; ++q) fext[q] = 0.0;
    if (s->F[0] != 0.0 || s->F[1] != 0.0 || s->F[2] != 0.0) {
        double rho = cfg->rho0 + s->drho;
        double js[3] = {s->j[0] + s->F[0], s->j[1] + s->F[1], s->j[2] + s->F[2]};
        double e0[QMAX], e1[QMAX];
        (void)rho;
        equilibrium_dev(L, cfg->rho0, s->drho, s->j, e0);
        equilibrium_dev(L, cfg->rho0, s->drho, js, e1); /* u + F/rho = (j + F)/rho */
        for (int q = 0; q < Q; ++q) fext[q] = e1[q] - e0[q];
    }
    for (int q = 0; q < Q; ++q) post[q] = s->g[q] + upd[q] + fext[q];
}

static int check_cfg(const orc_config *cfg, lattice_t *L) {
    if (get_lattice(cfg->lattice, L)) return -1;
    if (cfg->nx <= 0 || cfg->ny <= 0 || cfg->nz <= 0 || cfg->batch <= 0) return -1;
    if (L->D == 2 && cfg->nz != 1) return -1;
    net_shape n;
    if (get_net(L->Q, cfg->hidden, cfg->net, &n)) return -1;
    if (cfg->collision != 0 && cfg->collision != 1) return -1;
    if (cfg->collision == 1 && (cfg->hidden != 0 || !(cfg->smag_cs >= 0.0))) return -1;
    return 0;
}

static inline int64_t wrap(int64_t i, int64_t n) {
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

/* The parameters the network computes with.  With quant and quant_weights
 * set this is a copy of theta whose weights are rounded to the format (the
 * biases as given), and *eff is cfg with quant_weights cleared: the rounding
 * of each weight is done once per call instead of once per node.  Otherwise
 * theta itself and *eff = *cfg.  *owned receives the copy to free (or NULL). */
static const double *effective_theta(const orc_config *cfg, const double *theta,
                                     orc_config *eff, double **owned) {
    *eff = *cfg;
    *owned = NULL;
    if (!theta || cfg->hidden <= 0 || !cfg->quant || !cfg->quant_weights) return theta;
    lattice_t L;
    net_shape n;
    if (get_lattice(cfg->lattice, &L) || get_net(L.Q, cfg->hidden, cfg->net, &n)) return theta;
    int64_t P = orc_param_elems(cfg->lattice, cfg->hidden, cfg->net);
    double *t = (double *)malloc(sizeof(double) * (size_t)P);
    if (!t) return NULL;
    int64_t o = 0;
    for (int l = 0; l < n.nl; ++l) {
        int64_t nw = (int64_t)n.width[l + 1] * n.width[l];
        for (int64_t i = 0; i < nw; ++i) t[o + i] = qweight(cfg, theta[o + i]);
        for (int64_t i = 0; i < n.width[l + 1]; ++i) t[o + nw + i] = theta[o + nw + i];
        o += nw + n.width[l + 1];
    }
    eff->quant_weights = 0;
    *owned = t;
    return t;
}

/* Host threads of the node loops.  Every node is computed on its own, in
 * the same order of operations whatever the thread count; only the
 * parameter-gradient sum of the adjoint is split into per-thread partial
 * sums (added in thread order).  1 (the default) runs everything serially. */
static int g_threads = 1;

int orc_set_threads(int n) {
#ifdef _OPENMP
    g_threads = n < 1 ? 1 : n;
#else
    (void)n;
    g_threads = 1;
#endif
    return g_threads;
}

/* One full step (collide at every node, then periodic streaming), on
 * canonical pre-collision deviations.  g_out must not alias g_in.  The rows
 * (field, z, y) are independent: each node writes its own Q destinations
 * (streaming is a permutation). */
int orc_step(const orc_config *cfg_in, const double *theta_in, const double *g_in, double *g_out) {
    lattice_t L;
    if (check_cfg(cfg_in, &L)) return -1;
    orc_config cfg_eff;
    double *owned;
    const double *theta = effective_theta(cfg_in, theta_in, &cfg_eff, &owned);
    if (theta_in && !theta) return -2;
    const orc_config *cfg = &cfg_eff;
    const int64_t nx = cfg->nx, ny = cfg->ny, nz = cfg->nz, Q = L.Q;
    const int64_t N = nx * ny * nz, rows = (int64_t)cfg->batch * nz * ny;
    int err = 0;
#pragma omp parallel num_threads(g_threads)
    {
        node_fwd *s = (node_fwd *)malloc(sizeof(node_fwd));
        if (!s) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(static)
        for (int64_t r = 0; r < rows; ++r) {
            if (!s) continue;
            const int64_t b = r / (nz * ny), z = (r / ny) % nz, y = r % ny;
            const double *gi = g_in + b * Q * N;
            double *go = g_out + b * Q * N;
            for (int64_t x = 0; x < nx; ++x) {
                int64_t n = (z * ny + y) * nx + x;
                for (int q = 0; q < Q; ++q) s->g[q] = gi[q * N + n];
                body_force(cfg, (int)x, (int)y, (int)z, s->F);
                double post[QMAX];
                collide_node(cfg, &L, theta, s, post);
                /* stream: f_q(x + c_q, t + 1) = f_q^post(x, t) */
                for (int q = 0; q < Q; ++q) {
                    int64_t xd = wrap(x + L.c[q][0], nx);
                    int64_t yd = wrap(y + L.c[q][1], ny);
                    int64_t zd = wrap(z + L.c[q][2], nz);
                    go[q * N + (zd * ny + yd) * nx + xd] = post[q];
                }
            }
        }
        free(s);
    }
    free(owned);
    return err;
}

/* nsteps steps in place on g (uses one scratch copy). */
int orc_run(const orc_config *cfg, const double *theta, double *g, int nsteps) {
    lattice_t L;
    if (check_cfg(cfg, &L)) return -1;
    int64_t total = (int64_t)cfg->batch * L.Q * cfg->nx * cfg->ny * cfg->nz;
    double *tmp = (double *)malloc(sizeof(double) * total);
    if (!tmp) return -2;
    for (int t = 0; t < nsteps; ++t) {
        int rc = orc_step(cfg, theta, g, tmp);
        if (rc) { free(tmp); return rc; }
        memcpy(g, tmp, sizeof(double) * total);
    }
    free(tmp);
    return 0;
}

/* Post-collision populations of every node, without streaming (used by the
 * tests to pin the collision alone). */
int orc_collide(const orc_config *cfg_in, const double *theta_in, const double *g_in,
                double *post_out) {
    lattice_t L;
    if (check_cfg(cfg_in, &L)) return -1;
    orc_config cfg_eff;
    double *owned;
    const double *theta = effective_theta(cfg_in, theta_in, &cfg_eff, &owned);
    if (theta_in && !theta) return -2;
    const orc_config *cfg = &cfg_eff;
    const int64_t nx = cfg->nx, ny = cfg->ny, nz = cfg->nz, Q = L.Q, N = nx * ny * nz;
    const int64_t rows = (int64_t)cfg->batch * nz * ny;
    int err = 0;
#pragma omp parallel num_threads(g_threads)
    {
        node_fwd *s = (node_fwd *)malloc(sizeof(node_fwd));
        if (!s) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(static)
        for (int64_t r = 0; r < rows; ++r) {
            if (!s) continue;
            const int64_t b = r / (nz * ny), z = (r / ny) % nz, y = r % ny;
            for (int64_t x = 0; x < nx; ++x) {
                int64_t n = (z * ny + y) * nx + x;
                for (int q = 0; q < Q; ++q) s->g[q] = g_in[(b * Q + q) * N + n];
                body_force(cfg, (int)x, (int)y, (int)z, s->F);
                double post[QMAX];
                collide_node(cfg, &L, theta, s, post);
                for (int q = 0; q < Q; ++q) post_out[(b * Q + q) * N + n] = post[q];
            }
        }
        free(s);
    }
    free(owned);
    return err;
}

/* Equilibrium initial state from a density and a velocity field:
 * g_q = f^eq_q(rho, u) - w_q rho0 with j = rho u.
 * rho: [B][nz][ny][nx]; u: [B][D][nz][ny][nx]. */
int orc_init(const orc_config *cfg, const double *rho, const double *u, double *g) {
    lattice_t L;
    if (check_cfg(cfg, &L)) return -1;
    int64_t N = (int64_t)cfg->nx * cfg->ny * cfg->nz, Q = L.Q, D = L.D;
    for (int64_t b = 0; b < cfg->batch; ++b)
        for (int64_t n = 0; n < N; ++n) {
            double r = rho[b * N + n];
            double j[3] = {0, 0, 0};
            for (int a = 0; a < D; ++a) j[a] = r * u[(b * D + a) * N + n];
            double geq[QMAX];
            equilibrium_dev(&L, cfg->rho0, r - cfg->rho0, j, geq);
            for (int q = 0; q < Q; ++q) g[(b * Q + q) * N + n] = geq[q];
        }
    return 0;
}

/* Moments and diagnostics of canonical pre-collision populations.
 * rho = rho0 + sum g; reported velocity u = (j + F/2) / rho (the usual EDM
 * convention).  diag per field: [total mass, kinetic energy 1/2 sum rho|u|^2,
 * number of nodes with a non-finite population, 0]. */
int orc_moments(const orc_config *cfg, const double *g, double *rho, double *u, double *diag) {
    lattice_t L;
    if (check_cfg(cfg, &L)) return -1;
    int64_t nx = cfg->nx, ny = cfg->ny, nz = cfg->nz, Q = L.Q, D = L.D, N = nx * ny * nz;
    for (int64_t b = 0; b < cfg->batch; ++b) {
        double mass = 0.0, ke = 0.0, bad = 0.0;
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    int64_t n = (z * ny + y) * nx + x;
                    double gq[QMAX];
                    int finite = 1;
                    for (int q = 0; q < Q; ++q) {
                        gq[q] = g[(b * Q + q) * N + n];
                        if (!isfinite(gq[q])) finite = 0;
                    }
                    double drho, j[3], F[3];
                    node_moments(&L, gq, &drho, j);
                    body_force(cfg, (int)x, (int)y, (int)z, F);
                    double r = cfg->rho0 + drho;
                    double uu = 0.0;
                    for (int a = 0; a < D; ++a) {
                        double ua = (j[a] + 0.5 * F[a]) / r;
                        if (u) u[(b * D + a) * N + n] = ua;
                        uu += ua * ua;
                    }
                    if (rho) rho[b * N + n] = r;
                    if (!finite) { bad += 1.0; continue; }
                    mass += r;
                    ke += 0.5 * r * uu;
                }
        if (diag) {
            diag[4 * b + 0] = mass;
            diag[4 * b + 1] = ke;
            diag[4 * b + 2] = bad;
            diag[4 * b + 3] = 0.0;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of one step                                                       */
/* ------------------------------------------------------------------------ */

/* Reverse pass of collide_node.  mu = dL/d(post) of this node.  Adds
 * dL/dg into lam (length Q) and dL/dtheta into dtheta.  The derivative is
 * that of the exact-arithmetic map: rounding in the emulated mode is passed
 * straight through. */
static void collide_node_adjoint(const orc_config *cfg, const lattice_t *L, const double *theta,
                                 node_fwd *s, const double mu[], double lam[], double *dtheta) {
    int Q = L->Q;
    double tau = cfg->tau, rho0 = cfg->rho0;
    /* Forward recompute. */
    double post[QMAX];
    collide_node(cfg, L, theta, s, post);
    double drho = s->drho, rho = rho0 + drho;
    const double *j = s->j;
    double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];

    /* post = g + P(upd) + fext */
    for (int q = 0; q < Q; ++q) lam[q] += mu[q];
    double nu[QMAX];
    for (int q = 0; q < Q; ++q) nu[q] = mu[q];
    project(L, nu); /* P is symmetric */

    /* upd = -(g - geq)/tau + (s_out/tau) y */
    for (int q = 0; q < Q; ++q) lam[q] += -nu[q] / tau;
    /* geq_q = w_q [drho + 3 c.j + (9/2 (c.j)^2 - 3/2 |j|^2) / rho] */
    double Grho = 0.0, Gj[3] = {0, 0, 0};
    for (int q = 0; q < Q; ++q) {
        double a = nu[q] / tau; /* dL/dgeq_q */
        double cu = L->c[q][0] * u[0] + L->c[q][1] * u[1] + L->c[q][2] * u[2];
        Grho += a * L->w[q] * (1.0 - 4.5 * cu * cu + 1.5 * uu);
        for (int al = 0; al < 3; ++al)
            Gj[al] += a * L->w[q] * (3.0 * L->c[q][al] + 9.0 * cu * L->c[q][al] - 3.0 * u[al]);
    }
    /* fext_q = w_q [3 c.F + (9/2((c.(j+F))^2 - (c.j)^2) - 3/2(|j+F|^2 - |j|^2)) / rho] */
    const double *F = s->F;
    if (F[0] != 0.0 || F[1] != 0.0 || F[2] != 0.0) {
        double jF[3] = {j[0] + F[0], j[1] + F[1], j[2] + F[2]};
        double jj = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
        double jFjF = jF[0] * jF[0] + jF[1] * jF[1] + jF[2] * jF[2];
        for (int q = 0; q < Q; ++q) {
            double cj = L->c[q][0] * j[0] + L->c[q][1] * j[1] + L->c[q][2] * j[2];
            double cjF = L->c[q][0] * jF[0] + L->c[q][1] * jF[1] + L->c[q][2] * jF[2];
            double cF = L->c[q][0] * F[0] + L->c[q][1] * F[1] + L->c[q][2] * F[2];
            double num = 4.5 * (cjF * cjF - cj * cj) - 1.5 * (jFjF - jj);
            Grho += mu[q] * L->w[q] * (-num / (rho * rho));
            for (int al = 0; al < 3; ++al)
                Gj[al] += mu[q] * L->w[q] * (9.0 * cF * L->c[q][al] - 3.0 * F[al]) / rho;
        }
    }
    for (int q = 0; q < Q; ++q)
        lam[q] += Grho + Gj[0] * L->c[q][0] + Gj[1] * L->c[q][1] + Gj[2] * L->c[q][2];

    if (cfg->hidden > 0) {
        net_shape n;
        get_net(Q, cfg->hidden, cfg->net, &n);
        /* parameter offsets of every layer */
        int64_t off[NLMAX + 1];
        off[0] = 0;
        for (int l = 0; l < n.nl; ++l)
            off[l + 1] = off[l] + (int64_t)n.width[l + 1] * (n.width[l] + 1);
        double dz[HMAX], din[HMAX];
        double k = cfg->out_scale / tau;
        for (int q = 0; q < Q; ++q) dz[q] = k * nu[q]; /* output layer is linear */
        for (int l = n.nl - 1; l >= 0; --l) {
            int nin = n.width[l], nout = n.width[l + 1];
            const double *W = theta + off[l];
            double *dW = dtheta + off[l], *db = dW + (int64_t)nout * nin;
            const double *in = l == 0 ? s->x0 : s->h[l - 1];
            for (int o = 0; o < nout; ++o) {
                db[o] += dz[o];
                for (int i = 0; i < nin; ++i) dW[(int64_t)o * nin + i] += dz[o] * in[i];
            }
            for (int i = 0; i < nin; ++i) {
                double d = 0.0;
                for (int o = 0; o < nout; ++o) d += qweight(cfg, W[(int64_t)o * nin + i]) * dz[o];
                din[i] = d;
            }
            if (l > 0) {
                for (int i = 0; i < nin; ++i)
                    dz[i] = din[i] * activation_slope(n.leaky, s->pre[l - 1][i], s->t[l - 1][i]);
            } else {
                for (int i = 0; i < nin; ++i) lam[i] += din[i];
            }
        }
    }
}

/* Adjoint of orc_step.  g_n: canonical state at step n; lam_n1 = dL/dg^{n+1};
 * writes lam_n = dL/dg^n and adds dL/dtheta into dtheta (may be NULL when
 * hidden == 0).  Streaming is a permutation, so its transpose reads
 * lam^{n+1}_q(x + c_q).  The parameter gradient of each thread's rows is
 * summed separately and the partial sums are added in thread order. */
int orc_step_adjoint(const orc_config *cfg_in, const double *theta_in, const double *g_n,
                     const double *lam_n1, double *lam_n, double *dtheta) {
    lattice_t L;
    if (check_cfg(cfg_in, &L)) return -1;
    if (cfg_in->collision != 0) return -3; /* the adjoint covers the fixed-tau collision only */
    orc_config cfg_eff;
    double *owned;
    const double *theta = effective_theta(cfg_in, theta_in, &cfg_eff, &owned);
    if (theta_in && !theta) return -2;
    const orc_config *cfg = &cfg_eff;
    const int64_t nx = cfg->nx, ny = cfg->ny, nz = cfg->nz, Q = L.Q, N = nx * ny * nz;
    const int64_t rows = (int64_t)cfg->batch * nz * ny;
    const int64_t P = cfg->hidden > 0 ? orc_param_elems(cfg->lattice, cfg->hidden, cfg->net) : 0;
    const int nt = g_threads;
    double *part = P > 0 ? (double *)calloc((size_t)(P * nt), sizeof(double)) : NULL;
    if (P > 0 && !part) {
        free(owned);
        return -2;
    }
    int err = 0;
#pragma omp parallel num_threads(nt)
    {
#ifdef _OPENMP
        const int tid = omp_get_thread_num();
#else
        const int tid = 0;
#endif
        double *dth = part ? part + (int64_t)tid * P : NULL;
        node_fwd *s = (node_fwd *)malloc(sizeof(node_fwd));
        if (!s) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(static)
        for (int64_t r = 0; r < rows; ++r) {
            if (!s) continue;
            const int64_t b = r / (nz * ny), z = (r / ny) % nz, y = r % ny;
            for (int64_t x = 0; x < nx; ++x) {
                int64_t n = (z * ny + y) * nx + x;
                double mu[QMAX], lam[QMAX];
                for (int q = 0; q < Q; ++q) {
                    int64_t xd = wrap(x + L.c[q][0], nx);
                    int64_t yd = wrap(y + L.c[q][1], ny);
                    int64_t zd = wrap(z + L.c[q][2], nz);
                    mu[q] = lam_n1[(b * Q + q) * N + (zd * ny + yd) * nx + xd];
                    s->g[q] = g_n[(b * Q + q) * N + n];
                    lam[q] = 0.0;
                }
                body_force(cfg, (int)x, (int)y, (int)z, s->F);
                collide_node_adjoint(cfg, &L, theta, s, mu, lam, dth);
                for (int q = 0; q < Q; ++q) lam_n[(b * Q + q) * N + n] = lam[q];
            }
        }
        free(s);
    }
    if (part && dtheta && !err)
        for (int t = 0; t < nt; ++t)
            for (int64_t i = 0; i < P; ++i) dtheta[i] += part[(int64_t)t * P + i];
    free(part);
    free(owned);
    return err;
}

/* ------------------------------------------------------------------------ */
/* Velocity-MSE loss of the training configuration                           */
/* ------------------------------------------------------------------------ */

/* L = mean over fields, nodes and components of (u - u_target)^2 with
 * u = (j + F/2)/rho of the canonical state g.  Writes dL/dg when dLdg is not
 * NULL.  Returns L through *loss. */
int orc_loss_velocity_mse(const orc_config *cfg, const double *g, const double *u_target,
                          double *loss, double *dLdg) {
    lattice_t L;
    if (check_cfg(cfg, &L)) return -1;
    int64_t nx = cfg->nx, ny = cfg->ny, nz = cfg->nz, Q = L.Q, D = L.D, N = nx * ny * nz;
    double count = (double)cfg->batch * N * D;
    double acc = 0.0;
    for (int64_t b = 0; b < cfg->batch; ++b)
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    int64_t n = (z * ny + y) * nx + x;
                    double gq[QMAX], drho, j[3], F[3];
                    for (int q = 0; q < Q; ++q) gq[q] = g[(b * Q + q) * N + n];
                    node_moments(&L, gq, &drho, j);
                    body_force(cfg, (int)x, (int)y, (int)z, F);
                    double rho = cfg->rho0 + drho;
                    double e[3] = {0, 0, 0}, u[3] = {0, 0, 0};
                    for (int a = 0; a < D; ++a) {
                        u[a] = (j[a] + 0.5 * F[a]) / rho;
                        e[a] = u[a] - u_target[(b * D + a) * N + n];
                        acc += e[a] * e[a];
                    }
                    if (dLdg) {
                        /* du_a/dg_q = (c_qa - u_a) / rho */
                        for (int q = 0; q < Q; ++q) {
                            double d = 0.0;
                            for (int a = 0; a < D; ++a) d += e[a] * (L.c[q][a] - u[a]);
                            dLdg[(b * Q + q) * N + n] = 2.0 * d / (rho * count);
                        }
                    }
                }
    *loss = acc / count;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Training set of the SI ("Definition of the Training Dataset")             */
/* ------------------------------------------------------------------------ */

/* Sub-sampling filter: the coarse grid keeps one lattice point in every
 * `factor` along each axis (only along x and y for 2-D lattices).  cfg is
 * the fine configuration; g is canonical, g_coarse [B][Q][nz/f][ny/f][nx/f]. */
int orc_subsample(const orc_config *cfg, const double *g, int factor, double *g_coarse) {
    lattice_t L;
    if (check_cfg(cfg, &L) || factor < 1) return -1;
    int fz = L.D == 3 ? factor : 1;
    if (cfg->nx % factor || cfg->ny % factor || cfg->nz % fz) return -1;
    int64_t nx = cfg->nx, ny = cfg->ny, nz = cfg->nz, Q = L.Q;
    int64_t cx = nx / factor, cy = ny / factor, cz = nz / fz;
    for (int64_t b = 0; b < cfg->batch; ++b)
        for (int64_t q = 0; q < Q; ++q)
            for (int64_t z = 0; z < cz; ++z)
                for (int64_t y = 0; y < cy; ++y)
                    for (int64_t x = 0; x < cx; ++x)
                        g_coarse[(((b * Q + q) * cz + z) * cy + y) * cx + x] =
                            g[(((b * Q + q) * nz + z * fz) * ny + y * factor) * nx + x * factor];
    return 0;
}

/* Population loss of eq. nn-loss on a node subset S.  g_model and g_target
 * are canonical pre-collision states at the end of the trajectory; the
 * post-collision populations they come from are recovered by the inverse of
 * the streaming (reversed directions, SI Fig. 2):
 *   post_q(x) = g_q(x + c_q).
 * L = sum over x in S and q of (post_model_q(x) - post_target_q(x))^2.
 * nodes: flat indices b * N + (z ny + y) nx + x.  dLdg (may be NULL) is the
 * gradient with respect to g_model, zero outside the nodes' sources. */
int orc_loss_population_sse(const orc_config *cfg, const double *g_model, const double *g_target,
                            const int32_t *nodes, int n_nodes, double *loss, double *dLdg) {
    lattice_t L;
    if (check_cfg(cfg, &L)) return -1;
    int64_t nx = cfg->nx, ny = cfg->ny, nz = cfg->nz, Q = L.Q, N = nx * ny * nz;
    if (dLdg) memset(dLdg, 0, sizeof(double) * (size_t)(cfg->batch * Q * N));
    double acc = 0.0;
    for (int i = 0; i < n_nodes; ++i) {
        int64_t k = nodes[i];
        if (k < 0 || k >= cfg->batch * N) return -1;
        int64_t b = k / N, n = k % N;
        int64_t x = n % nx, y = (n / nx) % ny, z = n / (nx * ny);
        for (int q = 0; q < Q; ++q) {
            int64_t xs = wrap(x + L.c[q][0], nx), ys = wrap(y + L.c[q][1], ny);
            int64_t zs = wrap(z + L.c[q][2], nz);
            int64_t e = (b * Q + q) * N + (zs * ny + ys) * nx + xs;
            double d = g_model[e] - g_target[e];
            acc += d * d;
            if (dLdg) dLdg[e] += 2.0 * d;
        }
    }
    *loss = acc;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Turbulence diagnostics                                                    */
/* ------------------------------------------------------------------------ */

/* Eulerian structure functions (SI, eq. structure-fun-sm) along the lattice
 * axes: for l = 1..lmax and p = 1..pmax,
 *   S[p-1][l-1]    = < (u_a(x + l e_a) - u_a(x))^p >,
 *   Sabs[p-1][l-1] = < |u_a(x + l e_a) - u_a(x)|^p >,
 * the mean over every node, field and axis a < D (periodic); the increment
 * is the longitudinal one (along the separation).  u: canonical velocity
 * field [B][D][nz][ny][nx]. */
int orc_structure_functions(const orc_config *cfg, const double *u, int lmax, int pmax,
                            double *S, double *Sabs) {
    lattice_t L;
    if (check_cfg(cfg, &L) || lmax < 1 || pmax < 1) return -1;
    int64_t nx = cfg->nx, ny = cfg->ny, nz = cfg->nz, D = L.D, N = nx * ny * nz;
    int64_t dims[3] = {nx, ny, nz};
    double count = (double)cfg->batch * N * D;
    for (int l = 1; l <= lmax; ++l) {
        for (int p = 0; p < pmax; ++p) {
            S[p * lmax + l - 1] = 0.0;
            Sabs[p * lmax + l - 1] = 0.0;
        }
        for (int64_t b = 0; b < cfg->batch; ++b)
            for (int64_t a = 0; a < D; ++a)
                for (int64_t z = 0; z < nz; ++z)
                    for (int64_t y = 0; y < ny; ++y)
                        for (int64_t x = 0; x < nx; ++x) {
                            int64_t r[3] = {x, y, z};
                            r[a] = (r[a] + l) % dims[a];
                            double u0 = u[(b * D + a) * N + (z * ny + y) * nx + x];
                            double u1 = u[(b * D + a) * N + (r[2] * ny + r[1]) * nx + r[0]];
                            double d = u1 - u0, v = 1.0, va = 1.0;
                            for (int p = 0; p < pmax; ++p) {
                                v *= d;
                                va *= fabs(d);
                                S[p * lmax + l - 1] += v;
                                Sabs[p * lmax + l - 1] += va;
                            }
                        }
        for (int p = 0; p < pmax; ++p) {
            S[p * lmax + l - 1] /= count;
            Sabs[p * lmax + l - 1] /= count;
        }
    }
    return 0;
}

/* The MRT moment matrix M of the SI (section on the physical
 * interpretation of the model's action), for the D3Q19 order of Table S1;
 * rows are (rho, e, eps, jx, qx, jy, qy, jz, qz, pxx, pixx, pww, piww, pxy,
 * pyz, pxz, mx, my, mz). */
static const int MRT_M[19][19] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-30, -11, -11, -11, -11, -11, -11, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8},
    {12, -4, -4, -4, -4, -4, -4, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, -1, 0, 0, 0, 0, 1, -1, -1, -1, -1, 0, 0, 0, 0, 1, 1, 1, 1},
    {0, 4, 0, 0, 0, 0, -4, -1, -1, -1, -1, 0, 0, 0, 0, 1, 1, 1, 1},
    {0, 0, -1, 0, 0, 1, 0, -1, 0, 0, 1, -1, -1, 1, 1, -1, 0, 0, 1},
    {0, 0, 4, 0, 0, -4, 0, -1, 0, 0, 1, -1, -1, 1, 1, -1, 0, 0, 1},
    {0, 0, 0, -1, 1, 0, 0, 0, -1, 1, 0, -1, 1, -1, 1, 0, -1, 1, 0},
    {0, 0, 0, 4, -4, 0, 0, 0, -1, 1, 0, -1, 1, -1, 1, 0, -1, 1, 0},
    {0, 2, -1, -1, -1, -1, 2, 1, 1, 1, 1, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, -4, 2, 2, 2, 2, -4, 1, 1, 1, 1, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 0, 1, -1, -1, 1, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, -2, 2, 2, -2, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 0, 0, 1, 0, 0, -1, 0, 0, 0, 0, -1, 0, 0, 1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 0, 0, -1, 1, 0},
    {0, 0, 0, 0, 0, 0, 0, -1, 1, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 0, 0, 1, 0, 0, -1, -1, -1, 1, 1, 1, 0, 0, -1},
    {0, 0, 0, 0, 0, 0, 0, 0, -1, 1, 0, 1, -1, 1, -1, 0, -1, 1, 0},
};

int orc_mrt_matrix(int32_t *M) {
    for (int i = 0; i < 19; ++i)
        for (int q = 0; q < 19; ++q) M[i * 19 + q] = MRT_M[i][q];
    return 0;
}

/* Regression sums of the SI's moment analysis (D3Q19): with f_pre the
 * canonical state g_n, f_post the post-collision populations recovered from
 * the next state by the inverse streaming, post_q(x) = g_n1_q(x + c_q),
 *   m_diff = M (f_post - f_pre - f_ext),   m_neq = M (f_eq - f_pre),
 * and for every moment i the sums over nodes and fields of
 *   m_neq, m_diff, m_neq^2, m_neq m_diff, m_diff^2   -> stats[i][0..4]
 * (a relaxation m_diff = m_neq / tau_i has slope 1 / tau_i). */
int orc_mrt_moment_sums(const orc_config *cfg, const double *g_n, const double *g_n1,
                        double *stats) {
    lattice_t L;
    if (check_cfg(cfg, &L) || L.Q != 19) return -1;
    int64_t nx = cfg->nx, ny = cfg->ny, nz = cfg->nz, N = nx * ny * nz;
    for (int i = 0; i < 19 * 5; ++i) stats[i] = 0.0;
    for (int64_t b = 0; b < cfg->batch; ++b)
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    int64_t n = (z * ny + y) * nx + x;
                    double pre[19], post[19], geq[19], fext[19], F[3], drho, j[3];
                    for (int q = 0; q < 19; ++q) {
                        pre[q] = g_n[(b * 19 + q) * N + n];
                        int64_t xs = wrap(x + L.c[q][0], nx), ys = wrap(y + L.c[q][1], ny);
                        int64_t zs = wrap(z + L.c[q][2], nz);
                        post[q] = g_n1[(b * 19 + q) * N + (zs * ny + ys) * nx + xs];
                    }
                    node_moments(&L, pre, &drho, j);
                    equilibrium_dev(&L, cfg->rho0, drho, j, geq);
                    body_force(cfg, (int)x, (int)y, (int)z, F);
                    double js[3] = {j[0] + F[0], j[1] + F[1], j[2] + F[2]}, e1[19];
                    equilibrium_dev(&L, cfg->rho0, drho, js, e1);
                    for (int q = 0; q < 19; ++q) fext[q] = e1[q] - geq[q];
                    for (int i = 0; i < 19; ++i) {
                        double md = 0.0, mn = 0.0;
                        for (int q = 0; q < 19; ++q) {
                            md += MRT_M[i][q] * (post[q] - pre[q] - fext[q]);
                            mn += MRT_M[i][q] * (geq[q] - pre[q]);
                        }
                        stats[i * 5 + 0] += mn;
                        stats[i * 5 + 1] += md;
                        stats[i * 5 + 2] += mn * mn;
                        stats[i * 5 + 3] += mn * md;
                        stats[i * 5 + 4] += md * md;
                    }
                }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Optimiser and coarse-graining of the training workloads                   */
/* ------------------------------------------------------------------------ */

/* One step of Adam with the weight decay added to the gradient as an L2
 * term (the optimiser and the "weight decay rate" of Table S2), for n
 * parameters, step count t >= 1 after this update:
 *   g  = grad + wd p
 *   m  = beta1 m + (1 - beta1) g
 *   v  = beta2 v + (1 - beta2) g^2
 *   p  = p - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps). */
int orc_adam(int64_t n, double *p, const double *grad, double *m, double *v, double lr,
             double beta1, double beta2, double eps, double wd, int t) {
    if (n < 0 || t < 1) return -1;
    double bc1 = 1.0 - pow(beta1, t), bc2 = 1.0 - pow(beta2, t);
    for (int64_t i = 0; i < n; ++i) {
        double g = grad[i] + wd * p[i];
        m[i] = beta1 * m[i] + (1.0 - beta1) * g;
        v[i] = beta2 * v[i] + (1.0 - beta2) * g * g;
        double mhat = m[i] / bc1, vhat = v[i] / bc2;
        p[i] -= lr * mhat / (sqrt(vhat) + eps);
    }
    return 0;
}

/* Block average of [batch][channels][nz][ny][nx] fields over factor^D fine
 * nodes (D = 3 when nz > 1, else 2): the coarse-graining of the training
 * data of the two-dimensional workload. */
int orc_box_filter(int batch, int channels, int nx, int ny, int nz, int factor, const double *src,
                   double *dst) {
    if (batch < 1 || channels < 1 || nx < 1 || ny < 1 || nz < 1 || factor < 1) return -1;
    int fz = nz > 1 ? factor : 1;
    if (nx % factor || ny % factor || nz % fz) return -1;
    int64_t cx = nx / factor, cy = ny / factor, cz = nz / fz;
    double inv = 1.0 / ((double)factor * factor * fz);
    for (int64_t p = 0; p < (int64_t)batch * channels; ++p)
        for (int64_t z = 0; z < cz; ++z)
            for (int64_t y = 0; y < cy; ++y)
                for (int64_t x = 0; x < cx; ++x) {
                    double acc = 0.0;
                    for (int64_t dz = 0; dz < fz; ++dz)
                        for (int64_t dy = 0; dy < factor; ++dy)
                            for (int64_t dx = 0; dx < factor; ++dx)
                                acc += src[((p * nz + z * fz + dz) * ny + y * factor + dy) * nx +
                                           x * factor + dx];
                    dst[((p * cz + z) * cy + y) * cx + x] = acc * inv;
                }
    return 0;
}
