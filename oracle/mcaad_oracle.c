/*
 * FP64 CPU oracle for the two-pass Monte Carlo adjoint gradient of
 *     G = 1/2 * sum_i (E y_i - C_i)^2                      (paper, eq. 241118A)
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
 * calls this file: it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the GPU library against a plain,
 * slow, obviously correct implementation.  It shares no code, header, table
 * or constant generator with the HIP library.
 *
 * What it computes, in the paper's order:
 *   - the forward algorithm F : R^{M+N} -> R^m (paper, section on the
 *     calculation of the gradient of G)
 *     for one path: an Euler-discretised SDE driven by N independent normals,
 *     producing the m payoffs y_i of that path;
 *   - the Monte Carlo expectation E y ~ (1/P) sum_k y(w_k) (paper, remarks on
 *     Monte Carlo simulations, eq. 1211A);
 *   - the gradient dG/dx_j = E( sum_i (E y_i - C_i) dy_i/dx_j ) by the
 *     paper's three-step algorithm: step 1 computes E y_i, step 2 fixes a path
 *     and runs the reverse algorithm seeded with lambda_i = E y_i - C_i
 *     (eq. 0711A), step 3 sums over paths.
 * and, for the pins only, two independent ways to get the same derivatives:
 *   - forward tangent mode (dE y_i / dtheta_j, the Jacobian), and
 *   - the complex-step derivative (Squire & Trapp 1998) of the forward sweep.
 *
 * Random numbers: the paper only says F takes N independent random variables.
 * They are drawn here from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 * counter (floor(q/4), path, instance, 0), key (seed lo, seed hi), where q is
 * the index of the normal within the path; words map to uniforms
 * u = ((w >> 9) + 0.5) * 2^-23 (exactly representable in FP32 and FP64,
 * so both precisions see the same uniforms) and pairs of uniforms to normals by
 * Box-Muller: rho = sqrt(-2 ln u0), z0 = rho cos(2 pi u1), z1 = rho sin(2 pi u1).
 *
 * Models (0 to 3 step the log-price x = ln(S/S0): the paper's Euler scheme read
 * as log-Euler; 4 takes it literally on S; payoffs are discounted calls):
 *   0  Black-Scholes GBM, theta = (sigma)
 *   1  Heston with full truncation, theta = (kappa, theta_bar, xi, rho, v0);
 *      the paper's test model with the leverage function set to one
 *   2  local volatility, theta = node values of a bilinear grid in (t, S)
 *   3  Heston stochastic local volatility (the paper's test model):
 *      dS/S = r dt + L(t,S) sqrt(v) dW1 with Heston's v, theta = (kappa,
 *      theta_bar, xi, rho, v0, leverage node values L[a][k]); L piecewise
 *      constant in t, linear across the spot nodes
 *   4  Black-Scholes GBM with the Euler scheme applied to the SDE as written
 *      in S (section "Test on the Heston SLV model calibration": a standard
 *      Euler discretisation of dS = mu S dt + sigma S dW), theta = (sigma):
 *      S_{n+1} = S_n (1 + r h + sigma sqrt(h) z_n); the state is S itself
 *
 * Sums over paths are taken in path order with Neumaier compensation.
 * Per-path work runs in parallel (OpenMP) into per-path buffers; only the
 * summation, which is sequential, fixes the order of floating point
 * operations.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

enum { ORC_BS = 0, ORC_HESTON = 1, ORC_LV = 2, ORC_SLV = 3, ORC_BSE = 4 };

typedef struct {
    int32_t model;
    int32_t n_params;   /* M */
    int32_t n_instr;    /* m */
    int32_t n_steps;    /* N */
    int64_t n_paths;    /* P */
    uint64_t seed;
    uint32_t inst;      /* third counter word: instance / draw index */
    uint32_t pad_;
    double s0, rate, t_max;
    const int32_t *instr_step;   /* [m], maturity step in 1..N */
    const double *instr_strike;  /* [m] */
    int32_t n_t_nodes, n_k_nodes;
    const double *t_nodes;       /* [n_t_nodes], increasing */
    const double *k_nodes;       /* [n_k_nodes], increasing */
    double sqrt_eps;             /* Heston: 0 = plain full truncation; > 0 = C1 square root below eps */
} orc_problem;

/* ------------------------------------------------------------------ */
/* Philox4x32-10, from the published definition (Salmon et al. 2011).  */
/* ------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;   /* Weyl key schedule */
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The same for n counters (ctr and out [n][4]) under one key, one after another. */
void orc_philox_many(const uint32_t *ctr, int64_t n, const uint32_t key[2], uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

static double orc_uniform(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* Four normals from one Philox call: pairs (u0,u1) and (u2,u3). */
static void orc_four_normals(uint64_t seed, uint32_t inst, uint32_t path, uint32_t call, double z[4])
{
    const double two_pi = 6.283185307179586476925286766559;
    uint32_t ctr[4] = {call, path, inst, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    for (int pair = 0; pair < 2; ++pair) {
        double u0 = orc_uniform(w[2 * pair]);
        double u1 = orc_uniform(w[2 * pair + 1]);
        double rho = sqrt(-2.0 * log(u0));
        z[2 * pair] = rho * cos(two_pi * u1);
        z[2 * pair + 1] = rho * sin(two_pi * u1);
    }
}

/* Normal number q of one path, with a one-call cache. */
typedef struct {
    uint64_t seed;
    uint32_t inst, path, call;
    int valid;
    double z[4];
} orc_rng;

static void rng_init(orc_rng *g, const orc_problem *pb, uint32_t path)
{
    g->seed = pb->seed; g->inst = pb->inst; g->path = path; g->call = 0; g->valid = 0;
}

static double rng_normal(orc_rng *g, uint32_t q)
{
    uint32_t call = q >> 2;
    if (!g->valid || g->call != call) {
        orc_four_normals(g->seed, g->inst, g->path, call, g->z);
        g->call = call; g->valid = 1;
    }
    return g->z[q & 3u];
}

/* Normals q0 .. q0+n-1 of one path (for tests of the random stream). */
void orc_normals(uint64_t seed, uint32_t inst, uint32_t path, uint32_t q0, int32_t n, double *out)
{
    orc_rng g; g.seed = seed; g.inst = inst; g.path = path; g.call = 0; g.valid = 0;
    for (int32_t i = 0; i < n; ++i) out[i] = rng_normal(&g, q0 + (uint32_t)i);
}

/* ------------------------------------------------------------------ */
/* Problem constants, per-step instrument lists                        */
/* ------------------------------------------------------------------ */
typedef struct {
    double h, sq, r, s0;
    int N, m, M, d;       /* d = normals per step */
    int *date_begin;      /* [N+2]: instruments maturing at step n are ids[date_begin[n] .. date_begin[n+1]) */
    int *ids;             /* [m] */
    double *disc;         /* [m], exp(-r * n_i * h) */
    const double *strike; /* [m] */
} orc_consts;

static int consts_make(const orc_problem *pb, orc_consts *c)
{
    c->date_begin = NULL; c->ids = NULL; c->disc = NULL;
    if (!pb || pb->n_steps <= 0 || pb->n_instr <= 0 || pb->n_paths <= 0 || pb->n_params <= 0) return ORC_EINVAL;
    if (pb->n_paths > (int64_t)1 << 32) return ORC_EINVAL;
    if (!pb->instr_step || !pb->instr_strike) return ORC_EINVAL;
    int N = pb->n_steps, m = pb->n_instr;
    for (int i = 0; i < m; ++i)
        if (pb->instr_step[i] < 1 || pb->instr_step[i] > N) return ORC_EINVAL;
    if ((pb->model == ORC_BS || pb->model == ORC_BSE) && pb->n_params != 1) return ORC_EINVAL;
    if (pb->model == ORC_HESTON && pb->n_params != 5) return ORC_EINVAL;
    if (pb->model == ORC_LV) {
        if (pb->n_t_nodes < 2 || pb->n_k_nodes < 2 || !pb->t_nodes || !pb->k_nodes) return ORC_EINVAL;
        if (pb->n_params != pb->n_t_nodes * pb->n_k_nodes) return ORC_EINVAL;
    }
    if (pb->model == ORC_SLV) {
        if (pb->n_t_nodes < 1 || pb->n_k_nodes < 2 || !pb->t_nodes || !pb->k_nodes) return ORC_EINVAL;
        if (pb->n_params != 5 + pb->n_t_nodes * pb->n_k_nodes) return ORC_EINVAL;
    }
    if (pb->model < 0 || pb->model > 4) return ORC_EINVAL;
    if (!(pb->sqrt_eps >= 0.0)) return ORC_EINVAL;
    c->h = pb->t_max / N;
    c->sq = sqrt(c->h);
    c->r = pb->rate;
    c->s0 = pb->s0;
    c->N = N; c->m = m; c->M = pb->n_params;
    c->d = (pb->model == ORC_HESTON || pb->model == ORC_SLV) ? 2 : 1;
    c->date_begin = (int *)calloc((size_t)N + 2, sizeof(int));
    c->ids = (int *)malloc(sizeof(int) * (size_t)m);
    c->disc = (double *)malloc(sizeof(double) * (size_t)m);
    if (!c->date_begin || !c->ids || !c->disc) return ORC_ENOMEM;
    for (int i = 0; i < m; ++i) c->date_begin[pb->instr_step[i] + 1]++;
    for (int n = 0; n <= N; ++n) c->date_begin[n + 1] += c->date_begin[n];
    int *fill = (int *)calloc((size_t)N + 1, sizeof(int));
    if (!fill) return ORC_ENOMEM;
    for (int i = 0; i < m; ++i) {
        int n = pb->instr_step[i];
        c->ids[c->date_begin[n] + fill[n]++] = i;
    }
    free(fill);
    for (int i = 0; i < m; ++i) c->disc[i] = exp(-pb->rate * pb->instr_step[i] * c->h);
    c->strike = pb->instr_strike;
    return ORC_OK;
}

static void consts_free(orc_consts *c)
{
    free(c->date_begin); free(c->ids); free(c->disc);
}

/* The spot price of state x: x itself for model 4 (Euler on S), S0 e^x otherwise. */
static double spot_of(const orc_problem *pb, const orc_consts *c, double x)
{
    return pb->model == ORC_BSE ? x : c->s0 * exp(x);
}

/* The state at step 0: S0 for model 4, log-price 0 otherwise. */
static double state0(const orc_problem *pb, const orc_consts *c)
{
    return pb->model == ORC_BSE ? c->s0 : 0.0;
}

/* Diffusion coefficient of the variance, s(v+) with v+ = max(v, 0).
 * eps = 0: s = sqrt(v+), the plain full-truncation scheme.
 * eps > 0: below eps the square root is replaced by the quadratic
 * v (3 - v/eps) / (2 sqrt(eps)), which meets sqrt(v) with equal value and
 * slope at v = eps, so ds/dv stays bounded by 3 / (2 sqrt(eps)). */
static double heston_s(double vp, double eps)
{
    if (vp <= 0.0) return 0.0;
    if (vp < eps) return vp * (3.0 - vp / eps) / (2.0 * sqrt(eps));
    return sqrt(vp);
}

static double heston_ds(double vp, double eps)
{
    if (vp <= 0.0) return 0.0;
    if (vp < eps) return (3.0 - 2.0 * vp / eps) / (2.0 * sqrt(eps));
    return 0.5 / sqrt(vp);
}

static double complex heston_s_c(double complex vp, double eps)
{
    double re = creal(vp);
    if (re <= 0.0) return 0.0;
    if (re < eps) return vp * (3.0 - vp / eps) / (2.0 * sqrt(eps));
    return csqrt(vp);
}

/* ------------------------------------------------------------------ */
/* Local volatility: bilinear interpolation in (t, S) on fixed nodes.  */
/* Flat extrapolation outside the node box; a point on a node line     */
/* belongs to the cell to its right.                                   */
/* ------------------------------------------------------------------ */
typedef struct {
    int a, b;           /* lower-left node */
    double al, be;      /* clamped weights in t and S */
    int s_inside;       /* 1 when K_0 <= S <= K_last (dsigma/dS is the cell slope) */
} lv_cell;

static int lv_find(const double *nodes, int n, double v)
{
    int j = 0;
    while (j + 1 < n - 1 && nodes[j + 1] <= v) ++j;
    return j;
}

static lv_cell lv_locate(const orc_problem *pb, double t, double S)
{
    lv_cell c;
    const double *T = pb->t_nodes, *K = pb->k_nodes;
    int nT = pb->n_t_nodes, nK = pb->n_k_nodes;
    c.a = lv_find(T, nT, t);
    double al = (t - T[c.a]) / (T[c.a + 1] - T[c.a]);
    c.al = al < 0.0 ? 0.0 : (al > 1.0 ? 1.0 : al);
    c.b = lv_find(K, nK, S);
    double be = (S - K[c.b]) / (K[c.b + 1] - K[c.b]);
    c.be = be < 0.0 ? 0.0 : (be > 1.0 ? 1.0 : be);
    c.s_inside = (S >= K[0] && S <= K[nK - 1]);
    return c;
}

static double lv_sigma(const orc_problem *pb, const double *grid, lv_cell c)
{
    int nK = pb->n_k_nodes;
    double s00 = grid[c.a * nK + c.b], s01 = grid[c.a * nK + c.b + 1];
    double s10 = grid[(c.a + 1) * nK + c.b], s11 = grid[(c.a + 1) * nK + c.b + 1];
    return (1.0 - c.al) * (1.0 - c.be) * s00 + (1.0 - c.al) * c.be * s01
         + c.al * (1.0 - c.be) * s10 + c.al * c.be * s11;
}

static double lv_dsigma_dS(const orc_problem *pb, const double *grid, lv_cell c)
{
    if (!c.s_inside) return 0.0;
    int nK = pb->n_k_nodes;
    double s00 = grid[c.a * nK + c.b], s01 = grid[c.a * nK + c.b + 1];
    double s10 = grid[(c.a + 1) * nK + c.b], s11 = grid[(c.a + 1) * nK + c.b + 1];
    double dK = pb->k_nodes[c.b + 1] - pb->k_nodes[c.b];
    return ((1.0 - c.al) * (s01 - s00) + c.al * (s11 - s10)) / dK;
}

/* ------------------------------------------------------------------ */
/* Heston stochastic local volatility: dS/S = r dt + L(t,S) sqrt(v) dW1, */
/* v as in Heston.  theta = (kappa, theta_bar, xi, rho, v0, L[a][k]).    */
/* L is piecewise constant in t: the row a of time t is the number of    */
/* nodes t_i <= t (capped at the last row), so row a governs the time    */
/* up to node a; across the spot nodes it is linear, flat outside.       */
/* ------------------------------------------------------------------ */
typedef struct {
    int a, b;
    double be;
    int s_inside;
} slv_cell;

static slv_cell slv_locate(const orc_problem *pb, double t, double S)
{
    slv_cell c;
    int nT = pb->n_t_nodes, nK = pb->n_k_nodes;
    int a = 0;
    while (a < nT && pb->t_nodes[a] <= t) ++a;
    c.a = a < nT - 1 ? a : nT - 1;
    c.b = lv_find(pb->k_nodes, nK, S);
    double be = (S - pb->k_nodes[c.b]) / (pb->k_nodes[c.b + 1] - pb->k_nodes[c.b]);
    c.be = be < 0.0 ? 0.0 : (be > 1.0 ? 1.0 : be);
    c.s_inside = (S >= pb->k_nodes[0] && S <= pb->k_nodes[nK - 1]);
    return c;
}

/* L at the cell and dL/dS; lev = theta + 5 */
static double slv_lev(const orc_problem *pb, const double *lev, slv_cell c)
{
    int nK = pb->n_k_nodes;
    return (1.0 - c.be) * lev[c.a * nK + c.b] + c.be * lev[c.a * nK + c.b + 1];
}

static double slv_dlev_dS(const orc_problem *pb, const double *lev, slv_cell c)
{
    if (!c.s_inside) return 0.0;
    int nK = pb->n_k_nodes;
    return (lev[c.a * nK + c.b + 1] - lev[c.a * nK + c.b]) / (pb->k_nodes[c.b + 1] - pb->k_nodes[c.b]);
}

/* ------------------------------------------------------------------ */
/* One path: forward algorithm F (payoffs only)                        */
/* ------------------------------------------------------------------ */
static void path_forward(const orc_problem *pb, const orc_consts *c, const double *th, uint32_t p, double *y)
{
    orc_rng g; rng_init(&g, pb, p);
    const double h = c->h, sq = c->sq, r = c->r;
    double x = state0(pb, c);
    const int hv = pb->model == ORC_HESTON || pb->model == ORC_SLV;   /* has a variance process */
    double v = hv ? th[4] : 0.0;
    const double rhop = hv ? sqrt(1.0 - th[3] * th[3]) : 0.0;
    for (int n = 0; n < c->N; ++n) {
        if (pb->model == ORC_BS) {
            double sig = th[0];
            double z = rng_normal(&g, (uint32_t)n);
            x = x + (r - 0.5 * sig * sig) * h + sig * sq * z;
        } else if (pb->model == ORC_HESTON) {
            double kap = th[0], thb = th[1], xi = th[2], rho = th[3];
            double z1 = rng_normal(&g, (uint32_t)(2 * n));
            double z2 = rng_normal(&g, (uint32_t)(2 * n + 1));
            double vp = v > 0.0 ? v : 0.0;
            double s = heston_s(vp, pb->sqrt_eps);
            double w = rho * z1 + rhop * z2;
            double xn = x + (r - 0.5 * vp) * h + s * sq * z1;
            double vn = v + kap * (thb - vp) * h + xi * s * sq * w;
            x = xn; v = vn;
        } else if (pb->model == ORC_SLV) {
            double kap = th[0], thb = th[1], xi = th[2], rho = th[3];
            double z1 = rng_normal(&g, (uint32_t)(2 * n));
            double z2 = rng_normal(&g, (uint32_t)(2 * n + 1));
            double vp = v > 0.0 ? v : 0.0;
            double s = heston_s(vp, pb->sqrt_eps);
            double w = rho * z1 + rhop * z2;
            double L = slv_lev(pb, th + 5, slv_locate(pb, n * h, c->s0 * exp(x)));
            double xn = x + (r - 0.5 * L * L * vp) * h + L * s * sq * z1;
            double vn = v + kap * (thb - vp) * h + xi * s * sq * w;
            x = xn; v = vn;
        } else if (pb->model == ORC_BSE) {
            double sig = th[0];
            double z = rng_normal(&g, (uint32_t)n);
            x = x * (1.0 + r * h + sig * sq * z);
        } else {
            double z = rng_normal(&g, (uint32_t)n);
            double S = c->s0 * exp(x);
            lv_cell cell = lv_locate(pb, n * h, S);
            double sig = lv_sigma(pb, th, cell);
            x = x + (r - 0.5 * sig * sig) * h + sig * sq * z;
        }
        for (int k = c->date_begin[n + 1]; k < c->date_begin[n + 2]; ++k) {
            int i = c->ids[k];
            double S = spot_of(pb, c, x);
            double pay = S - c->strike[i];
            y[i] = c->disc[i] * (pay > 0.0 ? pay : 0.0);
        }
    }
}

/* ------------------------------------------------------------------ */
/* One path: forward storing the trajectory, then the reverse sweep R  */
/* seeded with lam[i] (already divided by P). thbar[M] is overwritten. */
/* ------------------------------------------------------------------ */
static void path_reverse(const orc_problem *pb, const orc_consts *c, const double *th, uint32_t p,
                         const double *lam, double *thbar, double *work)
{
    const int N = c->N, M = c->M;
    const double h = c->h, sq = c->sq, r = c->r;
    double *xs = work;              /* x_0..x_N   */
    double *vs = xs + (N + 1);      /* v_0..v_N   */
    double *z1s = vs + (N + 1);     /* z1_0..z1_{N-1} */
    double *z2s = z1s + N;          /* z2_0..z2_{N-1} */
    orc_rng g; rng_init(&g, pb, p);
    const int hv = pb->model == ORC_HESTON || pb->model == ORC_SLV;
    const double rhop = hv ? sqrt(1.0 - th[3] * th[3]) : 0.0;

    /* forward, recording the states and normals of every step */
    xs[0] = state0(pb, c);
    vs[0] = hv ? th[4] : 0.0;
    for (int n = 0; n < N; ++n) {
        double x = xs[n];
        if (pb->model == ORC_BS) {
            double sig = th[0];
            double z = rng_normal(&g, (uint32_t)n);
            z1s[n] = z;
            xs[n + 1] = x + (r - 0.5 * sig * sig) * h + sig * sq * z;
        } else if (pb->model == ORC_HESTON) {
            double kap = th[0], thb = th[1], xi = th[2], rho = th[3];
            double z1 = rng_normal(&g, (uint32_t)(2 * n));
            double z2 = rng_normal(&g, (uint32_t)(2 * n + 1));
            double v = vs[n];
            double vp = v > 0.0 ? v : 0.0;
            double s = heston_s(vp, pb->sqrt_eps);
            double w = rho * z1 + rhop * z2;
            z1s[n] = z1; z2s[n] = z2;
            xs[n + 1] = x + (r - 0.5 * vp) * h + s * sq * z1;
            vs[n + 1] = v + kap * (thb - vp) * h + xi * s * sq * w;
        } else if (pb->model == ORC_SLV) {
            double kap = th[0], thb = th[1], xi = th[2], rho = th[3];
            double z1 = rng_normal(&g, (uint32_t)(2 * n));
            double z2 = rng_normal(&g, (uint32_t)(2 * n + 1));
            double v = vs[n];
            double vp = v > 0.0 ? v : 0.0;
            double s = heston_s(vp, pb->sqrt_eps);
            double w = rho * z1 + rhop * z2;
            double L = slv_lev(pb, th + 5, slv_locate(pb, n * h, c->s0 * exp(x)));
            z1s[n] = z1; z2s[n] = z2;
            xs[n + 1] = x + (r - 0.5 * L * L * vp) * h + L * s * sq * z1;
            vs[n + 1] = v + kap * (thb - vp) * h + xi * s * sq * w;
        } else if (pb->model == ORC_BSE) {
            double sig = th[0];
            double z = rng_normal(&g, (uint32_t)n);
            z1s[n] = z;
            xs[n + 1] = x * (1.0 + r * h + sig * sq * z);
        } else {
            double z = rng_normal(&g, (uint32_t)n);
            z1s[n] = z;
            double S = c->s0 * exp(x);
            lv_cell cell = lv_locate(pb, n * h, S);
            double sig = lv_sigma(pb, th, cell);
            xs[n + 1] = x + (r - 0.5 * sig * sig) * h + sig * sq * z;
        }
    }

    /* reverse sweep */
    for (int j = 0; j < M; ++j) thbar[j] = 0.0;
    double xb = 0.0, vb = 0.0;  /* adjoints of x_{n+1}, v_{n+1} */
    for (int n = N - 1; n >= 0; --n) {
        /* payoff adjoints enter at the maturity step n+1: dy_i/dx = D_i 1{S>K_i} S
         * for the log-price state, D_i 1{S>K_i} for the spot itself (model 4) */
        double Sn1 = spot_of(pb, c, xs[n + 1]);
        double dSdx = pb->model == ORC_BSE ? 1.0 : Sn1;
        for (int k = c->date_begin[n + 1]; k < c->date_begin[n + 2]; ++k) {
            int i = c->ids[k];
            if (Sn1 > c->strike[i]) xb += lam[i] * c->disc[i] * dSdx;
        }
        if (pb->model == ORC_BS) {
            double sig = th[0];
            /* x_{n+1} = x_n + (r - sig^2/2) h + sig sq z */
            thbar[0] += xb * (-sig * h + sq * z1s[n]);
            /* xb unchanged: dx_{n+1}/dx_n = 1 */
        } else if (pb->model == ORC_HESTON) {
            double kap = th[0], thb = th[1], xi = th[2], rho = th[3];
            double v = vs[n];
            double vp = v > 0.0 ? v : 0.0;
            double s = heston_s(vp, pb->sqrt_eps);
            double z1 = z1s[n], z2 = z2s[n];
            double w = rho * z1 + rhop * z2;
            double a = xb, b = vb;
            double sbar = a * sq * z1 + b * xi * sq * w;
            double vpbar = -0.5 * a * h - b * kap * h + sbar * heston_ds(vp, pb->sqrt_eps);
            thbar[0] += b * (thb - vp) * h;
            thbar[1] += b * kap * h;
            thbar[2] += b * s * sq * w;
            thbar[3] += b * xi * s * sq * (z1 - rho * z2 / rhop);
            xb = a;
            vb = b + (v > 0.0 ? vpbar : 0.0);
        } else if (pb->model == ORC_SLV) {
            /* x_{n+1} = x + (r - L^2 v+/2) h + L s sq z1, v_{n+1} as Heston, L = L(t_n, S_n) */
            double kap = th[0], thb = th[1], xi = th[2], rho = th[3];
            double v = vs[n];
            double vp = v > 0.0 ? v : 0.0;
            double s = heston_s(vp, pb->sqrt_eps);
            double z1 = z1s[n], z2 = z2s[n];
            double w = rho * z1 + rhop * z2;
            double S = c->s0 * exp(xs[n]);
            slv_cell cell = slv_locate(pb, n * h, S);
            double L = slv_lev(pb, th + 5, cell);
            double a = xb, b = vb;
            double Lbar = a * (-L * vp * h + s * sq * z1);
            double sbar = a * L * sq * z1 + b * xi * sq * w;
            double vpbar = -0.5 * a * L * L * h - b * kap * h + sbar * heston_ds(vp, pb->sqrt_eps);
            thbar[0] += b * (thb - vp) * h;
            thbar[1] += b * kap * h;
            thbar[2] += b * s * sq * w;
            thbar[3] += b * xi * s * sq * (z1 - rho * z2 / rhop);
            int nK = pb->n_k_nodes;
            thbar[5 + cell.a * nK + cell.b] += Lbar * (1.0 - cell.be);
            thbar[5 + cell.a * nK + cell.b + 1] += Lbar * cell.be;
            xb = a + Lbar * slv_dlev_dS(pb, th + 5, cell) * S;
            vb = b + (v > 0.0 ? vpbar : 0.0);
        } else if (pb->model == ORC_BSE) {
            /* S_{n+1} = S_n (1 + r h + sig sq z) */
            double sig = th[0], z = z1s[n];
            thbar[0] += xb * xs[n] * sq * z;
            xb = xb * (1.0 + r * h + sig * sq * z);
        } else {
            double x = xs[n];
            double S = c->s0 * exp(x);
            lv_cell cell = lv_locate(pb, n * h, S);
            double sig = lv_sigma(pb, th, cell);
            double sigbar = xb * (-sig * h + sq * z1s[n]);
            int nK = pb->n_k_nodes;
            thbar[cell.a * nK + cell.b] += sigbar * (1.0 - cell.al) * (1.0 - cell.be);
            thbar[cell.a * nK + cell.b + 1] += sigbar * (1.0 - cell.al) * cell.be;
            thbar[(cell.a + 1) * nK + cell.b] += sigbar * cell.al * (1.0 - cell.be);
            thbar[(cell.a + 1) * nK + cell.b + 1] += sigbar * cell.al * cell.be;
            xb = xb + sigbar * lv_dsigma_dS(pb, th, cell) * S;
        }
    }
    if (hv) thbar[4] += vb;  /* v_0 = theta[4] */
}

/* ------------------------------------------------------------------ */
/* One path: forward tangent mode, dy[i*M + j] = dy_i/dtheta_j          */
/* ------------------------------------------------------------------ */
static void path_tangent(const orc_problem *pb, const orc_consts *c, const double *th, uint32_t p,
                         double *y, double *dy, double *work)
{
    const int N = c->N, M = c->M;
    const double h = c->h, sq = c->sq, r = c->r;
    double *xd = work;        /* dx/dtheta_j */
    double *vd = work + M;    /* dv/dtheta_j */
    double *sd = work + 2 * M;/* dsigma/dtheta_j (LV), dL/dtheta_j (SLV) */
    orc_rng g; rng_init(&g, pb, p);
    double x = state0(pb, c), v = 0.0;
    for (int j = 0; j < M; ++j) { xd[j] = 0.0; vd[j] = 0.0; }
    double rhop = 0.0;
    if (pb->model == ORC_HESTON || pb->model == ORC_SLV) { v = th[4]; vd[4] = 1.0; rhop = sqrt(1.0 - th[3] * th[3]); }
    for (int n = 0; n < N; ++n) {
        if (pb->model == ORC_BS) {
            double sig = th[0];
            double z = rng_normal(&g, (uint32_t)n);
            xd[0] += (-sig * h + sq * z);
            x = x + (r - 0.5 * sig * sig) * h + sig * sq * z;
        } else if (pb->model == ORC_HESTON) {
            double kap = th[0], thb = th[1], xi = th[2], rho = th[3];
            double z1 = rng_normal(&g, (uint32_t)(2 * n));
            double z2 = rng_normal(&g, (uint32_t)(2 * n + 1));
            double vp = v > 0.0 ? v : 0.0;
            double s = heston_s(vp, pb->sqrt_eps);
            double dsdv = heston_ds(vp, pb->sqrt_eps);
            double w = rho * z1 + rhop * z2;
            double dw_drho = z1 - rho * z2 / rhop;
            for (int j = 0; j < 5; ++j) {
                double vpd = v > 0.0 ? vd[j] : 0.0;
                double sdj = dsdv * vpd;
                double wd = j == 3 ? dw_drho : 0.0;
                double kapd = j == 0 ? 1.0 : 0.0, thbd = j == 1 ? 1.0 : 0.0, xid = j == 2 ? 1.0 : 0.0;
                double xnd = xd[j] - 0.5 * vpd * h + sdj * sq * z1;
                double vnd = vd[j] + kapd * (thb - vp) * h + kap * (thbd - vpd) * h
                           + xid * s * sq * w + xi * sdj * sq * w + xi * s * sq * wd;
                xd[j] = xnd; vd[j] = vnd;
            }
            double xn = x + (r - 0.5 * vp) * h + s * sq * z1;
            double vn = v + kap * (thb - vp) * h + xi * s * sq * w;
            x = xn; v = vn;
        } else if (pb->model == ORC_SLV) {
            double kap = th[0], thb = th[1], xi = th[2], rho = th[3];
            double z1 = rng_normal(&g, (uint32_t)(2 * n));
            double z2 = rng_normal(&g, (uint32_t)(2 * n + 1));
            double vp = v > 0.0 ? v : 0.0;
            double s = heston_s(vp, pb->sqrt_eps);
            double dsdv = heston_ds(vp, pb->sqrt_eps);
            double w = rho * z1 + rhop * z2;
            double dw_drho = z1 - rho * z2 / rhop;
            double S = c->s0 * exp(x);
            slv_cell cell = slv_locate(pb, n * h, S);
            double L = slv_lev(pb, th + 5, cell);
            double dLdS = slv_dlev_dS(pb, th + 5, cell);
            int nK = pb->n_k_nodes;
            double *Ld = sd;   /* dL/dtheta_j */
            for (int j = 0; j < M; ++j) Ld[j] = dLdS * S * xd[j];
            Ld[5 + cell.a * nK + cell.b] += 1.0 - cell.be;
            Ld[5 + cell.a * nK + cell.b + 1] += cell.be;
            for (int j = 0; j < M; ++j) {
                double vpd = v > 0.0 ? vd[j] : 0.0;
                double sdj = dsdv * vpd;
                double wd = j == 3 ? dw_drho : 0.0;
                double kapd = j == 0 ? 1.0 : 0.0, thbd = j == 1 ? 1.0 : 0.0, xid = j == 2 ? 1.0 : 0.0;
                double xnd = xd[j] - 0.5 * (2.0 * L * Ld[j] * vp + L * L * vpd) * h + (Ld[j] * s + L * sdj) * sq * z1;
                double vnd = vd[j] + kapd * (thb - vp) * h + kap * (thbd - vpd) * h
                           + xid * s * sq * w + xi * sdj * sq * w + xi * s * sq * wd;
                xd[j] = xnd; vd[j] = vnd;
            }
            double xn = x + (r - 0.5 * L * L * vp) * h + L * s * sq * z1;
            double vn = v + kap * (thb - vp) * h + xi * s * sq * w;
            x = xn; v = vn;
        } else if (pb->model == ORC_BSE) {
            double sig = th[0];
            double z = rng_normal(&g, (uint32_t)n);
            double f = 1.0 + r * h + sig * sq * z;
            xd[0] = xd[0] * f + x * sq * z;
            x = x * f;
        } else {
            double z = rng_normal(&g, (uint32_t)n);
            double S = c->s0 * exp(x);
            lv_cell cell = lv_locate(pb, n * h, S);
            double sig = lv_sigma(pb, th, cell);
            double dsdS = lv_dsigma_dS(pb, th, cell);
            int nK = pb->n_k_nodes;
            for (int j = 0; j < M; ++j) sd[j] = dsdS * S * xd[j];
            sd[cell.a * nK + cell.b] += (1.0 - cell.al) * (1.0 - cell.be);
            sd[cell.a * nK + cell.b + 1] += (1.0 - cell.al) * cell.be;
            sd[(cell.a + 1) * nK + cell.b] += cell.al * (1.0 - cell.be);
            sd[(cell.a + 1) * nK + cell.b + 1] += cell.al * cell.be;
            double f = -sig * h + sq * z;
            for (int j = 0; j < M; ++j) xd[j] += f * sd[j];
            x = x + (r - 0.5 * sig * sig) * h + sig * sq * z;
        }
        for (int k = c->date_begin[n + 1]; k < c->date_begin[n + 2]; ++k) {
            int i = c->ids[k];
            double S = spot_of(pb, c, x);
            double dSdx = pb->model == ORC_BSE ? 1.0 : S;
            double pay = S - c->strike[i];
            y[i] = c->disc[i] * (pay > 0.0 ? pay : 0.0);
            for (int j = 0; j < M; ++j)
                dy[(size_t)i * M + j] = pay > 0.0 ? c->disc[i] * dSdx * xd[j] : 0.0;
        }
    }
}

/* ------------------------------------------------------------------ */
/* One path: complex-step forward, theta_j -> theta_j + i*hc.          */
/* Branches (max, indicator, cell choice) are decided on real parts.   */
/* ------------------------------------------------------------------ */
static void path_forward_cstep(const orc_problem *pb, const orc_consts *c, const double *th, int jdir,
                               double hc, uint32_t p, double complex *y, double complex *thc)
{
    const int M = c->M;
    for (int j = 0; j < M; ++j) thc[j] = th[j] + (j == jdir ? hc * I : 0.0);
    orc_rng g; rng_init(&g, pb, p);
    const double h = c->h, sq = c->sq, r = c->r;
    double complex x = state0(pb, c);
    const int hv = pb->model == ORC_HESTON || pb->model == ORC_SLV;
    double complex v = hv ? thc[4] : 0.0;
    double complex rhop = hv ? csqrt(1.0 - thc[3] * thc[3]) : 0.0;
    for (int n = 0; n < c->N; ++n) {
        if (pb->model == ORC_BS) {
            double complex sig = thc[0];
            double z = rng_normal(&g, (uint32_t)n);
            x = x + (r - 0.5 * sig * sig) * h + sig * sq * z;
        } else if (pb->model == ORC_HESTON) {
            double complex kap = thc[0], thb = thc[1], xi = thc[2], rho = thc[3];
            double z1 = rng_normal(&g, (uint32_t)(2 * n));
            double z2 = rng_normal(&g, (uint32_t)(2 * n + 1));
            double complex vp = creal(v) > 0.0 ? v : 0.0;
            double complex s = heston_s_c(vp, pb->sqrt_eps);
            double complex w = rho * z1 + rhop * z2;
            double complex xn = x + (r - 0.5 * vp) * h + s * sq * z1;
            double complex vn = v + kap * (thb - vp) * h + xi * s * sq * w;
            x = xn; v = vn;
        } else if (pb->model == ORC_SLV) {
            double complex kap = thc[0], thb = thc[1], xi = thc[2], rho = thc[3];
            double z1 = rng_normal(&g, (uint32_t)(2 * n));
            double z2 = rng_normal(&g, (uint32_t)(2 * n + 1));
            double complex vp = creal(v) > 0.0 ? v : 0.0;
            double complex s = heston_s_c(vp, pb->sqrt_eps);
            double complex w = rho * z1 + rhop * z2;
            double complex S = c->s0 * cexp(x);
            slv_cell cell = slv_locate(pb, n * h, creal(S));
            double complex be = cell.be;
            if (cell.be > 0.0 && cell.be < 1.0)
                be = (S - pb->k_nodes[cell.b]) / (pb->k_nodes[cell.b + 1] - pb->k_nodes[cell.b]);
            int nK = pb->n_k_nodes;
            double complex L = (1.0 - be) * thc[5 + cell.a * nK + cell.b] + be * thc[5 + cell.a * nK + cell.b + 1];
            double complex xn = x + (r - 0.5 * L * L * vp) * h + L * s * sq * z1;
            double complex vn = v + kap * (thb - vp) * h + xi * s * sq * w;
            x = xn; v = vn;
        } else if (pb->model == ORC_BSE) {
            double complex sig = thc[0];
            double z = rng_normal(&g, (uint32_t)n);
            x = x * (1.0 + r * h + sig * sq * z);
        } else {
            double z = rng_normal(&g, (uint32_t)n);
            double complex S = c->s0 * cexp(x);
            lv_cell cell = lv_locate(pb, n * h, creal(S));
            /* beta carries the imaginary part of S inside the S-range */
            double complex be = cell.be;
            if (cell.be > 0.0 && cell.be < 1.0)
                be = (S - pb->k_nodes[cell.b]) / (pb->k_nodes[cell.b + 1] - pb->k_nodes[cell.b]);
            int nK = pb->n_k_nodes;
            double complex s00 = thc[cell.a * nK + cell.b], s01 = thc[cell.a * nK + cell.b + 1];
            double complex s10 = thc[(cell.a + 1) * nK + cell.b], s11 = thc[(cell.a + 1) * nK + cell.b + 1];
            double complex sig = (1.0 - cell.al) * (1.0 - be) * s00 + (1.0 - cell.al) * be * s01
                               + cell.al * (1.0 - be) * s10 + cell.al * be * s11;
            x = x + (r - 0.5 * sig * sig) * h + sig * sq * z;
        }
        for (int k = c->date_begin[n + 1]; k < c->date_begin[n + 2]; ++k) {
            int i = c->ids[k];
            double complex S = pb->model == ORC_BSE ? x : c->s0 * cexp(x);
            double complex pay = S - c->strike[i];
            y[i] = creal(pay) > 0.0 ? c->disc[i] * pay : 0.0;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Path-ordered compensated sums                                       */
/* ------------------------------------------------------------------ */
typedef struct { double s, c; } nsum;

static void nadd(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

static double nval(const nsum *a) { return a->s + a->c; }

static int64_t chunk_paths(size_t bytes_per_path)
{
    size_t budget = (size_t)64 << 20;
    int64_t n = (int64_t)(budget / (bytes_per_path ? bytes_per_path : 1));
    if (n < 1) n = 1;
    if (n > 65536) n = 65536;
    return n;
}

static int g_threads = 0;

void orc_set_threads(int n) { g_threads = n; }

int orc_get_threads(void)
{
#ifdef _OPENMP
    return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Exported entry points                                               */
/* ------------------------------------------------------------------ */

/* Pass 1 / eq. 1211A: Ey[i] = (1/P) sum_p y_i(p). y_paths (optional) gets
 * the P x m per-path payoffs. */
int orc_forward(const orc_problem *pb, const double *theta, double *Ey, double *y_paths)
{
    orc_consts c;
    int rc = consts_make(pb, &c);
    if (rc) { consts_free(&c); return rc; }
    const int m = c.m;
    const int64_t P = pb->n_paths;
    int64_t CH = chunk_paths(sizeof(double) * (size_t)m);
    double *buf = (double *)malloc(sizeof(double) * (size_t)m * (size_t)CH);
    nsum *acc = (nsum *)calloc((size_t)m, sizeof(nsum));
    if (!buf || !acc) { free(buf); free(acc); consts_free(&c); return ORC_ENOMEM; }
    for (int64_t p0 = 0; p0 < P; p0 += CH) {
        int64_t np = P - p0 < CH ? P - p0 : CH;
#pragma omp parallel for schedule(static) num_threads(orc_get_threads())
        for (int64_t k = 0; k < np; ++k) {
            double *y = buf + (size_t)k * m;
            for (int i = 0; i < m; ++i) y[i] = 0.0;
            path_forward(pb, &c, theta, (uint32_t)(p0 + k), y);
        }
        for (int64_t k = 0; k < np; ++k)
            for (int i = 0; i < m; ++i) nadd(&acc[i], buf[(size_t)k * m + i]);
        if (y_paths) memcpy(y_paths + (size_t)p0 * m, buf, sizeof(double) * (size_t)m * (size_t)np);
    }
    for (int i = 0; i < m; ++i) Ey[i] = nval(&acc[i]) / (double)P;
    free(buf); free(acc); consts_free(&c);
    return ORC_OK;
}

/* Pass 2 / eq. 0711A summed over paths: grad[j] = sum_p sum_i (lambda_i/P) dy_i(p)/dtheta_j.
 * lambda is the adjoint of Ey.  g_paths (optional) gets the P x M per-path terms. */
int orc_vjp(const orc_problem *pb, const double *theta, const double *lambda, double *grad, double *g_paths)
{
    orc_consts c;
    int rc = consts_make(pb, &c);
    if (rc) { consts_free(&c); return rc; }
    const int M = c.M, m = c.m, N = c.N;
    const int64_t P = pb->n_paths;
    double *lam = (double *)malloc(sizeof(double) * (size_t)m);
    int64_t CH = chunk_paths(sizeof(double) * (size_t)M);
    double *buf = (double *)malloc(sizeof(double) * (size_t)M * (size_t)CH);
    nsum *acc = (nsum *)calloc((size_t)M, sizeof(nsum));
    if (!lam || !buf || !acc) { free(lam); free(buf); free(acc); consts_free(&c); return ORC_ENOMEM; }
    for (int i = 0; i < m; ++i) lam[i] = lambda[i] / (double)P;
    int nerr = 0;
    for (int64_t p0 = 0; p0 < P; p0 += CH) {
        int64_t np = P - p0 < CH ? P - p0 : CH;
#pragma omp parallel num_threads(orc_get_threads()) reduction(+ : nerr)
        {
            double *work = (double *)malloc(sizeof(double) * (size_t)(4 * N + 2));
            if (!work) nerr++;
#pragma omp for schedule(static)
            for (int64_t k = 0; k < np; ++k)
                if (work) path_reverse(pb, &c, theta, (uint32_t)(p0 + k), lam, buf + (size_t)k * M, work);
            free(work);
        }
        if (nerr) break;
        for (int64_t k = 0; k < np; ++k)
            for (int j = 0; j < M; ++j) nadd(&acc[j], buf[(size_t)k * M + j]);
        if (g_paths) memcpy(g_paths + (size_t)p0 * M, buf, sizeof(double) * (size_t)M * (size_t)np);
    }
    for (int j = 0; j < M; ++j) grad[j] = nval(&acc[j]);
    free(lam); free(buf); free(acc); consts_free(&c);
    return nerr ? ORC_ENOMEM : ORC_OK;
}

/* The paper's algorithm: step 1 (Ey), residual r = Ey - C and G = 1/2 sum r^2,
 * step 2 (reverse sweep per path seeded with lambda = r), step 3 (sum). */
int orc_gradient(const orc_problem *pb, const double *theta, const double *C,
                 double *Ey, double *G, double *grad)
{
    int rc = orc_forward(pb, theta, Ey, NULL);
    if (rc) return rc;
    const int m = pb->n_instr;
    double *r = (double *)malloc(sizeof(double) * (size_t)m);
    if (!r) return ORC_ENOMEM;
    nsum g = {0.0, 0.0};
    for (int i = 0; i < m; ++i) { r[i] = Ey[i] - C[i]; nadd(&g, 0.5 * r[i] * r[i]); }
    *G = nval(&g);
    rc = orc_vjp(pb, theta, r, grad, NULL);
    free(r);
    return rc;
}

/* Forward tangent mode: J[i*M + j] = dEy_i/dtheta_j (and Ey).  The optional
 * per-path outputs are P x m (y) and P x m x M (dy). */
int orc_jacobian(const orc_problem *pb, const double *theta, double *Ey, double *J,
                 double *y_paths, double *dy_paths)
{
    orc_consts c;
    int rc = consts_make(pb, &c);
    if (rc) { consts_free(&c); return rc; }
    const int M = c.M, m = c.m;
    const int64_t P = pb->n_paths;
    const size_t per = (size_t)m * (size_t)(M + 1);
    int64_t CH = chunk_paths(sizeof(double) * per);
    double *buf = (double *)malloc(sizeof(double) * per * (size_t)CH);
    nsum *acc = (nsum *)calloc(per, sizeof(nsum));
    if (!buf || !acc) { free(buf); free(acc); consts_free(&c); return ORC_ENOMEM; }
    int nerr = 0;
    for (int64_t p0 = 0; p0 < P; p0 += CH) {
        int64_t np = P - p0 < CH ? P - p0 : CH;
#pragma omp parallel num_threads(orc_get_threads()) reduction(+ : nerr)
        {
            double *work = (double *)malloc(sizeof(double) * (size_t)(3 * M + 1));
            if (!work) nerr++;
#pragma omp for schedule(static)
            for (int64_t k = 0; k < np; ++k) {
                double *y = buf + (size_t)k * per;
                double *dy = y + m;
                for (size_t t = 0; t < per; ++t) y[t] = 0.0;
                if (work) path_tangent(pb, &c, theta, (uint32_t)(p0 + k), y, dy, work);
            }
            free(work);
        }
        if (nerr) break;
        for (int64_t k = 0; k < np; ++k)
            for (size_t t = 0; t < per; ++t) nadd(&acc[t], buf[(size_t)k * per + t]);
        for (int64_t k = 0; k < np; ++k) {
            if (y_paths) memcpy(y_paths + (size_t)(p0 + k) * m, buf + (size_t)k * per, sizeof(double) * (size_t)m);
            if (dy_paths) memcpy(dy_paths + (size_t)(p0 + k) * m * M, buf + (size_t)k * per + m,
                                 sizeof(double) * (size_t)m * (size_t)M);
        }
    }
    for (int i = 0; i < m; ++i) Ey[i] = nval(&acc[i]) / (double)P;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < M; ++j) J[(size_t)i * M + j] = nval(&acc[m + (size_t)i * M + j]) / (double)P;
    free(buf); free(acc); consts_free(&c);
    return nerr ? ORC_ENOMEM : ORC_OK;
}

/* Complex-step forward: Ey evaluated at theta + i*hc*e_j; returns real and
 * imaginary parts.  d Ey_i/d theta_j = Ey_im[i] / hc. */
int orc_forward_cstep(const orc_problem *pb, const double *theta, int j, double hc,
                      double *Ey_re, double *Ey_im)
{
    orc_consts c;
    int rc = consts_make(pb, &c);
    if (rc) { consts_free(&c); return rc; }
    if (j < 0 || j >= c.M) { consts_free(&c); return ORC_EINVAL; }
    const int m = c.m, M = c.M;
    const int64_t P = pb->n_paths;
    int64_t CH = chunk_paths(sizeof(double complex) * (size_t)m);
    double complex *buf = (double complex *)malloc(sizeof(double complex) * (size_t)m * (size_t)CH);
    nsum *acc = (nsum *)calloc((size_t)(2 * m), sizeof(nsum));
    if (!buf || !acc) { free(buf); free(acc); consts_free(&c); return ORC_ENOMEM; }
    int nerr = 0;
    for (int64_t p0 = 0; p0 < P; p0 += CH) {
        int64_t np = P - p0 < CH ? P - p0 : CH;
#pragma omp parallel num_threads(orc_get_threads()) reduction(+ : nerr)
        {
            double complex *thc = (double complex *)malloc(sizeof(double complex) * (size_t)M);
            if (!thc) nerr++;
#pragma omp for schedule(static)
            for (int64_t k = 0; k < np; ++k) {
                double complex *y = buf + (size_t)k * m;
                for (int i = 0; i < m; ++i) y[i] = 0.0;
                if (thc) path_forward_cstep(pb, &c, theta, j, hc, (uint32_t)(p0 + k), y, thc);
            }
            free(thc);
        }
        if (nerr) break;
        for (int64_t k = 0; k < np; ++k)
            for (int i = 0; i < m; ++i) {
                nadd(&acc[i], creal(buf[(size_t)k * m + i]));
                nadd(&acc[m + i], cimag(buf[(size_t)k * m + i]));
            }
    }
    for (int i = 0; i < m; ++i) {
        Ey_re[i] = nval(&acc[i]) / (double)P;
        Ey_im[i] = nval(&acc[m + i]) / (double)P;
    }
    free(buf); free(acc); consts_free(&c);
    return nerr ? ORC_ENOMEM : ORC_OK;
}
