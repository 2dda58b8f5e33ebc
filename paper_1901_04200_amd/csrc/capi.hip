// C ABI of the library (declared in include/mcaad.h): problem validation,
// context and workspace ownership, and the sequence of kernel launches for
// each entry point.  Nothing here computes on the host beyond constants and
// table layout; every step of the path runs in the kernels of mc_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/mcaad.h"
#include "bse_kernels.hpp"
#include "mc_device.hpp"
#include "mc_kernels.hpp"

using namespace mcaad;

namespace {

constexpr int kMaxInstr = 2048;
constexpr int kMaxSteps = 65536;
constexpr int kMaxTimed = 256;

thread_local std::string g_err;

struct TimedPair {
    hipEvent_t a, b;
    int which;
};

}  // namespace

struct cal_ctx {
    int device = 0;
    int model = 0;
    bool fp64 = false;
    int M = 0, m = 0, N = 0;
    int64_t P = 0;
    int64_t nblocks = 0;
    int max_batch = 1;
    int K = 16;
    int ppl = 1;                 // paths per lane
    int64_t nblocks_tan = 0;     // tangent mode runs one path per lane
    int mode = CAL_CKPT_STORE;
    size_t real = 4;
    DevProblem dp{};
    // device workspace
    int32_t *d_date_step = nullptr;
    int32_t *d_date_begin = nullptr;
    double *d_strike = nullptr;
    float *d_strike_f = nullptr;
    double *d_disc = nullptr;
    int32_t *d_id = nullptr;
    int32_t *d_status = nullptr;
    double *d_part_y = nullptr;
    double *d_part_g = nullptr;
    void *d_lv_rows = nullptr;     // local volatility: [N][nK] grid rows of pass 2 (path precision)
    double *d_part_j = nullptr;
    void *d_lamD = nullptr;
    void *d_ckpt = nullptr;
    double *d_theta_ckpt = nullptr;   // the parameters d_ckpt was last written with
    bool ckpt_valid = false;          // d_ckpt holds every segment of a completed sweep
    double *d_t_nodes = nullptr;
    int32_t *d_step_row = nullptr;
    double *d_step_al = nullptr;      // local volatility: time weight of every step
    float *d_step_al_f = nullptr;
    // timing
    bool timing = false;
    std::vector<TimedPair> timed;
    std::vector<hipEvent_t> pool;
    std::string err;
};

static int fail(cal_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    g_err = msg;
    return code;
}

static int hip_fail(cal_ctx *ctx, hipError_t e, const char *where)
{
    return fail(ctx, CAL_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

static std::string validate(const cal_problem *pb, int *code)
{
    *code = CAL_EINVAL;
    if (!pb) return "null problem";
    if (pb->model != CAL_BS && pb->model != CAL_HESTON && pb->model != CAL_LV && pb->model != CAL_SLV &&
        pb->model != CAL_BS_EULER_S)
        return "unknown model";
    if (pb->precision != CAL_FP32 && pb->precision != CAL_FP64) return "unknown precision";
    if (pb->n_instr < 1 || pb->n_instr > kMaxInstr) return "n_instr must be in 1..2048";
    if (pb->n_steps < 1 || pb->n_steps > kMaxSteps) return "n_steps must be in 1..65536";
    if (pb->n_paths < 1 || pb->n_paths > ((int64_t)1 << 32)) return "n_paths must be in 1..2^32";
    if (!pb->instr_step || !pb->instr_strike) return "null instrument table";
    for (int i = 0; i < pb->n_instr; ++i) {
        if (pb->instr_step[i] < 1 || pb->instr_step[i] > pb->n_steps) return "instr_step outside 1..n_steps";
        if (!std::isfinite(pb->instr_strike[i]) || pb->instr_strike[i] < 0.0) return "strike must be finite and >= 0";
    }
    if (!(pb->s0 > 0.0) || !std::isfinite(pb->s0)) return "s0 must be positive";
    if (!(pb->t_max > 0.0) || !std::isfinite(pb->t_max)) return "t_max must be positive";
    if (!std::isfinite(pb->rate)) return "rate must be finite";
    if (!(pb->sqrt_eps >= 0.0) || !std::isfinite(pb->sqrt_eps)) return "sqrt_eps must be finite and >= 0";
    if (pb->sqrt_eps != 0.0) {
        *code = CAL_EUNSUPPORTED;
        return "sqrt_eps must be 0: the device path runs plain full truncation";
    }
    if (pb->ckpt_every != 0 && pb->ckpt_every != 8 && pb->ckpt_every != 16 && pb->ckpt_every != 32)
        return "ckpt_every must be 0, 8, 16 or 32";
    if (pb->ckpt_mode < CAL_CKPT_AUTO || pb->ckpt_mode > CAL_CKPT_STORE) return "unknown ckpt_mode";
    if (pb->paths_per_lane != 0 && pb->paths_per_lane != 1 && pb->paths_per_lane != 2 && pb->paths_per_lane != 4)
        return "paths_per_lane must be 0, 1, 2 or 4";
    if (pb->model == CAL_LV && pb->paths_per_lane > 2) {
        *code = CAL_EUNSUPPORTED;
        return "local volatility runs one or two paths per lane";
    }
    if (pb->max_batch < 0 || pb->max_batch > 65535) return "max_batch must be in 0..65535";
    if ((pb->model == CAL_BS || pb->model == CAL_BS_EULER_S) && pb->n_params != 1)
        return "Black-Scholes takes n_params = 1";
    if (pb->model == CAL_HESTON && pb->n_params != 5) return "Heston takes n_params = 5";
    if (pb->model == CAL_LV || pb->model == CAL_SLV) {
        const bool lv = pb->model == CAL_LV;
        const int nT = pb->n_t_nodes, nK = pb->n_k_nodes;
        if (lv && (nT < 2 || nK < 2 || nT > 64 || nK > 64)) return "local vol needs 2..64 time and spot nodes";
        if (!lv && (nT < 1 || nK < 2 || nT > 64 || nK > 64))
            return "stochastic local vol needs 1..64 time and 2..64 spot nodes";
        if (!pb->t_nodes || !pb->k_nodes) return "null node arrays";
        if (lv && pb->n_params != nT * nK) return "local vol takes n_params = n_t_nodes * n_k_nodes";
        if (!lv && pb->n_params != 5 + nT * nK)
            return "stochastic local vol takes n_params = 5 + n_t_nodes * n_k_nodes";
        for (int a = 0; a < nT; ++a)
            if (!std::isfinite(pb->t_nodes[a]) || (a > 0 && !(pb->t_nodes[a] > pb->t_nodes[a - 1])))
                return "t_nodes must be finite and increasing";
        const double K0 = pb->k_nodes[0], dK = (pb->k_nodes[nK - 1] - K0) / (nK - 1);
        if (!std::isfinite(K0) || !(dK > 0.0) || !std::isfinite(dK)) return "k_nodes must be finite and increasing";
        for (int k = 0; k < nK; ++k)
            if (std::fabs(pb->k_nodes[k] - (K0 + k * dK)) > 1e-9 * (std::fabs(K0) + nK * dK))
                return "k_nodes must be uniformly spaced";
    }
    *code = CAL_OK;
    return "";
}

static hipError_t alloc(void **p, size_t bytes)
{
    return hipMalloc(p, bytes ? bytes : 8);
}

// Host copies of the instrument tables the kernels read: instruments grouped
// by maturity step (ascending; original order within a step), their strikes
// (FP64 and FP32) and discount factors exp(-r n_i h), the original index of
// each, and the distinct maturity steps with the ranges they begin.
struct Tables {
    std::vector<int32_t> order, date_step, date_begin;
    std::vector<double> strike, disc;
    std::vector<float> strike_f;
};

static void build_tables(const cal_problem *pb, Tables &t)
{
    const int m = pb->n_instr;
    const double h = pb->t_max / pb->n_steps;
    t.order.resize(m);
    std::iota(t.order.begin(), t.order.end(), 0);
    std::stable_sort(t.order.begin(), t.order.end(),
                     [&](int a, int b) { return pb->instr_step[a] < pb->instr_step[b]; });
    t.date_step.clear();
    t.date_begin.clear();
    t.strike.resize(m);
    t.disc.resize(m);
    t.strike_f.resize(m);
    for (int k = 0; k < m; ++k) {
        const int i = t.order[k];
        const int s = pb->instr_step[i];
        if (t.date_step.empty() || t.date_step.back() != s) {
            t.date_step.push_back(s);
            t.date_begin.push_back(k);
        }
        t.strike[k] = pb->instr_strike[i];
        t.strike_f[k] = (float)pb->instr_strike[i];
        t.disc[k] = std::exp(-pb->rate * s * h);
    }
    t.date_begin.push_back(m);
}

// The scalar part of the kernels' problem description (table pointers are
// set by the caller).
static void set_scalars(DevProblem &d, const cal_problem *pb, int nd, int nseg, int K, int ppl)
{
    const double h = pb->t_max / pb->n_steps;
    d.N = pb->n_steps;
    d.m = pb->n_instr;
    d.M = pb->n_params;
    d.ndates = nd;
    d.nseg = nseg;
    d.K = K;
    d.ppl = ppl;
    d.P = pb->n_paths;
    d.k0 = (uint32_t)pb->seed;
    d.k1 = (uint32_t)(pb->seed >> 32);
    d.inst = pb->inst;
    d.s0 = pb->s0;
    d.rate = pb->rate;
    d.h = h;
    d.sq = std::sqrt(h);
}

extern "C" int cal_validate(const cal_problem *pb, char *msg, int32_t msg_len)
{
    int code;
    std::string s = validate(pb, &code);
    if (msg && msg_len > 0) {
        std::snprintf(msg, (size_t)msg_len, "%s", s.c_str());
    }
    if (code != CAL_OK) g_err = s;
    return code;
}

extern "C" int cal_destroy(cal_ctx *ctx)
{
    if (!ctx) return CAL_OK;
    (void)hipDeviceSynchronize();
    void *bufs[] = {ctx->d_date_step, ctx->d_date_begin, ctx->d_strike, ctx->d_strike_f, ctx->d_disc, ctx->d_id,
                    ctx->d_status, ctx->d_part_y, ctx->d_part_g, ctx->d_part_j, ctx->d_lamD, ctx->d_ckpt,
                    ctx->d_theta_ckpt, ctx->d_t_nodes, ctx->d_step_row, ctx->d_step_al, ctx->d_step_al_f,
                    ctx->d_lv_rows};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    for (auto &t : ctx->timed) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : ctx->pool) (void)hipEventDestroy(e);
    delete ctx;
    return CAL_OK;
}

extern "C" int cal_create(const cal_problem *pb, cal_ctx **out)
{
    if (!out) return fail(nullptr, CAL_EINVAL, "null output pointer");
    *out = nullptr;
    int code;
    std::string msg = validate(pb, &code);
    if (code != CAL_OK) return fail(nullptr, code, msg);

    cal_ctx *c = new cal_ctx();
    (void)hipGetDevice(&c->device);
    c->model = pb->model;
    c->fp64 = pb->precision == CAL_FP64;
    c->real = c->fp64 ? 8 : 4;
    c->M = pb->n_params;
    c->m = pb->n_instr;
    c->N = pb->n_steps;
    c->P = pb->n_paths;
    c->ppl = pb->paths_per_lane > 0 ? pb->paths_per_lane : 1;
    c->nblocks = (c->P + (int64_t)kBlock * c->ppl - 1) / ((int64_t)kBlock * c->ppl);
    c->nblocks_tan = (c->P + kBlock - 1) / kBlock;
    c->max_batch = pb->max_batch > 0 ? pb->max_batch : 1;
    c->K = pb->ckpt_every ? pb->ckpt_every : (c->fp64 || c->model == CAL_SLV ? 8 : 16);
    const int nv = c->model == CAL_HESTON || c->model == CAL_SLV ? 2 : 1;
    const int nseg = (c->N + c->K - 1) / c->K;
    const size_t ckpt_bytes = (size_t)nseg * nv * (size_t)c->P * c->real;
    c->mode = pb->ckpt_mode == CAL_CKPT_AUTO ? CAL_CKPT_STORE : pb->ckpt_mode;

    // instruments grouped by maturity date (ascending), original order within a date
    const int m = c->m;
    const double h = pb->t_max / c->N;
    Tables tb;
    build_tables(pb, tb);
    const std::vector<int32_t> &order = tb.order, &date_step = tb.date_step, &date_begin = tb.date_begin;
    const std::vector<double> &strike = tb.strike, &disc = tb.disc;
    const std::vector<float> &strike_f = tb.strike_f;
    const int nd = (int)date_step.size();

    // tangent mode serves Black-Scholes and Heston (labels); not the grid models
    const bool grid = c->model == CAL_LV || c->model == CAL_SLV;
    const size_t tan_w = grid ? 0 : (size_t)m * (c->M + 1);
    if (grid) {
        DevProblem probe{};
        probe.N = c->N;
        probe.m = m;
        probe.K = c->K;
        probe.nT = pb->n_t_nodes;
        probe.nK = pb->n_k_nodes;
        int max_lds = 0;
        if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess ||
            max_lds <= 0) {
            delete c;
            return fail(nullptr, CAL_EHIP, "device query failed (LDS bytes per workgroup)");
        }
        const size_t need = c->model == CAL_LV
                                ? std::max(lv_lds_bytes(probe, c->fp64, 1), lv_lds_bytes(probe, c->fp64, 2))
                                : std::max(slv_lds_bytes(probe, c->fp64, 1), slv_lds_bytes(probe, c->fp64, 2));
        if (need > (size_t)max_lds) {
            delete c;
            return fail(nullptr, CAL_EUNSUPPORTED,
                        "grid, steps and spacing too large for one workgroup's LDS (" + std::to_string(need) + " > " +
                            std::to_string(max_lds) + " bytes)");
        }
    }
    hipError_t e = hipSuccess;
    auto A = [&](void **p, size_t bytes) {
        if (e == hipSuccess) e = alloc(p, bytes);
    };
    A((void **)&c->d_date_step, sizeof(int32_t) * nd);
    A((void **)&c->d_date_begin, sizeof(int32_t) * (nd + 1));
    A((void **)&c->d_strike, sizeof(double) * m);
    A((void **)&c->d_strike_f, sizeof(float) * m);
    A((void **)&c->d_disc, sizeof(double) * m);
    A((void **)&c->d_id, sizeof(int32_t) * m);
    A((void **)&c->d_status, sizeof(int32_t));
    A((void **)&c->d_part_y, sizeof(double) * (size_t)c->nblocks * m);
    // local volatility: two partial columns per node (see launch_lv_reduce)
    A((void **)&c->d_part_g, sizeof(double) * (size_t)c->nblocks * c->M * (c->model == CAL_LV ? 2 : 1));
    if (c->model == CAL_LV) A(&c->d_lv_rows, c->real * (size_t)c->N * pb->n_k_nodes);
    A((void **)&c->d_part_j, sizeof(double) * (size_t)c->nblocks_tan * tan_w * c->max_batch);
    A(&c->d_lamD, c->real * m);
    A((void **)&c->d_theta_ckpt, sizeof(double) * c->M);
    if (c->model == CAL_LV) {
        A((void **)&c->d_t_nodes, sizeof(double) * pb->n_t_nodes);
        A((void **)&c->d_step_al, sizeof(double) * c->N);
        A((void **)&c->d_step_al_f, sizeof(float) * c->N);
    }
    if (c->model == CAL_LV || c->model == CAL_SLV) A((void **)&c->d_step_row, sizeof(int32_t) * c->N);
    if (e != hipSuccess) {
        cal_destroy(c);
        return fail(nullptr, CAL_ENOMEM, std::string("workspace allocation failed: ") + hipGetErrorString(e));
    }
    e = alloc(&c->d_ckpt, ckpt_bytes);
    if (e != hipSuccess) {
        cal_destroy(c);
        return fail(nullptr, CAL_ENOMEM, "checkpoint buffer allocation failed");
    }
    auto H2D = [&](void *dst, const void *src, size_t bytes) {
        if (e == hipSuccess) e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    };
    H2D(c->d_date_step, date_step.data(), sizeof(int32_t) * nd);
    H2D(c->d_date_begin, date_begin.data(), sizeof(int32_t) * (nd + 1));
    H2D(c->d_strike, strike.data(), sizeof(double) * m);
    H2D(c->d_strike_f, strike_f.data(), sizeof(float) * m);
    H2D(c->d_disc, disc.data(), sizeof(double) * m);
    H2D(c->d_id, order.data(), sizeof(int32_t) * m);
    if (c->model == CAL_LV) {
        H2D(c->d_t_nodes, pb->t_nodes, sizeof(double) * pb->n_t_nodes);
        // time cell a of step n (the last node row a + 1 <= nT - 1 with
        // t_nodes[a] <= n h, or 0) and its weight on row a + 1, clamped to [0, 1]
        std::vector<int32_t> cell(c->N);
        std::vector<double> al(c->N);
        std::vector<float> al_f(c->N);
        const int nT = pb->n_t_nodes;
        for (int n = 0; n < c->N; ++n) {
            const double t = n * h;
            int a = 0;
            while (a + 1 < nT - 1 && pb->t_nodes[a + 1] <= t) ++a;
            double w = (t - pb->t_nodes[a]) / (pb->t_nodes[a + 1] - pb->t_nodes[a]);
            w = w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
            cell[n] = a;
            al[n] = w;
            al_f[n] = (float)w;
        }
        H2D(c->d_step_row, cell.data(), sizeof(int32_t) * c->N);
        H2D(c->d_step_al, al.data(), sizeof(double) * c->N);
        H2D(c->d_step_al_f, al_f.data(), sizeof(float) * c->N);
    }
    if (c->model == CAL_SLV) {
        // leverage row of step n: the number of time nodes <= n h, capped at the last row
        std::vector<int32_t> row(c->N);
        for (int n = 0; n < c->N; ++n) {
            int a = 0;
            while (a < pb->n_t_nodes && pb->t_nodes[a] <= n * h) ++a;
            row[n] = a < pb->n_t_nodes - 1 ? a : pb->n_t_nodes - 1;
        }
        H2D(c->d_step_row, row.data(), sizeof(int32_t) * c->N);
    }
    if (e == hipSuccess) e = hipMemset(c->d_status, 0, sizeof(int32_t));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        cal_destroy(c);
        return fail(nullptr, CAL_EHIP, std::string("table upload failed: ") + hipGetErrorString(e));
    }

    DevProblem &d = c->dp;
    set_scalars(d, pb, nd, nseg, c->K, c->ppl);
    d.theta_save = c->d_theta_ckpt;
    d.date_step = c->d_date_step;
    d.date_begin = c->d_date_begin;
    d.strike = c->d_strike;
    d.strike_f = c->d_strike_f;
    d.disc = c->d_disc;
    d.id = c->d_id;
    d.status = c->d_status;
    if (grid) {
        d.nT = pb->n_t_nodes;
        d.nK = pb->n_k_nodes;
        d.K0 = pb->k_nodes[0];
        d.dK = (pb->k_nodes[d.nK - 1] - pb->k_nodes[0]) / (d.nK - 1);
        d.t_nodes = c->d_t_nodes;
        d.step_row = c->d_step_row;
        d.step_al = c->d_step_al;
        d.step_al_f = c->d_step_al_f;
    }
    *out = c;
    return CAL_OK;
}

// --- timing -----------------------------------------------------------------
static hipEvent_t get_event(cal_ctx *c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct Timed {
    cal_ctx *c;
    hipStream_t st;
    int which;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(cal_ctx *c_, hipStream_t s, int w) : c(c_), st(s), which(w)
    {
        if (c->timing && (int)c->timed.size() < kMaxTimed) {
            a = get_event(c);
            b = get_event(c);
            if (a && b && hipEventRecord(a, st) != hipSuccess) a = nullptr;
        }
    }
    void done()
    {
        if (a && b && hipEventRecord(b, st) == hipSuccess) c->timed.push_back({a, b, which});
    }
};

extern "C" int cal_timing_enable(cal_ctx *ctx, int32_t on)
{
    if (!ctx) return fail(nullptr, CAL_EINVAL, "null context");
    (void)hipDeviceSynchronize();
    for (auto &t : ctx->timed) {
        ctx->pool.push_back(t.a);
        ctx->pool.push_back(t.b);
    }
    ctx->timed.clear();
    ctx->timing = on != 0;
    return CAL_OK;
}

extern "C" int cal_timing_read(cal_ctx *ctx, int32_t which, double *ms_total, int64_t *launches)
{
    if (!ctx || !ms_total || !launches) return fail(ctx, CAL_EINVAL, "null argument");
    double tot = 0.0;
    int64_t n = 0;
    for (auto &t : ctx->timed) {
        if (t.which != which) continue;
        hipError_t e = hipEventSynchronize(t.b);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventSynchronize");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, t.a, t.b);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventElapsedTime");
        tot += ms;
        ++n;
    }
    *ms_total = tot;
    *launches = n;
    return CAL_OK;
}

extern "C" int cal_geometry(const cal_ctx *ctx, int32_t *threads, int64_t *blocks, int32_t *ckpt_every,
                            int32_t *ckpt_mode)
{
    if (!ctx) return CAL_EINVAL;
    if (threads) *threads = kBlock;
    if (blocks) *blocks = ctx->nblocks;
    if (ckpt_every) *ckpt_every = ctx->K;
    if (ckpt_mode) *ckpt_mode = ctx->mode;
    return CAL_OK;
}

// --- entry points -------------------------------------------------------------
static int check_ctx(cal_ctx *ctx)
{
    if (!ctx) return fail(nullptr, CAL_EINVAL, "null context");
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != ctx->device) return fail(ctx, CAL_EINVAL, "context belongs to another device");
    ctx->err.clear();
    return CAL_OK;
}

static int run_pass1(cal_ctx *c, const double *theta, bool store, hipStream_t st)
{
    if (c->model == CAL_LV || c->model == CAL_SLV) {
        hipError_t ec = launch_check_theta(c->dp, theta, c->model, st);
        if (ec != hipSuccess) return hip_fail(c, ec, "theta check launch");
    }
    Timed t(c, st, 0);
    hipError_t e;
    if (c->model == CAL_LV) {
        e = launch_lv_rows(c->dp, c->fp64, theta, c->d_lv_rows, st);
        if (e == hipSuccess)
            e = launch_lv_pass1(c->dp, c->fp64, store, theta, c->d_lv_rows, c->d_part_y, c->d_ckpt, c->nblocks, st);
    } else if (c->model == CAL_SLV) {
        e = launch_slv_pass1(c->dp, c->fp64, store, theta, c->d_part_y, c->d_ckpt, c->nblocks, st);
    } else if (c->model == CAL_BS_EULER_S) {
        e = launch_bse_pass1(c->dp, c->fp64, store, theta, c->d_part_y, c->d_ckpt, c->nblocks, st);
    } else {
        e = launch_pass1(c->dp, c->model, c->fp64, store, theta, c->d_part_y, c->d_ckpt, c->nblocks, st);
    }
    t.done();
    if (e != hipSuccess) return hip_fail(c, e, "pass-1 launch");
    return CAL_OK;
}

// dG/dtheta from pass 2's partial columns
static hipError_t reduce_grad(cal_ctx *c, double *d_grad, hipStream_t st)
{
    if (c->model == CAL_LV) return launch_lv_reduce(c->d_part_g, c->nblocks, c->M, d_grad, c->d_status, st);
    return launch_reduce_sorted(c->d_part_g, c->nblocks, c->M, nullptr, 1.0, d_grad, c->d_status, st);
}

static int run_pass2(cal_ctx *c, const double *theta, bool from_ckpt, hipStream_t st)
{
    Timed t(c, st, 1);
    hipError_t e;
    if (c->model == CAL_LV) {
        e = launch_lv_rows(c->dp, c->fp64, theta, c->d_lv_rows, st);
        if (e == hipSuccess)
            e = launch_lv_pass2(c->dp, c->fp64, from_ckpt, theta, c->d_lv_rows, c->d_lamD, c->d_part_g, c->d_ckpt,
                                c->nblocks, st);
    } else if (c->model == CAL_SLV) {
        e = launch_slv_pass2(c->dp, c->fp64, from_ckpt, theta, c->d_lamD, c->d_part_g, c->d_ckpt, c->nblocks, st);
    } else if (c->model == CAL_BS_EULER_S) {
        e = launch_bse_pass2(c->dp, c->fp64, from_ckpt, theta, c->d_lamD, c->d_part_g, c->d_ckpt, c->nblocks, st);
    } else {
        e = launch_pass2(c->dp, c->model, c->fp64, from_ckpt, theta, c->d_lamD, c->d_part_g, c->d_ckpt, c->nblocks,
                         st);
    }
    t.done();
    if (e != hipSuccess) return hip_fail(c, e, "pass-2 launch");
    return CAL_OK;
}

extern "C" int calibrate_forward(cal_ctx *ctx, const double *d_theta, double *d_Ey, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!d_theta || !d_Ey) return fail(ctx, CAL_EINVAL, "null device pointer");
    hipStream_t st = (hipStream_t)stream;
    rc = run_pass1(ctx, d_theta, false, st);
    if (rc) return rc;
    hipError_t e = launch_reduce_sorted(ctx->d_part_y, ctx->nblocks, ctx->m, ctx->d_id, 1.0 / (double)ctx->P,
                                        d_Ey, ctx->d_status, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "reduce launch");
    return CAL_OK;
}

extern "C" int calibrate_forward_store(cal_ctx *ctx, const double *d_theta, double *d_Ey, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!d_theta || !d_Ey) return fail(ctx, CAL_EINVAL, "null device pointer");
    hipStream_t st = (hipStream_t)stream;
    ctx->ckpt_valid = false;
    rc = run_pass1(ctx, d_theta, true, st);
    if (rc) return rc;
    // a sweep writing every checkpoint segment is enqueued; its workgroup 0
    // copies theta beside the buffer (DevProblem::theta_save)
    ctx->ckpt_valid = true;
    hipError_t e = launch_reduce_sorted(ctx->d_part_y, ctx->nblocks, ctx->m, ctx->d_id, 1.0 / (double)ctx->P,
                                        d_Ey, ctx->d_status, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "reduce launch");
    return CAL_OK;
}

// Pass 2 with a caller-given output adjoint; from_ckpt: from the buffer's
// checkpoints (which must be there), else re-running the forward sweep.
static int vjp(cal_ctx *ctx, const double *d_theta, const double *d_lambda, double *d_grad, bool from_ckpt,
               hipStream_t st)
{
    if (!d_theta || !d_lambda || !d_grad) return fail(ctx, CAL_EINVAL, "null device pointer");
    if (from_ckpt && !ctx->ckpt_valid)
        return fail(ctx, CAL_EINVAL, "no stored checkpoints on this context (no completed storing sweep yet)");
    // sigma's domain is the same under both Black-Scholes schemes
    hipError_t e = launch_check_theta(ctx->dp, d_theta, ctx->model == CAL_BS_EULER_S ? CAL_BS : ctx->model, st);
    if (e == hipSuccess)
        e = launch_lambda(ctx->dp, ctx->fp64, d_lambda, ctx->d_lamD, from_ckpt ? ctx->d_theta_ckpt : nullptr, d_theta,
                          st);
    if (e != hipSuccess) return hip_fail(ctx, e, "lambda launch");
    if (!from_ckpt) ctx->ckpt_valid = false;
    int rc = run_pass2(ctx, d_theta, from_ckpt, st);
    if (rc) return rc;
    if (!from_ckpt) ctx->ckpt_valid = true;   // the re-run wrote every segment
    e = reduce_grad(ctx, d_grad, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "reduce launch");
    return CAL_OK;
}

extern "C" int calibrate_vjp(cal_ctx *ctx, const double *d_theta, const double *d_lambda, double *d_grad,
                             void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    return vjp(ctx, d_theta, d_lambda, d_grad, false, (hipStream_t)stream);
}

extern "C" int calibrate_vjp_stored(cal_ctx *ctx, const double *d_theta, const double *d_lambda, double *d_grad,
                                    void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    return vjp(ctx, d_theta, d_lambda, d_grad, true, (hipStream_t)stream);
}

extern "C" int calibrate_gradient(cal_ctx *ctx, const double *d_theta, const double *d_C, double *d_Ey,
                                  double *d_G, double *d_grad, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!d_theta || !d_C || !d_Ey || !d_G || !d_grad) return fail(ctx, CAL_EINVAL, "null device pointer");
    hipStream_t st = (hipStream_t)stream;
    const bool store = ctx->mode == CAL_CKPT_STORE;
    ctx->ckpt_valid = false;
    rc = run_pass1(ctx, d_theta, store, st);
    if (rc) return rc;
    hipError_t e = launch_reduce_sorted(ctx->d_part_y, ctx->nblocks, ctx->m, ctx->d_id, 1.0 / (double)ctx->P,
                                        d_Ey, ctx->d_status, st);
    if (e == hipSuccess) e = launch_residual(ctx->dp, ctx->fp64, d_Ey, d_C, d_G, ctx->d_lamD, d_theta, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "residual launch");
    rc = run_pass2(ctx, d_theta, store, st);
    if (rc) return rc;
    ctx->ckpt_valid = true;   // either pass wrote every segment
    e = reduce_grad(ctx, d_grad, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "reduce launch");
    return CAL_OK;
}

// --- the allocation-free gradient ------------------------------------------------
// One static device array per device holds every buffer calibrate_gradient_static
// needs beyond its caller's inputs and outputs.  Host code never passes the
// array's name to a kernel or a copy: it uses the address hipGetSymbolAddress
// returns for the current device, taken once per device on the first call there.
namespace {

constexpr int kMaxDevices = 64;
constexpr size_t kAlign = 256;

}  // namespace

static __device__ __align__(256) unsigned char scratch[CAL_STATIC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[kMaxDevices] = {};

static int scratch_address(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, CAL_EUNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = (unsigned char *)p;
    }
    *out = g_scratch_ptr[dev];
    return CAL_OK;
}

__global__ void k_clear_status(int32_t *status)
{
    if (threadIdx.x == 0) *status = 0;
}

static size_t align_up(size_t o)
{
    return (o + kAlign - 1) / kAlign * kAlign;
}

extern "C" int calibrate_gradient_static(const cal_problem *pb, const double *d_theta, const double *d_C,
                                         double *d_Ey, double *d_G, double *d_grad, int32_t *d_status, void *stream)
{
    int code;
    std::string msg = validate(pb, &code);
    if (code != CAL_OK) return fail(nullptr, code, msg);
    if (pb->model != CAL_BS && pb->model != CAL_HESTON)
        return fail(nullptr, CAL_EUNSUPPORTED, "calibrate_gradient_static serves Black-Scholes and Heston");
    if (!d_theta || !d_C || !d_Ey || !d_G || !d_grad || !d_status)
        return fail(nullptr, CAL_EINVAL, "null device pointer");
    const bool fp64 = pb->precision == CAL_FP64;
    const size_t real = fp64 ? 8 : 4;
    const int m = pb->n_instr, M = pb->n_params, N = pb->n_steps;
    const int64_t P = pb->n_paths;
    const int ppl = pb->paths_per_lane > 0 ? pb->paths_per_lane : 1;
    const int K = pb->ckpt_every ? pb->ckpt_every : (fp64 ? 8 : 16);
    const int nv = pb->model == CAL_HESTON ? 2 : 1;
    const int nseg = (N + K - 1) / K;
    const int64_t nblocks = (P + (int64_t)kBlock * ppl - 1) / ((int64_t)kBlock * ppl);
    const bool store = pb->ckpt_mode != CAL_CKPT_RERUN;

    thread_local Tables tb;   // host staging; keeps its capacity between calls
    build_tables(pb, tb);
    const int nd = (int)tb.date_step.size();

    // layout of the scratch array: the tables, then the pass buffers
    size_t o = 0;
    const size_t o_date_step = o;
    o = align_up(o + sizeof(int32_t) * nd);
    const size_t o_date_begin = o;
    o = align_up(o + sizeof(int32_t) * (nd + 1));
    const size_t o_strike = o;
    o = align_up(o + sizeof(double) * m);
    const size_t o_strike_f = o;
    o = align_up(o + sizeof(float) * m);
    const size_t o_disc = o;
    o = align_up(o + sizeof(double) * m);
    const size_t o_id = o;
    o = align_up(o + sizeof(int32_t) * m);
    const size_t tables_end = o;
    const size_t o_part_y = o;
    o = align_up(o + sizeof(double) * (size_t)nblocks * m);
    const size_t o_part_g = o;
    o = align_up(o + sizeof(double) * (size_t)nblocks * M);
    const size_t o_lamD = o;
    o = align_up(o + real * m);
    const size_t o_ckpt = o;
    o = align_up(o + real * (size_t)nseg * nv * (size_t)P);
    if (o > (size_t)CAL_STATIC_SCRATCH_BYTES)
        return fail(nullptr, CAL_EINVAL,
                    "problem needs " + std::to_string(o) + " bytes of scratch, more than the " +
                        std::to_string((size_t)CAL_STATIC_SCRATCH_BYTES) +
                        " of the static buffer (fewer paths, or a wider checkpoint spacing)");

    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
    unsigned char *base = nullptr;
    int rc = scratch_address(dev, &base);
    if (rc) return rc;

    thread_local std::vector<unsigned char> stage;
    stage.assign(tables_end, 0);
    std::memcpy(stage.data() + o_date_step, tb.date_step.data(), sizeof(int32_t) * nd);
    std::memcpy(stage.data() + o_date_begin, tb.date_begin.data(), sizeof(int32_t) * (nd + 1));
    std::memcpy(stage.data() + o_strike, tb.strike.data(), sizeof(double) * m);
    std::memcpy(stage.data() + o_strike_f, tb.strike_f.data(), sizeof(float) * m);
    std::memcpy(stage.data() + o_disc, tb.disc.data(), sizeof(double) * m);
    std::memcpy(stage.data() + o_id, tb.order.data(), sizeof(int32_t) * m);
    hipStream_t st = (hipStream_t)stream;
    e = hipMemcpyAsync(base, stage.data(), tables_end, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);   // the staging buffer is reused by the next call
    if (e != hipSuccess) return hip_fail(nullptr, e, "table upload");

    DevProblem d{};
    set_scalars(d, pb, nd, nseg, K, ppl);
    d.date_step = (const int32_t *)(base + o_date_step);
    d.date_begin = (const int32_t *)(base + o_date_begin);
    d.strike = (const double *)(base + o_strike);
    d.strike_f = (const float *)(base + o_strike_f);
    d.disc = (const double *)(base + o_disc);
    d.id = (const int32_t *)(base + o_id);
    d.status = d_status;
    d.theta_save = nullptr;
    double *part_y = (double *)(base + o_part_y), *part_g = (double *)(base + o_part_g);
    void *lamD = base + o_lamD, *ckpt = base + o_ckpt;

    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, st, d_status);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_pass1(d, pb->model, fp64, store, d_theta, part_y, ckpt, nblocks, st);
    if (e == hipSuccess) e = launch_reduce_sorted(part_y, nblocks, m, d.id, 1.0 / (double)P, d_Ey, d_status, st);
    if (e == hipSuccess) e = launch_residual(d, fp64, d_Ey, d_C, d_G, lamD, d_theta, st);
    if (e == hipSuccess) e = launch_pass2(d, pb->model, fp64, store, d_theta, lamD, part_g, ckpt, nblocks, st);
    if (e == hipSuccess) e = launch_reduce_sorted(part_g, nblocks, M, nullptr, 1.0, d_grad, d_status, st);
    if (e != hipSuccess) return hip_fail(nullptr, e, "launch");
    return CAL_OK;
}

extern "C" int calibrate_jacobian_batch(cal_ctx *ctx, const double *d_theta, int32_t n_inst, uint32_t inst0,
                                        double *d_Ey, double *d_J, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!d_theta || !d_Ey || !d_J) return fail(ctx, CAL_EINVAL, "null device pointer");
    if (ctx->model != CAL_BS && ctx->model != CAL_HESTON)
        return fail(ctx, CAL_EUNSUPPORTED, "tangent mode serves Black-Scholes (log-Euler) and Heston");
    if (n_inst < 1 || n_inst > ctx->max_batch) return fail(ctx, CAL_EINVAL, "n_inst outside 1..max_batch");
    if ((size_t)ctx->m * (ctx->M + 1) * kWavesPerBlock * sizeof(double) > 64 * 1024)
        return fail(ctx, CAL_EUNSUPPORTED, "m * (M + 1) too large for the tangent kernel's LDS");
    hipStream_t st = (hipStream_t)stream;
    DevProblem dp = ctx->dp;
    dp.inst = inst0;
    hipError_t e;
    {
        Timed t(ctx, st, 2);
        e = launch_tangent(dp, ctx->model, ctx->fp64, d_theta, ctx->d_part_j, ctx->nblocks_tan, n_inst, st);
        t.done();
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "tangent launch");
    e = launch_reduce_jac(ctx->d_part_j, ctx->nblocks_tan, ctx->M, ctx->m, ctx->d_id, 1.0 / (double)ctx->P, d_Ey, d_J,
                          ctx->d_status, n_inst, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "reduce launch");
    return CAL_OK;
}

extern "C" int calibrate_jacobian(cal_ctx *ctx, const double *d_theta, double *d_Ey, double *d_J, void *stream)
{
    if (!ctx) return fail(nullptr, CAL_EINVAL, "null context");
    return calibrate_jacobian_batch(ctx, d_theta, 1, ctx->dp.inst, d_Ey, d_J, stream);
}

extern "C" int cal_status(cal_ctx *ctx, void *stream)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    int32_t flags = 0;
    hipError_t e = hipMemcpyAsync(&flags, ctx->d_status, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->d_status, 0, sizeof(int32_t), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(ctx, e, "status read");
    return flags;
}

extern "C" const char *cal_last_error(const cal_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_err.c_str();
}

extern "C" int cal_philox(const uint32_t *d_ctr, uint32_t key0, uint32_t key1, int64_t n, uint32_t *d_out,
                          void *stream)
{
    if (n < 0 || (n > 0 && (!d_ctr || !d_out))) return fail(nullptr, CAL_EINVAL, "bad philox arguments");
    if (n == 0) return CAL_OK;
    hipError_t e = launch_philox(d_ctr, key0, key1, n, d_out, (hipStream_t)stream);
    return e == hipSuccess ? CAL_OK : hip_fail(nullptr, e, "philox launch");
}

extern "C" int cal_normals(int32_t precision, uint64_t seed, uint32_t inst, uint32_t path0, int64_t n_paths,
                           uint32_t q0, int32_t nq, void *d_out, void *stream)
{
    if ((precision != CAL_FP32 && precision != CAL_FP64) || n_paths < 0 || nq < 0)
        return fail(nullptr, CAL_EINVAL, "bad normals arguments");
    if (n_paths == 0 || nq == 0) return CAL_OK;
    if (!d_out) return fail(nullptr, CAL_EINVAL, "null output");
    hipError_t e = launch_normals(precision == CAL_FP64, (uint32_t)seed, (uint32_t)(seed >> 32), inst, path0, n_paths,
                                  q0, nq, d_out, (hipStream_t)stream);
    return e == hipSuccess ? CAL_OK : hip_fail(nullptr, e, "normals launch");
}

// ---------------------------------------------------------------------------
// Batched instances
// ---------------------------------------------------------------------------
struct calb_ctx {
    int device = 0;
    int model = 0;
    bool fp64 = false;
    int n_inst = 0;
    int M = 0;
    int K = 16;
    int wpc = 0;                       // persistent workgroups per CU (0 = occupancy limit)
    int ppl = 1;                       // paths per lane
    int cus = 256;
    std::vector<BatchInst> host;       // descriptors (device pointers inside)
    std::vector<int64_t> offsets;      // [n_inst + 1] instrument offsets
    std::vector<int> nsteps;
    std::vector<int64_t> npaths;
    std::vector<int> order;            // instances, more steps first
    int2 *d_items = nullptr;
    BatchLaunch L{};
    std::vector<void *> allocs;
    int32_t *d_status = nullptr;
    BatchInst *d_insts = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string err;
};

static int bfail(calb_ctx *c, int code, const std::string &m)
{
    if (c) c->err = m;
    g_err = m;
    return code;
}

extern "C" int calb_destroy(calb_ctx *c)
{
    if (!c) return CAL_OK;
    (void)hipDeviceSynchronize();
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    for (void *p : c->allocs) (void)hipFree(p);
    delete c;
    return CAL_OK;
}

// Descriptors and work items for the current checkpoint spacing and paths
// per lane, uploaded synchronously.  Items: (instance, workgroup) pairs,
// instances with more steps first, workgroups in order.
static int calb_upload(calb_ctx *c)
{
    std::vector<int2> items;
    for (int i = 0; i < c->n_inst; ++i) {
        BatchInst &I = c->host[i];
        I.pb.K = c->K;
        I.pb.nseg = (c->nsteps[i] + c->K - 1) / c->K;
        I.pb.ppl = c->ppl;
        I.nblocks = (c->npaths[i] + (int64_t)kBlock * c->ppl - 1) / ((int64_t)kBlock * c->ppl);
    }
    for (int i : c->order)
        for (int64_t b = 0; b < c->host[i].nblocks; ++b) items.push_back(make_int2(i, (int)b));
    hipError_t e = hipMemcpy(c->d_insts, c->host.data(), sizeof(BatchInst) * c->n_inst, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bfail(c, CAL_EHIP, std::string("descriptor upload: ") + hipGetErrorString(e));
    c->L.n_items = (int)items.size();
    const int bpc = batch_blocks_per_cu(c->model, c->fp64, c->K, c->L.max_m);
    const int per = c->wpc > 0 ? std::min(c->wpc, bpc) : bpc;
    c->L.grid = (unsigned)std::max(1, std::min(c->L.n_items, per * c->cus));
    c->L.K = c->K;
    if (c->exec) {
        (void)hipGraphExecDestroy(c->exec);
        c->exec = nullptr;
    }
    if (c->graph) {
        (void)hipGraphDestroy(c->graph);
        c->graph = nullptr;
    }
    return CAL_OK;
}

extern "C" int calb_create(const cal_problem *problems, int32_t n_inst, calb_ctx **out)
{
    if (!out || !problems) return bfail(nullptr, CAL_EINVAL, "null argument");
    *out = nullptr;
    if (n_inst < 1 || n_inst > 65535) return bfail(nullptr, CAL_EINVAL, "n_inst must be in 1..65535");
    for (int i = 0; i < n_inst; ++i) {
        int code;
        std::string msg = validate(&problems[i], &code);
        if (code != CAL_OK) return bfail(nullptr, code, "instance " + std::to_string(i) + ": " + msg);
        if (problems[i].model != CAL_BS && problems[i].model != CAL_HESTON)
            return bfail(nullptr, CAL_EUNSUPPORTED, "batches take BS (log-Euler) or Heston");
        if (problems[i].model != problems[0].model || problems[i].precision != problems[0].precision)
            return bfail(nullptr, CAL_EINVAL, "all instances of a batch share model and precision");
    }
    calb_ctx *c = new calb_ctx();
    (void)hipGetDevice(&c->device);
    if (hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || c->cus <= 0) {
        delete c;
        return bfail(nullptr, CAL_EHIP, "device query failed (compute units)");
    }
    c->model = problems[0].model;
    c->fp64 = problems[0].precision == CAL_FP64;
    c->n_inst = n_inst;
    c->M = problems[0].n_params;
    c->K = problems[0].ckpt_every ? problems[0].ckpt_every : (c->fp64 ? 8 : 16);
    const size_t real = c->fp64 ? 8 : 4;
    const int nv = c->model == CAL_HESTON ? 2 : 1;

    // host tables, concatenated
    std::vector<int32_t> date_step, date_begin, ids;
    std::vector<double> strike, disc;
    std::vector<float> strike_f;
    std::vector<size_t> ds_off(n_inst), db_off(n_inst), in_off(n_inst);
    std::vector<size_t> py_off(n_inst), pg_off(n_inst), lam_off(n_inst), ck_off(n_inst);
    std::vector<int64_t> nblocks(n_inst);
    size_t py = 0, pg = 0, lam = 0, ck = 0;
    int max_m = 0;
    c->offsets.assign(n_inst + 1, 0);
    c->nsteps.resize(n_inst);
    c->npaths.resize(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        const cal_problem *pb = &problems[i];
        const int m = pb->n_instr;
        max_m = std::max(max_m, m);
        c->offsets[i + 1] = c->offsets[i] + m;
        c->nsteps[i] = pb->n_steps;
        c->npaths[i] = pb->n_paths;
        std::vector<int32_t> order(m);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return pb->instr_step[a] < pb->instr_step[b]; });
        ds_off[i] = date_step.size();
        db_off[i] = date_begin.size();
        in_off[i] = strike.size();
        const double h = pb->t_max / pb->n_steps;
        int nd = 0;
        for (int k = 0; k < m; ++k) {
            const int s = pb->instr_step[order[k]];
            if (nd == 0 || date_step.back() != s) {
                date_step.push_back(s);
                date_begin.push_back(k);
                ++nd;
            }
            strike.push_back(pb->instr_strike[order[k]]);
            strike_f.push_back((float)pb->instr_strike[order[k]]);
            disc.push_back(std::exp(-pb->rate * s * h));
            ids.push_back(order[k]);
        }
        date_begin.push_back(m);
        nblocks[i] = (pb->n_paths + kBlock - 1) / kBlock;
        py_off[i] = py;
        py += (size_t)nblocks[i] * m;
        pg_off[i] = pg;
        pg += (size_t)nblocks[i] * c->M;
        lam_off[i] = lam;
        lam += (size_t)m;
        ck_off[i] = ck;
        ck += (size_t)((pb->n_steps + 7) / 8) * nv * (size_t)pb->n_paths;   // sized for the densest spacing
        BatchInst &I = c->host.emplace_back();
        std::memset(&I, 0, sizeof(I));
        DevProblem &d = I.pb;
        d.N = pb->n_steps;
        d.m = m;
        d.M = c->M;
        d.ndates = nd;
        d.P = pb->n_paths;
        d.k0 = (uint32_t)pb->seed;
        d.k1 = (uint32_t)(pb->seed >> 32);
        d.inst = pb->inst;
            d.s0 = pb->s0;
        d.rate = pb->rate;
        d.h = h;
        d.sq = std::sqrt(h);
            I.nblocks = nblocks[i];
        I.y_off = (int32_t)c->offsets[i];
    }
    hipError_t e = hipSuccess;
    auto A = [&](void **p, size_t bytes) {
        if (e != hipSuccess) return;
        e = hipMalloc(p, bytes ? bytes : 16);
        if (e == hipSuccess) c->allocs.push_back(*p);
    };
    int32_t *d_ds, *d_db, *d_id;
    double *d_strike, *d_disc, *d_py, *d_pg;
    float *d_strike_f;
    void *d_lam, *d_ck;
    int2 *d_items;
    unsigned *d_counters;
    A((void **)&d_ds, 4 * date_step.size());
    A((void **)&d_db, 4 * date_begin.size());
    A((void **)&d_id, 4 * ids.size());
    A((void **)&d_strike, 8 * strike.size());
    A((void **)&d_strike_f, 4 * strike_f.size());
    A((void **)&d_disc, 8 * disc.size());
    A((void **)&d_py, 8 * py);
    A((void **)&d_pg, 8 * pg);
    A(&d_lam, real * lam);
    A(&d_ck, real * ck);
    A((void **)&c->d_status, 4);
    A((void **)&c->d_insts, sizeof(BatchInst) * n_inst);
    // work items (one path per lane is the most there can be); calb_upload fills them
    c->order.resize(n_inst);
    std::iota(c->order.begin(), c->order.end(), 0);
    std::stable_sort(c->order.begin(), c->order.end(), [&](int a, int b) { return c->nsteps[a] > c->nsteps[b]; });
    size_t max_items = 0;
    for (int i = 0; i < n_inst; ++i) max_items += (size_t)nblocks[i];
    A((void **)&d_items, sizeof(int2) * max_items);
    A((void **)&d_counters, 2 * sizeof(unsigned));
    if (e != hipSuccess) {
        calb_destroy(c);
        return bfail(nullptr, CAL_ENOMEM, std::string("batch workspace allocation failed: ") + hipGetErrorString(e));
    }
    auto H2D = [&](void *dst, const void *src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    };
    H2D(d_ds, date_step.data(), 4 * date_step.size());
    H2D(d_db, date_begin.data(), 4 * date_begin.size());
    H2D(d_id, ids.data(), 4 * ids.size());
    H2D(d_strike, strike.data(), 8 * strike.size());
    H2D(d_strike_f, strike_f.data(), 4 * strike_f.size());
    H2D(d_disc, disc.data(), 8 * disc.size());
    if (e == hipSuccess) e = hipMemset(c->d_status, 0, 4);
    if (e != hipSuccess) {
        calb_destroy(c);
        return bfail(nullptr, CAL_EHIP, std::string("batch table upload failed: ") + hipGetErrorString(e));
    }
    for (int i = 0; i < n_inst; ++i) {
        BatchInst &I = c->host[i];
        DevProblem &d = I.pb;
        d.date_step = d_ds + ds_off[i];
        d.date_begin = d_db + db_off[i];
        d.strike = d_strike + in_off[i];
        d.strike_f = d_strike_f + in_off[i];
        d.disc = d_disc + in_off[i];
        d.id = d_id + in_off[i];
        d.status = c->d_status;
        d.ppl = 1;
        I.part_y = d_py + py_off[i];
        I.part_g = d_pg + pg_off[i];
        I.lamD = (char *)d_lam + real * lam_off[i];
        I.ckpt = (char *)d_ck + real * ck_off[i];
    }
    c->L.model = c->model;
    c->L.fp64 = c->fp64;
    c->L.n_inst = n_inst;
    c->L.max_m = max_m;
    c->L.insts = c->d_insts;
    c->L.items = d_items;
    c->d_items = d_items;
    c->L.counters = d_counters;
    int rc = calb_upload(c);
    if (rc) {
        calb_destroy(c);
        return rc;
    }
    *out = c;
    return CAL_OK;
}

extern "C" int calb_offsets(const calb_ctx *c, int64_t *instr_offsets)
{
    if (!c || !instr_offsets) return CAL_EINVAL;
    for (int i = 0; i <= c->n_inst; ++i) instr_offsets[i] = c->offsets[i];
    return CAL_OK;
}

extern "C" int calb_configure(calb_ctx *c, int32_t ckpt_every, int32_t workgroups_per_cu, int32_t paths_per_lane)
{
    if (!c) return bfail(nullptr, CAL_EINVAL, "null context");
    if (ckpt_every != 8 && ckpt_every != 16 && ckpt_every != 32) return bfail(c, CAL_EINVAL, "ckpt_every must be 8, 16 or 32");
    if (workgroups_per_cu < 0 || workgroups_per_cu > 64) return bfail(c, CAL_EINVAL, "workgroups_per_cu in 0..64");
    if (paths_per_lane != 1 && paths_per_lane != 2 && paths_per_lane != 4)
        return bfail(c, CAL_EINVAL, "paths_per_lane must be 1, 2 or 4");
    (void)hipDeviceSynchronize();
    c->K = ckpt_every;
    c->wpc = workgroups_per_cu;
    c->ppl = paths_per_lane;
    return calb_upload(c);
}

extern "C" int calb_geometry(const calb_ctx *c, int32_t *ckpt_every, int32_t *grid, int32_t *n_items,
                             int32_t *paths_per_lane)
{
    if (!c) return CAL_EINVAL;
    if (ckpt_every) *ckpt_every = c->K;
    if (grid) *grid = (int32_t)c->L.grid;
    if (n_items) *n_items = c->L.n_items;
    if (paths_per_lane) *paths_per_lane = c->ppl;
    return CAL_OK;
}

static int calb_bind(calb_ctx *c, const double *d_theta, const double *d_C, double *d_Ey, double *d_G, double *d_grad)
{
    if (!c) return bfail(nullptr, CAL_EINVAL, "null context");
    if (!d_theta || !d_C || !d_Ey || !d_G || !d_grad) return bfail(c, CAL_EINVAL, "null device pointer");
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != c->device) return bfail(c, CAL_EINVAL, "context belongs to another device");
    c->L.theta = d_theta;
    c->L.C = d_C;
    c->L.Ey = d_Ey;
    c->L.G = d_G;
    c->L.grad = d_grad;
    c->err.clear();
    return CAL_OK;
}

extern "C" int calibrate_gradient_batch(calb_ctx *c, const double *d_theta, const double *d_C, double *d_Ey,
                                        double *d_G, double *d_grad, void *stream)
{
    int rc = calb_bind(c, d_theta, d_C, d_Ey, d_G, d_grad);
    if (rc) return rc;
    hipError_t e = launch_batch_step(c->L, (hipStream_t)stream);
    return e == hipSuccess ? CAL_OK : bfail(c, CAL_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
}

extern "C" int calb_capture(calb_ctx *c, const double *d_theta, const double *d_C, double *d_Ey, double *d_G,
                            double *d_grad, void *stream)
{
    int rc = calb_bind(c, d_theta, d_C, d_Ey, d_G, d_grad);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (!st) return bfail(c, CAL_EINVAL, "capture needs a created (non-null) stream");
    if (c->exec) {
        (void)hipGraphExecDestroy(c->exec);
        c->exec = nullptr;
    }
    if (c->graph) {
        (void)hipGraphDestroy(c->graph);
        c->graph = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bfail(c, CAL_EHIP, std::string("begin capture: ") + hipGetErrorString(e));
    hipError_t el = launch_batch_step(c->L, st);
    e = hipStreamEndCapture(st, &c->graph);
    if (el != hipSuccess || e != hipSuccess)
        return bfail(c, CAL_EHIP, std::string("capture: ") + hipGetErrorString(el != hipSuccess ? el : e));
    e = hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return bfail(c, CAL_EHIP, std::string("instantiate: ") + hipGetErrorString(e));
    return CAL_OK;
}

extern "C" int calb_replay(calb_ctx *c, void *stream)
{
    if (!c) return bfail(nullptr, CAL_EINVAL, "null context");
    if (!c->exec) return bfail(c, CAL_EINVAL, "no captured step (call calb_capture first)");
    hipError_t e = hipGraphLaunch(c->exec, (hipStream_t)stream);
    return e == hipSuccess ? CAL_OK : bfail(c, CAL_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
}

extern "C" int calb_status(calb_ctx *c, void *stream)
{
    if (!c) return bfail(nullptr, CAL_EINVAL, "null context");
    hipStream_t st = (hipStream_t)stream;
    int32_t flags = 0;
    hipError_t e = hipMemcpyAsync(&flags, c->d_status, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemsetAsync(c->d_status, 0, 4, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bfail(c, CAL_EHIP, std::string("status read: ") + hipGetErrorString(e));
    return flags;
}

extern "C" const char *calb_last_error(const calb_ctx *c) { return c ? c->err.c_str() : g_err.c_str(); }
