// Per-lane model arithmetic shared by the Monte Carlo passes: constants from
// theta, the Euler steps of Black-Scholes and Heston in the sweep variables,
// and the parameter-domain check.  gfx950, one path per lane.
#pragma once

#include <hip/hip_runtime.h>

#include "mc_device.hpp"
#include "mc_kernels.hpp"

namespace mcaad {

// ---------------------------------------------------------------------------
// Model constants, computed per lane from theta (uniform values)
//
// Variables of the sweeps (same maps as the paper's F, rewritten to save
// instructions; the oracle keeps the textbook form):
//   z'  = sqrt(h) z: the normals come out of Box-Muller already scaled
//         (h goes under its square root), so no step multiplies by sqrt(h);
//   x~  = x - n r h: the log-price without its deterministic drift, which is
//         added back only where a payoff needs S = s0 exp(x~ + n r h);
//   w'  = rho z1' + rho' z2', the variance shock, rho' = sqrt(1 - rho^2).
// Black-Scholes:  x~ <- x~ - sigma^2 h / 2 + sigma z'
// Heston:         x~ <- x~ - (h/2) v+ + s z1'
//                 v  <- v + (kappa theta_bar h - kappa h v+) + xi s w'
//                 with v+ = max(v, 0), s = sqrt(v+) (full truncation).
// ---------------------------------------------------------------------------
template <typename R>
struct Consts {
    R s0, rh, bm;          // spot, r h, Box-Muller constant for normals scaled by sqrt(h)
    R bs_drift, bs_vol, bs_gh;   // -sigma^2 h/2, sigma, -sigma h
    R hh, kh, khth, xi, rho, rhop, thbh, h, v0;
    // FP64 factors turning a segment's FP32 sums into gradient terms (Heston)
    double g_kh, g_rho;   // kappa h, xi / (1 - rho^2)
};

template <typename R>
__device__ __forceinline__ R exp_r(R x)
{
    if constexpr (sizeof(R) == 4) return __expf(x);
    else return exp(x);
}

template <int MODEL, typename R>
__device__ __forceinline__ void load_consts(const DevProblem &pb, const double *th, Consts<R> &c)
{
    c.s0 = (R)pb.s0;
    c.rh = (R)(pb.rate * pb.h);
    c.bm = box_muller_scale<R>(pb.h);
    if constexpr (MODEL == kBS) {
        const double sig = th[0];
        c.bs_drift = (R)(-0.5 * sig * sig * pb.h);
        c.bs_vol = (R)sig;
        c.bs_gh = (R)(-sig * pb.h);
    } else {
        const double kap = th[0], thb = th[1], xi = th[2], rho = th[3], v0 = th[4];
        c.hh = (R)(0.5 * pb.h);
        c.kh = (R)(kap * pb.h);
        c.khth = (R)(kap * thb * pb.h);
        c.xi = (R)xi;
        c.rho = (R)rho;
        c.rhop = (R)sqrt(1.0 - rho * rho);
        c.thbh = (R)(thb * pb.h);
        c.h = (R)pb.h;
        c.v0 = (R)v0;
        c.g_kh = kap * pb.h;
        c.g_rho = xi / (1.0 - rho * rho);
    }
}

// v+ = max(v, 0).  In FP32 one integer max on the bit pattern: a float with
// the sign bit set is a negative int32 (so -0 and negatives give +0), with no
// canonicalising instruction in front as the float max needs.
template <typename R>
__device__ __forceinline__ R vplus(R v)
{
    if constexpr (sizeof(R) == 4) return __int_as_float(max(__float_as_int(v), 0));
    else return fmax(v, 0.0);
}

template <typename R>
__device__ __forceinline__ R sqrt_r(R v)
{
    if constexpr (sizeof(R) == 4) return __builtin_amdgcn_sqrtf(v);
    else return sqrt(v);
}

template <typename R>
__device__ __forceinline__ R rcp_r(R s)
{
    if constexpr (sizeof(R) == 4) return __builtin_amdgcn_rcpf(s);
    else return 1.0 / s;
}

// S = s0 exp(x~ + n r h) after step n-1, i.e. at time n h
template <typename R>
__device__ __forceinline__ R spot(const Consts<R> &c, R xt, int n)
{
    return c.s0 * exp_r(xt + (R)n * c.rh);
}

// One Heston step on (x~, v) with scaled normals z0, z1; returns what the
// reverse sweep needs (v+, s, w').  Every sweep steps through this function,
// so all passes follow bitwise the same path.
template <typename R>
struct HestonStep {
    R vp, s, w;
};

template <typename R>
__device__ __forceinline__ HestonStep<R> heston_step(const Consts<R> &c, R &x, R &v, R z0, R z1)
{
    HestonStep<R> q;
    q.vp = vplus(v);
    q.s = sqrt_r(q.vp);
    q.w = c.rhop * z1 + c.rho * z0;
    x = q.s * z0 + (x - c.hh * q.vp);
    v = q.s * (c.xi * q.w) + (v + (c.khth - c.kh * q.vp));
    return q;
}

// One Euler step of the forward algorithm F on (x~, v); z = the step's scaled normals.
template <int MODEL, typename R>
__device__ __forceinline__ void euler_step(const Consts<R> &c, R &x, R &v, const R *z)
{
    if constexpr (MODEL == kBS) x = x + c.bs_drift + c.bs_vol * z[0];
    else (void)heston_step(c, x, v, z[0], z[1]);
}

// Workgroups covering the problem's paths (kBlock lanes x ppl paths each);
// block partials are stored [column][workgroup], so each column's
// fixed-order sum reads contiguous memory.
__device__ __forceinline__ int64_t nblocks_of(const DevProblem &pb)
{
    const int64_t per = (int64_t)kBlock * pb.ppl;
    return (pb.P + per - 1) / per;
}

template <int MODEL>
struct Traits;
template <>
struct Traits<kBS> {
    static constexpr int D = 1;   // normals per step
    static constexpr int NV = 1;  // state variables in a checkpoint
    static constexpr int NP = 1;  // parameters
};
template <>
struct Traits<kHeston> {
    static constexpr int D = 2;
    static constexpr int NV = 2;
    static constexpr int NP = 5;
};

// Flags theta outside the model's domain (one lane of the grid).
template <int MODEL>
__device__ void check_theta(const DevProblem &pb, const double *th)
{
    bool ok;
    if constexpr (MODEL == kBS) {
        ok = isfinite(th[0]) && th[0] >= 0.0;
    } else {
        ok = true;
        for (int j = 0; j < 5; ++j) ok = ok && isfinite(th[j]);
        ok = ok && th[0] >= 0.0 && th[1] >= 0.0 && th[2] >= 0.0 && th[3] > -1.0 && th[3] < 1.0 && th[4] >= 0.0;
    }
    if (!ok) atomicOr(pb.status, 1);
}

}  // namespace mcaad
