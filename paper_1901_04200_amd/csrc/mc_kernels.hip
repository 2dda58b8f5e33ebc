// Monte Carlo passes of the two-pass adjoint calibration gradient on gfx950.
//
// One path per lane, path state in VGPRs, normals regenerated from the
// counter-based Philox stream whenever they are needed (never stored), FP64
// sums over paths: wavefront sum by cross-lane moves (eight values per
// reduction where there are several) -> LDS (one slot per wave) -> one FP64
// partial per workgroup -> fixed-order final sum in a separate kernel.
//
//  pass 1 (paper: algorithm step 1, cost eq. 1211A)
//      Euler sweep F_v, payoffs at maturity dates, block partials of sum y_i;
//      optionally stores the state every K steps (in the paper's step 2 the
//      results of step 1 are kept in memory).
//  pass 2 (paper: algorithm step 2, eq. 0711A; step 3 is the final sum)
//      per path: forward sweep again (or the stored checkpoints), then for
//      every K-step segment from the last to the first: reload the segment's
//      checkpoint, recompute its K steps keeping states and normals in
//      registers, and run the reverse sweep R_v over them seeded with
//      lambda_i D_i / P at the maturity dates.
//  tangent
//      forward sweep carrying dx/dtheta, dv/dtheta (Jacobian of E y).
#include <hip/hip_runtime.h>

#include "mc_device.hpp"
#include "mc_kernels.hpp"
#include "models.hpp"

namespace mcaad {

// ---------------------------------------------------------------------------
// Pass 1: forward sweep, payoffs, block partials of sum_p y_i(p)
// ---------------------------------------------------------------------------
// One workgroup's share: paths blk*256 .. blk*256+255; lds holds
// [kWavesPerBlock][m] doubles.
// Wave priority from the share of the wave's work still ahead (left of
// total units, uniform in the wave): waves with more left are issued first, so
// the waves sharing a SIMD finish closer together and fewer run alone,
// latency-bound, at the end of the launch (the forward sweep: 4% shorter at
// 2^20 paths; the reverse sweep gains nothing from it, nor do the persistent
// batched grids, whose waves keep taking new items until the queue is empty).
__device__ __forceinline__ void prio_by_work_left(int left, int total)
{
    switch ((4 * left) / (total + 1)) {
    case 0: __builtin_amdgcn_s_setprio(0); break;
    case 1: __builtin_amdgcn_s_setprio(1); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    default: __builtin_amdgcn_s_setprio(3); break;
    }
}

template <int MODEL, typename R, bool STORE, bool PRIO>
__device__ __forceinline__ void pass1_block(const DevProblem &pb, const double *__restrict__ theta,
                                            double *__restrict__ partial, R *__restrict__ ckpt, int64_t blk,
                                            double *lds)
{
    using T = Traits<MODEL>;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    if (blk == 0 && tid == 0) check_theta<MODEL>(pb, theta);
    if constexpr (STORE) save_theta(pb, theta, blk);

    Consts<R> c;
    load_consts<MODEL, R>(pb, theta, c);
    constexpr int SPC = 4 / T::D;   // steps per Philox call
    const int ncalls = (pb.N * T::D + 3) / 4;
    // Philox calls per checkpoint segment (K is a multiple of SPC; at least one
    // call per segment whatever K holds, so the loop below always advances)
    const int cps = max(pb.K / SPC, 1);
    // the workgroup's paths: ppl runs of kBlock consecutive paths, one after another
    for (int sp = 0; sp < pb.ppl; ++sp) {
        const int64_t p = (blk * pb.ppl + sp) * kBlock + tid;
        const bool active = p < pb.P;
        const uint32_t path = (uint32_t)p;
        R x = (R)0;
        R v = MODEL == kHeston ? c.v0 : (R)0;
        int d = 0;
        int next = pb.ndates > 0 ? ldc(pb.date_step, 0) : -1;
        // segments of K steps; the state at a segment's start is its checkpoint
        R *cp = ckpt + p;
        for (int call = 0; call < ncalls; cp += (int64_t)T::NV * pb.P) {
            if constexpr (PRIO) prio_by_work_left((pb.ppl - sp) * ncalls - call, pb.ppl * ncalls);
            if constexpr (STORE) {
                if (active) {
                    cp[0] = x;
                    if constexpr (T::NV == 2) cp[pb.P] = v;
                }
            }
            const int cend = min(call + cps, ncalls);
            for (; call < cend; ++call) {
                R z[4];
                normals4<R>((uint32_t)call, path, pb.inst, pb.k0, pb.k1, c.bm, z);
#pragma unroll
                for (int j = 0; j < SPC; ++j) {
                    const int n = call * SPC + j;
                    if (n < pb.N) {
                        euler_step<MODEL, R>(c, x, v, z + j * T::D);
                        if (n + 1 == next) {
                            const double S = (double)spot(c, x, n + 1);
                            payoff_sums(pb.strike, pb.disc, S, active, lane, ldc(pb.date_begin, d),
                                        ldc(pb.date_begin, d + 1), lds + wave * pb.m, sp > 0);
                            ++d;
                            next = d < pb.ndates ? ldc(pb.date_step, d) : -1;
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int k = tid; k < pb.m; k += kBlock) {
        double s = lds[k];
#pragma unroll
        for (int w = 1; w < kWavesPerBlock; ++w) s += lds[w * pb.m + k];
        partial[(int64_t)k * nblocks_of(pb) + blk] = s;
    }
}

template <int MODEL, typename R, bool STORE>
__global__ __launch_bounds__(kBlock) void k_pass1(DevProblem pb, const double *__restrict__ theta,
                                                  double *__restrict__ partial, R *__restrict__ ckpt)
{
    extern __shared__ double lds[];
    pass1_block<MODEL, R, STORE, true>(pb, theta, partial, ckpt, blockIdx.x, lds);
}

// ---------------------------------------------------------------------------
// Pass 2: (re-run forward with checkpoints) + reverse sweep, block partials
// of sum_p thetabar(p)
// ---------------------------------------------------------------------------
// LDS bytes of one pass-2 workgroup: [kWavesPerBlock][NP] doubles for the
// gradient sums, then [K][kBlock] reals, one column per lane, for the payoff
// adjoints of the maturity dates of the current segment.
template <int MODEL, typename R, int K>
constexpr size_t pass2_lds_bytes()
{
    return sizeof(double) * kWavesPerBlock * Traits<MODEL>::NP + sizeof(R) * K * kBlock;
}

// One workgroup's share; lds as pass2_lds_bytes describes.
template <int MODEL, typename R, bool FROM_CKPT, int K>
__device__ __forceinline__ void pass2_block(const DevProblem &pb, const double *__restrict__ theta,
                                            const R *__restrict__ lamD, double *__restrict__ partial,
                                            R *__restrict__ ckpt, int64_t blk, double *lds)
{
    using T = Traits<MODEL>;
    constexpr int NP = T::NP;
    constexpr int SPC = 4 / T::D;
    static_assert(K % SPC == 0, "segments must start on a Philox call");
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;

    Consts<R> c;
    load_consts<MODEL, R>(pb, theta, c);
    const R *strike_r;
    if constexpr (sizeof(R) == 4) strike_r = pb.strike_f;
    else strike_r = pb.strike;
    R *inj_lds = reinterpret_cast<R *>(lds + kWavesPerBlock * NP);

    if constexpr (!FROM_CKPT) save_theta(pb, theta, blk);

    double g[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) g[j] = 0.0;
    // the workgroup's paths: ppl runs of kBlock consecutive paths, one after another
    for (int sp = 0; sp < pb.ppl; ++sp) {
        const int64_t p = (blk * pb.ppl + sp) * kBlock + tid;
        const bool active = p < pb.P;
        const uint32_t path = (uint32_t)p;

        if constexpr (!FROM_CKPT) {
            // The forward re-run of the paper's step 2: sweep again, keep the state
            // at the start of every segment.
            R x = (R)0;
            R v = MODEL == kHeston ? c.v0 : (R)0;
            const int ncalls = (pb.N * T::D + 3) / 4;
            for (int call = 0; call < ncalls; ++call) {
                R z[4];
                normals4<R>((uint32_t)call, path, pb.inst, pb.k0, pb.k1, c.bm, z);
#pragma unroll
                for (int j = 0; j < SPC; ++j) {
                    const int n = call * SPC + j;
                    if (n < pb.N) {
                        if ((n % K) == 0 && active) {
                            const int64_t base = (int64_t)((n / K) * T::NV) * pb.P + p;
                            ckpt[base] = x;
                            if constexpr (T::NV == 2) ckpt[base + pb.P] = v;
                        }
                        euler_step<MODEL, R>(c, x, v, z + j * T::D);
                    }
                }
            }
        }

        R xb = (R)0, vb = (R)0;     // adjoints of the state after the current step
        const double on = active ? 1.0 : 0.0;   // inactive lanes add nothing
        int dhi = pb.ndates;        // dates with index < dhi mature at or before this segment's end

        // The checkpoint of the segment after the current one is requested
        // before the current segment's sweeps run, so that its load latency
        // is hidden behind them.  Inactive lanes (past the last path) load
        // path 0's slot but run a harmless path from (0, v0) instead and add
        // nothing: in the re-run mode another workgroup may still be writing
        // that slot.
        const int64_t pl = active ? p : 0;
        R x_next = ckpt[(int64_t)((pb.nseg - 1) * T::NV) * pb.P + pl];
        R v_next = (R)0;
        if constexpr (T::NV == 2) v_next = ckpt[(int64_t)((pb.nseg - 1) * T::NV + 1) * pb.P + pl];
        for (int seg = pb.nseg - 1; seg >= 0; --seg) {
            const int n0 = seg * K;
            R x = active ? x_next : (R)0;
            R v = (R)0;
            if constexpr (MODEL == kHeston) v = active ? v_next : c.v0;
            if (seg > 0) {
                const int64_t base = (int64_t)((seg - 1) * T::NV) * pb.P + pl;
                x_next = ckpt[base];
                if constexpr (T::NV == 2) v_next = ckpt[base + pb.P];
            }
            int dlo = dhi;
            while (dlo > 0 && ldc(pb.date_step, dlo - 1) > n0) --dlo;
            int d = dlo;
            int next = d < dhi ? ldc(pb.date_step, d) : -1;

            // recompute the segment, keeping what the reverse sweep needs in
            // registers (Heston: z1', w', s = sqrt(v+) of every step, v+ is taken
            // back as s^2; Black-Scholes: z'), and the payoff adjoint of a
            // maturity date in this lane's LDS column
            R s_z1[K], s_w[K], s_s[K];
            R z[4];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int n = n0 + j;
                s_z1[j] = (R)0;
                s_w[j] = (R)0;
                s_s[j] = (R)0;
                if (n < pb.N) {
                    if (j % SPC == 0) normals4<R>((uint32_t)(n / SPC), path, pb.inst, pb.k0, pb.k1, c.bm, z);
                    const R *zs = z + (j % SPC) * T::D;
                    s_z1[j] = zs[0];
                    if constexpr (MODEL == kHeston) {
                        const HestonStep<R> q = heston_step(c, x, v, zs[0], zs[1]);
                        s_w[j] = q.w;
                        s_s[j] = q.s;
                    } else {
                        euler_step<MODEL, R>(c, x, v, zs);
                    }
                    if (n + 1 == next) {
                        // payoff adjoints of this date: sum_i lambda_i D_i / P 1{S > K_i} S
                        const R S = spot(c, x, n + 1);
                        R inj = (R)0;
                        for (int k = ldc(pb.date_begin, d); k < ldc(pb.date_begin, d + 1); ++k)
                            inj += S > ldc(strike_r, k) ? ldc(lamD, k) * S : (R)0;
                        inj_lds[j * kBlock + tid] = inj;
                        ++d;
                        next = d < dhi ? ldc(pb.date_step, d) : -1;
                    }
                }
            }
            dhi = dlo;

            // reverse sweep over the segment; its dates are dlo .. d-1, met last
            // first.  xb, the adjoint of x~, changes only at those dates.
            // Heston: sums over the segment's steps (b = vb before the step)
            //   tk = sum b (theta_bar h - h v+), sb = sum b, t2 = sum b s w',
            //   t3 = sum b s (z1' - rho w'),
            // from which d/d(kappa) = tk, d/d(theta_bar) = kappa h sb, d/d(xi) = t2,
            // d/d(rho) = xi t3 / (1 - rho^2).  (tk is summed per step: its two
            // parts nearly cancel when v+ stays near theta_bar.)
            int dr = d - 1;
            int rnext = dr >= dlo ? ldc(pb.date_step, dr) : -1;
            R ca = -(c.hh * xb);
            R sb = (R)0, tk = (R)0, t2 = (R)0, t3 = (R)0;
#pragma unroll
            for (int j = K - 1; j >= 0; --j) {
                if (n0 + j < pb.N) {
                    if (n0 + j + 1 == rnext) {
                        xb += inj_lds[j * kBlock + tid];
                        ca = -(c.hh * xb);
                        --dr;
                        rnext = dr >= dlo ? ldc(pb.date_step, dr) : -1;
                    }
                    if constexpr (MODEL == kBS) {
                        // d x~' / d sigma = -sigma h + z'
                        sb += xb * (c.bs_gh + s_z1[j]);
                    } else {
                        const R sv = s_s[j], z1 = s_z1[j], w = s_w[j];
                        const R vp = sv * sv;
                        const R b = vb;
                        const R sbar = (b * c.xi) * w + xb * z1;
                        const R vpbar = sbar * ((R)0.5 * rcp_r(sv)) + (ca - c.kh * b);
                        sb += b;
                        tk += b * (c.thbh - c.h * vp);
                        const R t = b * sv;
                        t2 += t * w;
                        t3 += t * (z1 - c.rho * w);
                        vb = sv > (R)0 ? b + vpbar : b;
                    }
                }
            }
            if constexpr (MODEL == kBS) {
                g[0] += on * (double)sb;
            } else {
                g[0] += on * (double)tk;
                g[1] += on * (c.g_kh * (double)sb);
                g[2] += on * (double)t2;
                g[3] += on * (c.g_rho * (double)t3);
            }
        }
        if constexpr (MODEL == kHeston) g[4] += on * (double)vb;   // v_0 is theta[4]
    }

    static_assert(NP <= 8, "one wave_sum8 per path's gradient");
    double a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = j < NP ? g[j] : 0.0;
    const double t = wave_sum8(a);
    if ((lane & 7) == 0 && (lane >> 3) < NP) lds[wave * NP + (lane >> 3)] = t;
    __syncthreads();
    if (tid < NP) {
        double s = lds[tid];
#pragma unroll
        for (int w = 1; w < kWavesPerBlock; ++w) s += lds[w * NP + tid];
        partial[(int64_t)tid * nblocks_of(pb) + blk] = s;
    }
}

template <int MODEL, typename R, bool FROM_CKPT, int K>
__global__ __launch_bounds__(kBlock) void k_pass2(DevProblem pb, const double *__restrict__ theta,
                                                  const R *__restrict__ lamD, double *__restrict__ partial,
                                                  R *__restrict__ ckpt)
{
    extern __shared__ double lds[];
    pass2_block<MODEL, R, FROM_CKPT, K>(pb, theta, lamD, partial, ckpt, blockIdx.x, lds);
}

// ---------------------------------------------------------------------------
// Forward tangent mode: block partials of y_i and dy_i/dtheta_j
// ---------------------------------------------------------------------------
// blockIdx.y selects an instance: its parameters theta + y*M and Philox
// counter word 2 = inst + y; its partials start at partial + y*gridDim.x*m*W.
template <int MODEL, typename R>
__global__ __launch_bounds__(kBlock) void k_tangent(DevProblem pb, const double *__restrict__ theta_all,
                                                    double *__restrict__ partial_all)
{
    using T = Traits<MODEL>;
    constexpr int NP = T::NP;
    constexpr int W = NP + 1;
    static_assert(W <= 8, "E y and its derivatives in one wave_sum8");
    extern __shared__ double lds[];   // [kWavesPerBlock][m * W]
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const int64_t p = (int64_t)blockIdx.x * kBlock + tid;
    const bool active = p < pb.P;
    const uint32_t path = (uint32_t)p;
    const double *theta = theta_all + (int64_t)blockIdx.y * NP;
    double *partial = partial_all + (int64_t)blockIdx.y * gridDim.x * pb.m * W;
    pb.inst += blockIdx.y;
    if (blockIdx.x == 0 && tid == 0) check_theta<MODEL>(pb, theta);

    Consts<R> c;
    load_consts<MODEL, R>(pb, theta, c);
    R x = (R)0;
    R v = MODEL == kHeston ? c.v0 : (R)0;
    R xd[NP], vd[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        xd[j] = (R)0;
        vd[j] = (R)0;
    }
    if constexpr (MODEL == kHeston) vd[4] = (R)1;

    constexpr int SPC = 4 / T::D;
    const int ncalls = (pb.N * T::D + 3) / 4;
    int d = 0;
    int next = pb.ndates > 0 ? pb.date_step[0] : -1;
    for (int call = 0; call < ncalls; ++call) {
        R z[4];
        normals4<R>((uint32_t)call, path, pb.inst, pb.k0, pb.k1, c.bm, z);
#pragma unroll
        for (int j = 0; j < SPC; ++j) {
            const int n = call * SPC + j;
            if (n < pb.N) {
                const R *zs = z + j * T::D;
                if constexpr (MODEL == kBS) {
                    xd[0] += c.bs_gh + zs[0];
                    euler_step<MODEL, R>(c, x, v, zs);
                } else {
                    // tangents of (x~, v) through one step, before the step moves v
                    const bool pos = v > (R)0;
                    const R z1 = zs[0];
                    const HestonStep<R> q = heston_step(c, x, v, z1, zs[1]);
                    const R ds = pos ? (R)0.5 * rcp_r(q.s) : (R)0;
                    const R xw = c.xi * q.w;
                    const R dw_drho = (z1 - c.rho * q.w) * ((R)1 / (c.rhop * c.rhop));
#pragma unroll
                    for (int k = 0; k < NP; ++k) {
                        const R vpd = pos ? vd[k] : (R)0;
                        const R sd = ds * vpd;
                        R direct = (R)0;
                        if (k == 0) direct = c.thbh - c.h * q.vp;
                        if (k == 1) direct = c.kh;
                        if (k == 2) direct = q.s * q.w;
                        if (k == 3) direct = c.xi * q.s * dw_drho;
                        xd[k] = xd[k] - c.hh * vpd + z1 * sd;
                        vd[k] = vd[k] - c.kh * vpd + xw * sd + direct;
                    }
                }
                if (n + 1 == next) {
                    const double S = (double)spot(c, x, n + 1);
                    for (int k = pb.date_begin[d]; k < pb.date_begin[d + 1]; ++k) {
                        // y and its NP derivatives, one wave_sum8
                        const bool itm = active && S > pb.strike[k];
                        const double dS = itm ? pb.disc[k] * S : 0.0;
                        double a[8];
                        a[0] = itm ? pb.disc[k] * (S - pb.strike[k]) : 0.0;
#pragma unroll
                        for (int q = 1; q < 8; ++q) a[q] = q <= NP ? dS * (double)xd[q <= NP ? q - 1 : 0] : 0.0;
                        const double t = wave_sum8(a);
                        if ((lane & 7) == 0 && (lane >> 3) < W) lds[wave * pb.m * W + k * W + (lane >> 3)] = t;
                    }
                    ++d;
                    next = d < pb.ndates ? pb.date_step[d] : -1;
                }
            }
        }
    }
    __syncthreads();
    const int width = pb.m * W;
    for (int k = tid; k < width; k += kBlock) {
        double s = lds[k];
#pragma unroll
        for (int w = 1; w < kWavesPerBlock; ++w) s += lds[w * width + k];
        partial[(int64_t)k * gridDim.x + blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// Fixed-order reductions and the FP64 epilogues
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (tid < s) sh[tid] += sh[tid + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// One workgroup per output column k: thread t sums blocks t, t+256, ... in
// order, then a fixed tree.
__global__ __launch_bounds__(kBlock) void k_reduce_sorted(const double *__restrict__ partial, int64_t nblocks,
                                                          const int32_t *__restrict__ id,
                                                          double scale, double *__restrict__ out,
                                                          int32_t *status)
{
    __shared__ double sh[kBlock];
    const int k = blockIdx.x;
    double acc = 0.0;
    const double *col = partial + (int64_t)k * nblocks;
    for (int64_t b = threadIdx.x; b < nblocks; b += kBlock) acc += col[b];
    const double s = block_sum(acc, sh) * scale;
    if (threadIdx.x == 0) {
        out[id ? id[k] : k] = s;
        if (!isfinite(s)) atomicOr(status, 2);
    }
}

// Tangent-mode columns: k*W + 0 -> Ey[id[k]], k*W + 1 + j -> J[id[k]*M + j];
// blockIdx.y is the instance.
__global__ __launch_bounds__(kBlock) void k_reduce_jac(const double *__restrict__ partial_all, int64_t nblocks,
                                                       int32_t M, int32_t m, const int32_t *__restrict__ id,
                                                       double scale, double *__restrict__ Ey_all,
                                                       double *__restrict__ J_all, int32_t *status)
{
    __shared__ double sh[kBlock];
    const int col = blockIdx.x;
    const int W = M + 1;
    const int width = m * W;
    const double *partial = partial_all + (int64_t)blockIdx.y * nblocks * width;
    double *Ey = Ey_all + (int64_t)blockIdx.y * m;
    double *J = J_all + (int64_t)blockIdx.y * m * M;
    double acc = 0.0;
    const double *cp = partial + (int64_t)col * nblocks;
    for (int64_t b = threadIdx.x; b < nblocks; b += kBlock) acc += cp[b];
    const double s = block_sum(acc, sh) * scale;
    if (threadIdx.x == 0) {
        const int k = col / W, t = col % W;
        if (t == 0) Ey[id[k]] = s;
        else J[(int64_t)id[k] * M + (t - 1)] = s;
        if (!isfinite(s)) atomicOr(status, 2);
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_residual(DevProblem pb, const double *__restrict__ Ey,
                                                     const double *__restrict__ C, double *__restrict__ G,
                                                     R *__restrict__ lamD)
{
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int i = threadIdx.x; i < pb.m; i += kBlock) {
        const double r = Ey[i] - C[i];
        acc += 0.5 * r * r;
    }
    const double g = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        G[0] = g;
        if (!isfinite(g)) atomicOr(pb.status, 2);
    }
    const double invP = 1.0 / (double)pb.P;
    for (int k = threadIdx.x; k < pb.m; k += kBlock) {
        const int i = pb.id[k];
        lamD[k] = (R)((Ey[i] - C[i]) * pb.disc[k] * invP);
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_lambda(DevProblem pb, const double *__restrict__ lambda,
                                                   R *__restrict__ lamD, const double *__restrict__ saved,
                                                   const double *__restrict__ theta)
{
    const double invP = 1.0 / (double)pb.P;
    for (int k = threadIdx.x; k < pb.m; k += kBlock) lamD[k] = (R)(lambda[pb.id[k]] * pb.disc[k] * invP);
    if (saved) {
        // pass 2 is about to read checkpoints written with `saved`: same bits?
        bool same = true;
        for (int i = threadIdx.x; i < pb.M; i += kBlock)
            same = same && __double_as_longlong(theta[i]) == __double_as_longlong(saved[i]);
        if (!same) atomicOr(pb.status, 4);
    }
}

__global__ void k_check_theta(DevProblem pb, const double *theta, int model)
{
    if (model == kBS) {
        if (threadIdx.x == 0) check_theta<kBS>(pb, theta);
    } else if (model == kHeston) {
        if (threadIdx.x == 0) check_theta<kHeston>(pb, theta);
    } else if (model == kSLV) {
        // Heston parameters, then every leverage node finite and >= 0
        if (threadIdx.x == 0) check_theta<kHeston>(pb, theta);
        bool ok = true;
        for (int i = 5 + threadIdx.x; i < pb.M; i += blockDim.x) ok = ok && isfinite(theta[i]) && theta[i] >= 0.0;
        if (!ok) atomicOr(pb.status, 1);
    } else {
        // local volatility: every node value finite and >= 0
        bool ok = true;
        for (int i = threadIdx.x; i < pb.M; i += blockDim.x) ok = ok && isfinite(theta[i]) && theta[i] >= 0.0;
        if (!ok) atomicOr(pb.status, 1);
    }
}

__global__ __launch_bounds__(kBlock) void k_philox(const uint32_t *__restrict__ ctr, uint32_t k0, uint32_t k1,
                                                   int64_t n, uint32_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    uint32_t w[4];
    philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1, w);
    for (int j = 0; j < 4; ++j) out[4 * i + j] = w[j];
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_normals(uint32_t k0, uint32_t k1, uint32_t inst, uint32_t path0,
                                                    int64_t npaths, uint32_t q0, int32_t nq, R *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= npaths * nq) return;
    const int64_t pp = i / nq;
    const uint32_t q = q0 + (uint32_t)(i % nq);
    R z[4];
    normals4<R>(q >> 2, path0 + (uint32_t)pp, inst, k0, k1, box_muller_scale<R>(1.0), z);
    out[i] = z[q & 3u];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int MODEL, typename R>
static hipError_t pass1_t(const DevProblem &pb, bool store, const double *theta, double *partial, void *ckpt,
                          int64_t nblocks, hipStream_t st)
{
    const size_t lds = sizeof(double) * kWavesPerBlock * pb.m;
    if (store)
        hipLaunchKernelGGL((k_pass1<MODEL, R, true>), dim3((unsigned)nblocks), dim3(kBlock), lds, st, pb, theta,
                           partial, (R *)ckpt);
    else
        hipLaunchKernelGGL((k_pass1<MODEL, R, false>), dim3((unsigned)nblocks), dim3(kBlock), lds, st, pb, theta,
                           partial, (R *)ckpt);
    return hipGetLastError();
}

hipError_t launch_pass1(const DevProblem &pb, int model, bool fp64, bool store, const double *theta,
                        double *partial, void *ckpt, int64_t nblocks, hipStream_t st)
{
    if (model == kBS)
        return fp64 ? pass1_t<kBS, double>(pb, store, theta, partial, ckpt, nblocks, st)
                    : pass1_t<kBS, float>(pb, store, theta, partial, ckpt, nblocks, st);
    return fp64 ? pass1_t<kHeston, double>(pb, store, theta, partial, ckpt, nblocks, st)
                : pass1_t<kHeston, float>(pb, store, theta, partial, ckpt, nblocks, st);
}

template <int MODEL, typename R, int K>
static hipError_t pass2_k(const DevProblem &pb, bool from_ckpt, const double *theta, const void *lamD,
                          double *partial, void *ckpt, int64_t nblocks, hipStream_t st)
{
    const size_t lds = pass2_lds_bytes<MODEL, R, K>();
    if (from_ckpt)
        hipLaunchKernelGGL((k_pass2<MODEL, R, true, K>), dim3((unsigned)nblocks), dim3(kBlock), lds, st, pb, theta,
                           (const R *)lamD, partial, (R *)ckpt);
    else
        hipLaunchKernelGGL((k_pass2<MODEL, R, false, K>), dim3((unsigned)nblocks), dim3(kBlock), lds, st, pb,
                           theta, (const R *)lamD, partial, (R *)ckpt);
    return hipGetLastError();
}

template <int MODEL, typename R>
static hipError_t pass2_t(const DevProblem &pb, bool from_ckpt, const double *theta, const void *lamD,
                          double *partial, void *ckpt, int64_t nblocks, hipStream_t st)
{
    switch (pb.K) {
    case 8: return pass2_k<MODEL, R, 8>(pb, from_ckpt, theta, lamD, partial, ckpt, nblocks, st);
    case 16: return pass2_k<MODEL, R, 16>(pb, from_ckpt, theta, lamD, partial, ckpt, nblocks, st);
    case 32: return pass2_k<MODEL, R, 32>(pb, from_ckpt, theta, lamD, partial, ckpt, nblocks, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pass2(const DevProblem &pb, int model, bool fp64, bool from_ckpt, const double *theta,
                        const void *lamD, double *partial, void *ckpt, int64_t nblocks, hipStream_t st)
{
    if (model == kBS)
        return fp64 ? pass2_t<kBS, double>(pb, from_ckpt, theta, lamD, partial, ckpt, nblocks, st)
                    : pass2_t<kBS, float>(pb, from_ckpt, theta, lamD, partial, ckpt, nblocks, st);
    return fp64 ? pass2_t<kHeston, double>(pb, from_ckpt, theta, lamD, partial, ckpt, nblocks, st)
                : pass2_t<kHeston, float>(pb, from_ckpt, theta, lamD, partial, ckpt, nblocks, st);
}

template <int MODEL, typename R>
static hipError_t tangent_t(const DevProblem &pb, const double *theta, double *partial, int64_t nblocks,
                            int ninst, hipStream_t st)
{
    const size_t lds = sizeof(double) * kWavesPerBlock * pb.m * (Traits<MODEL>::NP + 1);
    hipLaunchKernelGGL((k_tangent<MODEL, R>), dim3((unsigned)nblocks, (unsigned)ninst), dim3(kBlock), lds, st, pb,
                       theta, partial);
    return hipGetLastError();
}

hipError_t launch_tangent(const DevProblem &pb, int model, bool fp64, const double *theta, double *partial,
                          int64_t nblocks, int ninst, hipStream_t st)
{
    if (model == kBS)
        return fp64 ? tangent_t<kBS, double>(pb, theta, partial, nblocks, ninst, st)
                    : tangent_t<kBS, float>(pb, theta, partial, nblocks, ninst, st);
    return fp64 ? tangent_t<kHeston, double>(pb, theta, partial, nblocks, ninst, st)
                : tangent_t<kHeston, float>(pb, theta, partial, nblocks, ninst, st);
}

hipError_t launch_reduce_sorted(const double *partial, int64_t nblocks, int32_t count, const int32_t *id,
                                double scale, double *out, int32_t *status, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_sorted, dim3((unsigned)count), dim3(kBlock), 0, st, partial, nblocks, id, scale, out,
                       status);
    return hipGetLastError();
}

hipError_t launch_reduce_jac(const double *partial, int64_t nblocks, int32_t M, int32_t m, const int32_t *id,
                             double scale, double *Ey, double *J, int32_t *status, int ninst, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_jac, dim3((unsigned)(m * (M + 1)), (unsigned)ninst), dim3(kBlock), 0, st, partial,
                       nblocks, M, m, id, scale, Ey, J, status);
    return hipGetLastError();
}

hipError_t launch_residual(const DevProblem &pb, bool fp64, const double *Ey, const double *C, double *G,
                           void *lamD, const double *theta, hipStream_t st)
{
    if (fp64) hipLaunchKernelGGL(k_residual<double>, dim3(1), dim3(kBlock), 0, st, pb, Ey, C, G, (double *)lamD);
    else hipLaunchKernelGGL(k_residual<float>, dim3(1), dim3(kBlock), 0, st, pb, Ey, C, G, (float *)lamD);
    (void)theta;
    return hipGetLastError();
}

hipError_t launch_lambda(const DevProblem &pb, bool fp64, const double *lambda, void *lamD, const double *saved,
                         const double *theta, hipStream_t st)
{
    if (fp64)
        hipLaunchKernelGGL(k_lambda<double>, dim3(1), dim3(kBlock), 0, st, pb, lambda, (double *)lamD, saved, theta);
    else hipLaunchKernelGGL(k_lambda<float>, dim3(1), dim3(kBlock), 0, st, pb, lambda, (float *)lamD, saved, theta);
    return hipGetLastError();
}

hipError_t launch_check_theta(const DevProblem &pb, const double *theta, int model, hipStream_t st)
{
    hipLaunchKernelGGL(k_check_theta, dim3(1), dim3(64), 0, st, pb, theta, model);
    return hipGetLastError();
}

hipError_t launch_philox(const uint32_t *ctr, uint32_t k0, uint32_t k1, int64_t n, uint32_t *out, hipStream_t st)
{
    const int64_t nb = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_philox, dim3((unsigned)nb), dim3(kBlock), 0, st, ctr, k0, k1, n, out);
    return hipGetLastError();
}

hipError_t launch_normals(bool fp64, uint32_t k0, uint32_t k1, uint32_t inst, uint32_t path0, int64_t npaths,
                          uint32_t q0, int32_t nq, void *out, hipStream_t st)
{
    const int64_t total = npaths * nq;
    const int64_t nb = (total + kBlock - 1) / kBlock;
    if (fp64)
        hipLaunchKernelGGL(k_normals<double>, dim3((unsigned)nb), dim3(kBlock), 0, st, k0, k1, inst, path0, npaths,
                           q0, nq, (double *)out);
    else
        hipLaunchKernelGGL(k_normals<float>, dim3((unsigned)nb), dim3(kBlock), 0, st, k0, k1, inst, path0, npaths,
                           q0, nq, (float *)out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched instances: persistent workgroups take (instance, path block) work
// items from a queue (an atomic counter over a list ordered longest-first),
// run the same per-block bodies as the single-instance kernels, and exit
// when the queue is empty.  Per-instance finalizers sum the block partials
// in the same fixed order as k_reduce_sorted, so every instance's result is
// bitwise the one its own context would give.
// ---------------------------------------------------------------------------
__global__ void k_batch_reset(unsigned *counters)
{
    if (threadIdx.x < 2) counters[threadIdx.x] = 0u;
}

__device__ __forceinline__ int next_item(unsigned *counter)
{
    __shared__ int s_item;
    __syncthreads();   // the previous item's LDS traffic is over
    if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
    __syncthreads();
    // the same value in every lane; saying so keeps the item's tables and
    // problem constants in scalar registers
    return __builtin_amdgcn_readfirstlane(s_item);
}

template <int MODEL, typename R, bool STORE>
__global__ __launch_bounds__(kBlock) void k_batch_pass1(const BatchInst *__restrict__ insts,
                                                        const int2 *__restrict__ items, int n_items,
                                                        unsigned *counter, const double *__restrict__ theta_all)
{
    extern __shared__ double lds[];
    for (;;) {
        const int it = next_item(counter);
        if (it >= n_items) break;
        const int2 w = items[it];
        const DevProblem pb = insts[w.x].pb;
        pass1_block<MODEL, R, STORE, false>(pb, theta_all + (int64_t)w.x * Traits<MODEL>::NP, insts[w.x].part_y,
                                            (R *)insts[w.x].ckpt, w.y, lds);
    }
}

template <int MODEL, typename R, bool FROM_CKPT, int K>
__global__ __launch_bounds__(kBlock) void k_batch_pass2(const BatchInst *__restrict__ insts,
                                                        const int2 *__restrict__ items, int n_items,
                                                        unsigned *counter, const double *__restrict__ theta_all)
{
    extern __shared__ double lds[];
    for (;;) {
        const int it = next_item(counter);
        if (it >= n_items) break;
        const int2 w = items[it];
        const DevProblem pb = insts[w.x].pb;
        pass2_block<MODEL, R, FROM_CKPT, K>(pb, theta_all + (int64_t)w.x * Traits<MODEL>::NP,
                                            (const R *)insts[w.x].lamD, insts[w.x].part_g, (R *)insts[w.x].ckpt,
                                            w.y, lds);
    }
}

// grid (max m, n_inst): Ey[y_off + id[k]] = sum_b part_y[b][k] / P
__global__ __launch_bounds__(kBlock) void k_batch_reduce_y(const BatchInst *__restrict__ insts,
                                                           double *__restrict__ Ey)
{
    __shared__ double sh[kBlock];
    const BatchInst &I = insts[blockIdx.y];
    const int k = blockIdx.x;
    if (k >= I.pb.m) return;   // uniform per workgroup
    double acc = 0.0;
    const double *col = I.part_y + (int64_t)k * I.nblocks;
    for (int64_t b = threadIdx.x; b < I.nblocks; b += kBlock) acc += col[b];
    const double s = block_sum(acc, sh) * (1.0 / (double)I.pb.P);
    if (threadIdx.x == 0) {
        Ey[I.y_off + I.pb.id[k]] = s;
        if (!isfinite(s)) atomicOr(I.pb.status, 2);
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_batch_residual(const BatchInst *__restrict__ insts,
                                                           const double *__restrict__ Ey_all,
                                                           const double *__restrict__ C_all, double *__restrict__ G)
{
    __shared__ double sh[kBlock];
    const BatchInst &I = insts[blockIdx.x];
    const DevProblem &pb = I.pb;
    const double *Ey = Ey_all + I.y_off;
    const double *C = C_all + I.y_off;
    double acc = 0.0;
    for (int i = threadIdx.x; i < pb.m; i += kBlock) {
        const double r = Ey[i] - C[i];
        acc += 0.5 * r * r;
    }
    const double g = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        G[blockIdx.x] = g;
        if (!isfinite(g)) atomicOr(pb.status, 2);
    }
    const double invP = 1.0 / (double)pb.P;
    R *lamD = (R *)I.lamD;
    for (int k = threadIdx.x; k < pb.m; k += kBlock) {
        const int i = pb.id[k];
        lamD[k] = (R)((Ey[i] - C[i]) * pb.disc[k] * invP);
    }
}

// grid (NP, n_inst)
__global__ __launch_bounds__(kBlock) void k_batch_reduce_g(const BatchInst *__restrict__ insts, int NP,
                                                           double *__restrict__ grad)
{
    __shared__ double sh[kBlock];
    const BatchInst &I = insts[blockIdx.y];
    const int j = blockIdx.x;
    double acc = 0.0;
    const double *col = I.part_g + (int64_t)j * I.nblocks;
    for (int64_t b = threadIdx.x; b < I.nblocks; b += kBlock) acc += col[b];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        grad[(int64_t)blockIdx.y * NP + j] = s;
        if (!isfinite(s)) atomicOr(I.pb.status, 2);
    }
}

template <int MODEL, typename R, int K>
static hipError_t batch_step_t(const BatchLaunch &L, hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, L.counters);
    const size_t lds1 = sizeof(double) * kWavesPerBlock * L.max_m;
    const size_t lds2 = pass2_lds_bytes<MODEL, R, K>();
    hipLaunchKernelGGL((k_batch_pass1<MODEL, R, true>), dim3(L.grid), dim3(kBlock), lds1, st, L.insts, L.items,
                       L.n_items, L.counters, L.theta);
    hipLaunchKernelGGL(k_batch_reduce_y, dim3(L.max_m, L.n_inst), dim3(kBlock), 0, st, L.insts, L.Ey);
    hipLaunchKernelGGL(k_batch_residual<R>, dim3(L.n_inst), dim3(kBlock), 0, st, L.insts, L.Ey, L.C, L.G);
    hipLaunchKernelGGL((k_batch_pass2<MODEL, R, true, K>), dim3(L.grid), dim3(kBlock), lds2, st, L.insts, L.items,
                       L.n_items, L.counters + 1, L.theta);
    hipLaunchKernelGGL(k_batch_reduce_g, dim3(Traits<MODEL>::NP, L.n_inst), dim3(kBlock), 0, st, L.insts,
                       Traits<MODEL>::NP, L.grad);
    return hipGetLastError();
}

template <int MODEL, typename R>
static hipError_t batch_step_m(const BatchLaunch &L, hipStream_t st)
{
    switch (L.K) {
    case 8: return batch_step_t<MODEL, R, 8>(L, st);
    case 16: return batch_step_t<MODEL, R, 16>(L, st);
    case 32: return batch_step_t<MODEL, R, 32>(L, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_step(const BatchLaunch &L, hipStream_t st)
{
    if (L.model == kBS) return L.fp64 ? batch_step_m<kBS, double>(L, st) : batch_step_m<kBS, float>(L, st);
    return L.fp64 ? batch_step_m<kHeston, double>(L, st) : batch_step_m<kHeston, float>(L, st);
}

int batch_blocks_per_cu(int model, bool fp64, int K, int max_m)
{
    int n1 = 0, n2 = 0;
    const size_t lds1 = sizeof(double) * kWavesPerBlock * max_m;
#define MCAAD_OCC(M_, R_, K_)                                                                                  \
    do {                                                                                                       \
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n1, k_batch_pass1<M_, R_, true>, kBlock, lds1);    \
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n2, k_batch_pass2<M_, R_, true, K_>, kBlock,        \
                                                           pass2_lds_bytes<M_, R_, K_>());                   \
    } while (0)
    if (model == kBS) {
        if (fp64) { if (K == 8) MCAAD_OCC(kBS, double, 8); else if (K == 16) MCAAD_OCC(kBS, double, 16); else MCAAD_OCC(kBS, double, 32); }
        else { if (K == 8) MCAAD_OCC(kBS, float, 8); else if (K == 16) MCAAD_OCC(kBS, float, 16); else MCAAD_OCC(kBS, float, 32); }
    } else {
        if (fp64) { if (K == 8) MCAAD_OCC(kHeston, double, 8); else if (K == 16) MCAAD_OCC(kHeston, double, 16); else MCAAD_OCC(kHeston, double, 32); }
        else { if (K == 8) MCAAD_OCC(kHeston, float, 8); else if (K == 16) MCAAD_OCC(kHeston, float, 16); else MCAAD_OCC(kHeston, float, 32); }
    }
#undef MCAAD_OCC
    const int n = n1 < n2 ? n1 : n2;
    return n > 0 ? n : 1;
}

}  // namespace mcaad
