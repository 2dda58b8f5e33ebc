// Heston stochastic local volatility on gfx950 (the paper's test model):
// dS/S = r dt + L(t, S) sqrt(v) dW1 with Heston's variance process, theta =
// (kappa, theta_bar, xi, rho, v0, L[a][k]).  L is piecewise constant in time
// (step n uses row step_row[n]: the number of time nodes <= n h, capped at the
// last row, tabulated on the host) and linear across uniformly spaced spot
// nodes K0 + k dK, flat outside.
//
// Sweep variables as for Heston (models.hpp): scaled normals z', the
// drift-free log-price x~, w' = rho z1' + rho' z2';
//   x~ <- L s z1' + (x~ - (h/2) L^2 v+),  v as Heston,  L = L(t_n, S_n).
// The leverage grid is copied into LDS once per workgroup.
//
// Reverse sweep, per step (a = adjoint of x~, b = adjoint of v after it):
//   Lbar = a (s z1' - h L v+), spread over the step's two spot nodes with
//   weights 1 - be, be into per-lane LDS slices of the current time row (in
//   the path precision),
//   which a fixed tree sums into FP64 node sums when the row changes;
//   a += Lbar dL/dS S; the Heston part as in the Heston reverse sweep with
//   sbar = b xi w' + a L z1' and v+bar = sbar/(2s) - (h/2) L^2 a - kappa h b.
#include <hip/hip_runtime.h>

#include "mc_device.hpp"
#include "mc_kernels.hpp"
#include "models.hpp"

namespace mcaad {
namespace {

constexpr int kHes = 5;   // Heston parameters ahead of the leverage nodes

// LDS carve-up.  pass 1: [waves][m] payoff sums, leverage grid.
// pass 2: [nT*nK] FP64 node sums, [waves][5] FP64 Heston sums, leverage grid,
// [K][kBlock] payoff adjoints of the segment's dates, [nK][kBlock] node slices
// of the current row in the path precision (one column per lane).
template <typename R>
struct SlvLds {
    double *sums;
    double *hes;
    R *lev;
    R *inj;
    R *slices;
};

__host__ __device__ inline size_t align16(size_t o) { return (o + 15) & ~(size_t)15; }

template <typename R>
__device__ SlvLds<R> carve(const DevProblem &pb, unsigned char *base, int pass)
{
    SlvLds<R> L{};
    size_t o = 0;
    const int nn = pb.nT * pb.nK;
    L.sums = (double *)(base + o);
    o += sizeof(double) * (pass == 1 ? (size_t)kWavesPerBlock * pb.m : (size_t)nn);
    L.hes = (double *)(base + o);
    if (pass == 2) o += sizeof(double) * kWavesPerBlock * kHes;
    o = align16(o);
    L.lev = (R *)(base + o);
    o = align16(o + sizeof(R) * nn);
    L.inj = (R *)(base + o);
    if (pass == 2) o = align16(o + sizeof(R) * (size_t)pb.K * kBlock);
    L.slices = (R *)(base + o);
    return L;
}

template <typename R>
__device__ void load_grid(const DevProblem &pb, const double *theta, R *lev)
{
    for (int i = threadIdx.x; i < pb.nT * pb.nK; i += kBlock) lev[i] = (R)theta[kHes + i];
}

// One step of the stochastic local volatility sweep on (x~, v); returns what
// the reverse sweep needs.  Every sweep steps through this function.
template <typename R>
struct SlvStep {
    R vp, s, w, S;
};

template <typename R>
struct SpotCell {
    int b;
    R be, r0, r1, L;
    bool inside;
};

template <typename R>
__device__ __forceinline__ SpotCell<R> spot_cell(const R *row, R S, R K0, R invdK, R Klast, int nK)
{
    SpotCell<R> q;
    const R u = (S - K0) * invdK;
    int b = (int)floor(u);
    b = b < 0 ? 0 : (b > nK - 2 ? nK - 2 : b);
    R be = u - (R)b;
    be = be < (R)0 ? (R)0 : (be > (R)1 ? (R)1 : be);
    q.b = b;
    q.be = be;
    q.r0 = row[b];
    q.r1 = row[b + 1];
    q.L = q.r0 + be * (q.r1 - q.r0);
    q.inside = S >= K0 && S <= Klast;
    return q;
}

template <typename R>
__device__ __forceinline__ SlvStep<R> slv_step(const Consts<R> &c, R &x, R &v, R z0, R z1, const R *row, int n,
                                               R K0, R invdK, R Klast, int nK)
{
    SlvStep<R> q;
    q.vp = vplus(v);
    q.s = sqrt_r(q.vp);
    q.w = c.rhop * z1 + c.rho * z0;
    q.S = spot(c, x, n);
    const R L = spot_cell(row, q.S, K0, invdK, Klast, nK).L;
    x = (L * q.s) * z0 + (x - c.hh * (L * L) * q.vp);
    v = q.s * (c.xi * q.w) + (v + (c.khth - c.kh * q.vp));
    return q;
}

template <typename R, bool STORE>
__global__ __launch_bounds__(kBlock) void k_slv_pass1(DevProblem pb, const double *__restrict__ theta,
                                                      double *__restrict__ partial, R *__restrict__ ckpt)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    SlvLds<R> L = carve<R>(pb, lds_raw, 1);
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    load_grid<R>(pb, theta, L.lev);
    if constexpr (STORE) save_theta(pb, theta, blockIdx.x);
    __syncthreads();

    Consts<R> c;
    load_consts<kHeston, R>(pb, theta, c);
    const R K0 = (R)pb.K0, invdK = (R)(1.0 / pb.dK), Klast = (R)(pb.K0 + (pb.nK - 1) * pb.dK);
    const int kmask = pb.K - 1;
    const int kshift = __builtin_ctz(pb.K);
    const int ncalls = (pb.N * 2 + 3) / 4;
    // the workgroup's paths: ppl runs of kBlock consecutive paths, one after another
    for (int sp = 0; sp < pb.ppl; ++sp) {
        const int64_t p = ((int64_t)blockIdx.x * pb.ppl + sp) * kBlock + tid;
        const bool active = p < pb.P;
        const uint32_t path = (uint32_t)p;
        R x = (R)0;
        R v = c.v0;
        int d = 0;
        int next = pb.ndates > 0 ? ldc(pb.date_step, 0) : -1;
        for (int call = 0; call < ncalls; ++call) {
            R z[4];
            normals4<R>((uint32_t)call, path, pb.inst, pb.k0, pb.k1, c.bm, z);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int n = call * 2 + j;
                if (n < pb.N) {
                    if constexpr (STORE) {
                        if ((n & kmask) == 0 && active) {
                            const int64_t base = (int64_t)((n >> kshift) * 2) * pb.P + p;
                            ckpt[base] = x;
                            ckpt[base + pb.P] = v;
                        }
                    }
                    const R *row = L.lev + ldc(pb.step_row, n) * pb.nK;
                    (void)slv_step(c, x, v, z[2 * j], z[2 * j + 1], row, n, K0, invdK, Klast, pb.nK);
                    if (n + 1 == next) {
                        const double S = (double)spot(c, x, n + 1);
                        payoff_sums(pb.strike, pb.disc, S, active, lane, ldc(pb.date_begin, d),
                                    ldc(pb.date_begin, d + 1), L.sums + wave * pb.m, sp > 0);
                        ++d;
                        next = d < pb.ndates ? ldc(pb.date_step, d) : -1;
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int k = tid; k < pb.m; k += kBlock) {
        double s = L.sums[k];
#pragma unroll
        for (int w = 1; w < kWavesPerBlock; ++w) s += L.sums[w * pb.m + k];
        partial[(int64_t)k * gridDim.x + blockIdx.x] = s;
    }
}

// Sum the lane slices of time row `a` over the workgroup into the FP64 node
// sums, then clear them.  Called by every thread (uniform).
template <typename R>
__device__ void flush_row(const DevProblem &pb, SlvLds<R> &L, int a)
{
    flush_slices(L.slices, pb.nK, L.sums + a * pb.nK);
}

template <typename R, bool FROM_CKPT, int K>
__global__ __launch_bounds__(kBlock) void k_slv_pass2(DevProblem pb, const double *__restrict__ theta,
                                                      const R *__restrict__ lamD, double *__restrict__ partial,
                                                      R *__restrict__ ckpt)
{
    static_assert(K % 2 == 0, "segments start on a Philox call");
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    SlvLds<R> L = carve<R>(pb, lds_raw, 2);
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    load_grid<R>(pb, theta, L.lev);
    if constexpr (!FROM_CKPT) save_theta(pb, theta, blockIdx.x);
    for (int i = tid; i < pb.nT * pb.nK; i += kBlock) L.sums[i] = 0.0;
    for (int i = tid; i < pb.nK * kBlock; i += kBlock) L.slices[i] = (R)0;
    __syncthreads();

    Consts<R> c;
    load_consts<kHeston, R>(pb, theta, c);
    const R K0 = (R)pb.K0, invdK = (R)(1.0 / pb.dK), Klast = (R)(pb.K0 + (pb.nK - 1) * pb.dK);
    const int nK = pb.nK;
    const R *strike_r;
    if constexpr (sizeof(R) == 4) strike_r = pb.strike_f;
    else strike_r = pb.strike;

    double g[kHes];
#pragma unroll
    for (int j = 0; j < kHes; ++j) g[j] = 0.0;
    R *my = L.slices + tid;   // this lane's column of the slices
    int cur_a = ldc(pb.step_row, pb.N - 1);
    // the workgroup's paths: ppl runs of kBlock consecutive paths, one after another
    for (int sp = 0; sp < pb.ppl; ++sp) {
        const int64_t p = ((int64_t)blockIdx.x * pb.ppl + sp) * kBlock + tid;
        const bool active = p < pb.P;
        const uint32_t path = (uint32_t)p;
        const double on = active ? 1.0 : 0.0;
        if constexpr (!FROM_CKPT) {
            R x = (R)0;
            R v = c.v0;
            const int ncalls = (pb.N * 2 + 3) / 4;
            for (int call = 0; call < ncalls; ++call) {
                R z[4];
                normals4<R>((uint32_t)call, path, pb.inst, pb.k0, pb.k1, c.bm, z);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int n = call * 2 + j;
                    if (n < pb.N) {
                        if ((n % K) == 0 && active) {
                            const int64_t base = (int64_t)((n / K) * 2) * pb.P + p;
                            ckpt[base] = x;
                            ckpt[base + pb.P] = v;
                        }
                        const R *row = L.lev + ldc(pb.step_row, n) * nK;
                        (void)slv_step(c, x, v, z[2 * j], z[2 * j + 1], row, n, K0, invdK, Klast, nK);
                    }
                }
            }
        }

        R xb = (R)0, vb = (R)0;
        int dhi = pb.ndates;
        for (int seg = pb.nseg - 1; seg >= 0; --seg) {
            const int n0 = seg * K;
            // inactive lanes (past the last path) run a harmless path from
            // (0, v0) with zero adjoints; they read no checkpoint, since in the
            // re-run mode another workgroup may still be writing the one they
            // would share
            R x = (R)0, v = c.v0;
            if (active) {
                const int64_t base = (int64_t)(seg * 2) * pb.P + p;
                x = ckpt[base];
                v = ckpt[base + pb.P];
            }
            int dlo = dhi;
            while (dlo > 0 && ldc(pb.date_step, dlo - 1) > n0) --dlo;
            int d = dlo;
            int next = d < dhi ? ldc(pb.date_step, d) : -1;

            // recompute the segment, keeping (S, z1', w', s = sqrt(v+)) of every
            // step; v+ is taken back as s^2
            R s_S[K], s_z1[K], s_w[K], s_s[K];
            R z[4];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int n = n0 + j;
                s_S[j] = (R)0;
                s_z1[j] = (R)0;
                s_w[j] = (R)0;
                s_s[j] = (R)0;
                if (n < pb.N) {
                    if (j % 2 == 0) normals4<R>((uint32_t)(n / 2), path, pb.inst, pb.k0, pb.k1, c.bm, z);
                    const R *zs = z + (j % 2) * 2;
                    const R *row = L.lev + ldc(pb.step_row, n) * nK;
                    const SlvStep<R> q = slv_step(c, x, v, zs[0], zs[1], row, n, K0, invdK, Klast, nK);
                    s_S[j] = q.S;
                    s_z1[j] = zs[0];
                    s_w[j] = q.w;
                    s_s[j] = q.s;
                    if (n + 1 == next) {
                        // payoff adjoints of this date: sum_i lambda_i D_i / P 1{S > K_i} S
                        const R S = spot(c, x, n + 1);
                        R inj = (R)0;
                        for (int k = ldc(pb.date_begin, d); k < ldc(pb.date_begin, d + 1); ++k)
                            inj += S > ldc(strike_r, k) ? ldc(lamD, k) * S : (R)0;
                        L.inj[j * kBlock + tid] = active ? inj : (R)0;
                        ++d;
                        next = d < dhi ? ldc(pb.date_step, d) : -1;
                    }
                }
            }
            dhi = dlo;

            // reverse sweep over the segment; its dates are dlo .. d-1, met last first
            int dr = d - 1;
            int rnext = dr >= dlo ? ldc(pb.date_step, dr) : -1;
            R sb = (R)0, tk = (R)0, t2 = (R)0, t3 = (R)0;
#pragma unroll
            for (int j = K - 1; j >= 0; --j) {
                const int n = n0 + j;
                if (n < pb.N) {
                    if (n + 1 == rnext) {
                        xb += L.inj[j * kBlock + tid];
                        --dr;
                        rnext = dr >= dlo ? ldc(pb.date_step, dr) : -1;
                    }
                    const int a_n = ldc(pb.step_row, n);
                    if (a_n != cur_a) {
                        flush_row<R>(pb, L, cur_a);
                        cur_a = a_n;
                    }
                    const R S = s_S[j], sv = s_s[j], z1 = s_z1[j], w = s_w[j];
                    const R vp = sv * sv;
                    const SpotCell<R> q = spot_cell(L.lev + a_n * nK, S, K0, invdK, Klast, nK);
                    const R b = vb;
                    const R Lbar = xb * (sv * z1 - c.h * q.L * vp);
                    const R sbar = (b * c.xi) * w + (xb * q.L) * z1;
                    const R vpbar = sbar * ((R)0.5 * rcp_r(sv)) - c.hh * (q.L * q.L) * xb - c.kh * b;
                    sb += b;
                    tk += b * (c.thbh - c.h * vp);
                    const R t = b * sv;
                    t2 += t * w;
                    t3 += t * (z1 - c.rho * w);
                    const R w1 = Lbar * q.be;
                    my[q.b * kBlock] += Lbar - w1;
                    my[(q.b + 1) * kBlock] += w1;
                    xb = xb + Lbar * (q.inside ? (q.r1 - q.r0) * invdK : (R)0) * S;
                    vb = sv > (R)0 ? b + vpbar : b;
                }
            }
            g[0] += on * (double)tk;
            g[1] += on * (c.g_kh * (double)sb);
            g[2] += on * (double)t2;
            g[3] += on * (c.g_rho * (double)t3);
        }
        g[4] += on * (double)vb;   // v_0 is theta[4]
    }
    flush_row<R>(pb, L, cur_a);

    double a8[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a8[j] = j < kHes ? g[j] : 0.0;
    const double t = wave_sum8(a8);
    if ((lane & 7) == 0 && (lane >> 3) < kHes) L.hes[wave * kHes + (lane >> 3)] = t;
    __syncthreads();
    if (tid < kHes) {
        double s = L.hes[tid];
#pragma unroll
        for (int w = 1; w < kWavesPerBlock; ++w) s += L.hes[w * kHes + tid];
        partial[(int64_t)tid * gridDim.x + blockIdx.x] = s;
    }
    for (int i = tid; i < pb.nT * nK; i += kBlock) partial[(int64_t)(kHes + i) * gridDim.x + blockIdx.x] = L.sums[i];
}

template <typename R>
hipError_t pass1_t(const DevProblem &pb, bool store, const double *theta, double *partial, void *ckpt, int64_t nb,
                   hipStream_t st)
{
    const size_t lds = slv_lds_bytes(pb, sizeof(R) == 8, 1);
    if (store)
        hipLaunchKernelGGL((k_slv_pass1<R, true>), dim3((unsigned)nb), dim3(kBlock), lds, st, pb, theta, partial,
                           (R *)ckpt);
    else
        hipLaunchKernelGGL((k_slv_pass1<R, false>), dim3((unsigned)nb), dim3(kBlock), lds, st, pb, theta, partial,
                           (R *)ckpt);
    return hipGetLastError();
}

template <typename R, int K>
hipError_t pass2_k(const DevProblem &pb, bool from_ckpt, const double *theta, const void *lamD, double *partial,
                   void *ckpt, int64_t nb, hipStream_t st)
{
    const size_t lds = slv_lds_bytes(pb, sizeof(R) == 8, 2);
    if (from_ckpt)
        hipLaunchKernelGGL((k_slv_pass2<R, true, K>), dim3((unsigned)nb), dim3(kBlock), lds, st, pb, theta,
                           (const R *)lamD, partial, (R *)ckpt);
    else
        hipLaunchKernelGGL((k_slv_pass2<R, false, K>), dim3((unsigned)nb), dim3(kBlock), lds, st, pb, theta,
                           (const R *)lamD, partial, (R *)ckpt);
    return hipGetLastError();
}

template <typename R>
hipError_t pass2_t(const DevProblem &pb, bool from_ckpt, const double *theta, const void *lamD, double *partial,
                   void *ckpt, int64_t nb, hipStream_t st)
{
    switch (pb.K) {
    case 8: return pass2_k<R, 8>(pb, from_ckpt, theta, lamD, partial, ckpt, nb, st);
    case 16: return pass2_k<R, 16>(pb, from_ckpt, theta, lamD, partial, ckpt, nb, st);
    case 32: return pass2_k<R, 32>(pb, from_ckpt, theta, lamD, partial, ckpt, nb, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t slv_lds_bytes(const DevProblem &pb, bool fp64, int pass)
{
    const size_t real = fp64 ? 8 : 4;
    const size_t nn = (size_t)pb.nT * pb.nK;
    size_t o = sizeof(double) * (pass == 1 ? (size_t)kWavesPerBlock * pb.m : nn);
    if (pass == 2) o += sizeof(double) * kWavesPerBlock * kHes;
    o = align16(o);
    o = align16(o + real * nn);
    if (pass == 2) {
        o = align16(o + real * (size_t)pb.K * kBlock);
        o += real * (size_t)pb.nK * kBlock;
    }
    return o;
}

hipError_t launch_slv_pass1(const DevProblem &pb, bool fp64, bool store, const double *theta, double *partial,
                            void *ckpt, int64_t nb, hipStream_t st)
{
    return fp64 ? pass1_t<double>(pb, store, theta, partial, ckpt, nb, st)
                : pass1_t<float>(pb, store, theta, partial, ckpt, nb, st);
}

hipError_t launch_slv_pass2(const DevProblem &pb, bool fp64, bool from_ckpt, const double *theta, const void *lamD,
                            double *partial, void *ckpt, int64_t nb, hipStream_t st)
{
    return fp64 ? pass2_t<double>(pb, from_ckpt, theta, lamD, partial, ckpt, nb, st)
                : pass2_t<float>(pb, from_ckpt, theta, lamD, partial, ckpt, nb, st);
}

}  // namespace mcaad
