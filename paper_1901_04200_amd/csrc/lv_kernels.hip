// Local-volatility model on gfx950: sigma(t, S) bilinear on a grid of node
// values theta[a*nK + k] at times t_nodes[a] and spots K0 + k dK, flat
// outside the grid; log-Euler x' = x + (r - sigma^2/2) h + sigma sqrt(h) z.
//
// The time weights of step n are the same for every path, so each
// workgroup interpolates the grid in time into LDS, for the K steps of the
// current checkpoint segment at a time (a window of K rows keeps the LDS
// footprint small):
// row_n[k] = (1 - al_n) theta[a_n][k] + al_n theta[a_n + 1][k].  A path-step
// then needs its spot cell b, the weight be and two LDS reads.
//
// Reverse sweep: sigmabar_n = xbar (-sigma h + sqrt(h) z); the node adjoints
// get sigmabar (1-al)(1-be), (1-al) be, al (1-be), al be at (a, b), (a, b+1),
// (a+1, b), (a+1, b+1).  b differs per lane, a and al do not: each lane
// accumulates sum (1-al) w_k and sum al w_k over the steps of one time cell in
// its own LDS slice (in the path precision: FP32, or FP64 in the FP64 mode),
// and when the time cell changes the workgroup sums the slices over lanes in a
// fixed tree into FP64 node sums.
#include <hip/hip_runtime.h>

#include "mc_device.hpp"
#include "mc_kernels.hpp"

namespace mcaad {
namespace {

template <typename R>
__device__ __forceinline__ R exp_t(R x)
{
    if constexpr (sizeof(R) == 4) return __expf(x);
    else return exp(x);
}

// LDS carve-up shared by both passes: [dbl area][rows: R K*nK][slices]
template <typename R>
struct LvLds {
    double *dbl;   // pass 1: [waves][m] payoff sums; pass 2: [nT*nK] node sums
    R *rows;
    R *slices;   // pass 2: [2*nK][kBlock], path precision
};

template <typename R>
__device__ LvLds<R> carve(const DevProblem &pb, unsigned char *base, int ndbl)
{
    LvLds<R> L;
    size_t o = 0;
    L.dbl = (double *)(base + o);
    o += sizeof(double) * ndbl;
    L.rows = (R *)(base + o);
    o += sizeof(R) * pb.K * pb.nK;
    o = (o + 15) & ~(size_t)15;
    L.slices = (R *)(base + o);
    return L;
}

// time weight al_n of step n in the path precision (host table, uniform)
template <typename R>
__device__ __forceinline__ R step_al(const DevProblem &pb, int n)
{
    if constexpr (sizeof(R) == 4) return ldc(pb.step_al_f, n);
    else return ldc(pb.step_al, n);
}

// the time-interpolated rows of steps n0 .. n0 + K - 1 (those < N) into the
// window, row n at L.rows + (n - n0) * nK; every thread calls it (uniform)
template <typename R>
__device__ void build_window(const DevProblem &pb, const double *theta, LvLds<R> &L, int n0)
{
    const int tid = threadIdx.x;
    __syncthreads();   // the previous window is no longer read
    const int total = pb.K * pb.nK;
    for (int i = tid; i < total; i += kBlock) {
        const int n = n0 + i / pb.nK, k = i % pb.nK;
        if (n < pb.N) {
            const int a = pb.step_row[n];
            const double al = (double)step_al<R>(pb, n);
            L.rows[i] = (R)((1.0 - al) * theta[a * pb.nK + k] + al * theta[(a + 1) * pb.nK + k]);
        }
    }
    __syncthreads();
}

template <typename R>
struct Cell {
    int b;
    R be, r0, r1, sig;
    bool inside;
};

template <typename R>
__device__ __forceinline__ Cell<R> locate(const DevProblem &pb, const R *row, R S, R K0, R invdK, R Klast)
{
    Cell<R> c;
    const R u = (S - K0) * invdK;
    int b = (int)floor(u);
    b = b < 0 ? 0 : (b > pb.nK - 2 ? pb.nK - 2 : b);
    R be = u - (R)b;
    be = be < (R)0 ? (R)0 : (be > (R)1 ? (R)1 : be);
    c.b = b;
    c.be = be;
    c.r0 = row[b];
    c.r1 = row[b + 1];
    c.sig = c.r0 + be * (c.r1 - c.r0);
    c.inside = S >= K0 && S <= Klast;
    return c;
}

// Pass 1.  A lane runs PPL paths side by side (independent dependency
// chains, which hide each other's latency): path i of the lane in workgroup
// blk is (blk * PPL + i) * kBlock + tid.
template <typename R, bool STORE, int PPL>
__global__ __launch_bounds__(kBlock) void k_lv_pass1(DevProblem pb, const double *__restrict__ theta,
                                                     double *__restrict__ partial, R *__restrict__ ckpt)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    LvLds<R> L = carve<R>(pb, lds_raw, kWavesPerBlock * pb.m);
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    int64_t p[PPL];
    bool active[PPL];
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
        p[i] = ((int64_t)blockIdx.x * PPL + i) * kBlock + tid;
        active[i] = p[i] < pb.P;
    }
    if constexpr (STORE) save_theta(pb, theta, blockIdx.x);

    const R s0 = (R)pb.s0, rh = (R)(pb.rate * pb.h), hh = (R)(0.5 * pb.h), sq = (R)pb.sq;
    const R K0 = (R)pb.K0, invdK = (R)(1.0 / pb.dK), Klast = (R)(pb.K0 + (pb.nK - 1) * pb.dK);
    R x[PPL];
#pragma unroll
    for (int i = 0; i < PPL; ++i) x[i] = (R)0;
    int d = 0;
    int next = pb.ndates > 0 ? pb.date_step[0] : -1;
    const int cps = max(pb.K / 4, 1);   // Philox calls per segment (K is a multiple of 4)
    const int ncalls = (pb.N + 3) / 4;
    int n0 = 0;                         // first step of the current segment and window
    for (int call = 0; call < ncalls; ++call) {
        if (call % cps == 0) {
            n0 = call * 4;
            build_window<R>(pb, theta, L, n0);
            if constexpr (STORE) {
#pragma unroll
                for (int i = 0; i < PPL; ++i)
                    if (active[i]) ckpt[(int64_t)(call / cps) * pb.P + p[i]] = x[i];
            }
        }
        R z[PPL][4];
#pragma unroll
        for (int i = 0; i < PPL; ++i)
            normals4<R>((uint32_t)call, (uint32_t)p[i], pb.inst, pb.k0, pb.k1, box_muller_scale<R>(1.0), z[i]);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = call * 4 + j;
            if (n < pb.N) {
#pragma unroll
                for (int i = 0; i < PPL; ++i) {
                    const R S = s0 * exp_t(x[i]);
                    const Cell<R> c = locate<R>(pb, L.rows + (n - n0) * pb.nK, S, K0, invdK, Klast);
                    x[i] = x[i] + (rh - hh * c.sig * c.sig) + (sq * c.sig) * z[i][j];
                }
                if (n + 1 == next) {
#pragma unroll
                    for (int i = 0; i < PPL; ++i) {
                        const double Sd = (double)(s0 * exp_t(x[i]));
                        payoff_sums(pb.strike, pb.disc, Sd, active[i], lane, pb.date_begin[d], pb.date_begin[d + 1],
                                    L.dbl + wave * pb.m, i > 0);
                    }
                    ++d;
                    next = d < pb.ndates ? pb.date_step[d] : -1;
                }
            }
        }
    }
    __syncthreads();
    for (int k = tid; k < pb.m; k += kBlock) {
        double s = L.dbl[k];
#pragma unroll
        for (int w = 1; w < kWavesPerBlock; ++w) s += L.dbl[w * pb.m + k];
        partial[(int64_t)k * gridDim.x + blockIdx.x] = s;
    }
}

// Sum the lane slices of time cell `a` (rows: cell a's nodes, then cell
// a + 1's) over the workgroup into the FP64 node sums, then clear them.
// Called by every thread (uniform).
template <typename R>
__device__ void flush_cell(const DevProblem &pb, LvLds<R> &L, int a)
{
    flush_slices(L.slices, 2 * pb.nK, L.dbl + a * pb.nK);
}

// Pass 2.  PPL paths per lane side by side, as in pass 1; their node
// adjoints go to the lane's one column of slices, path 0 first at every step.
template <typename R, bool FROM_CKPT, int K, int PPL>
__global__ __launch_bounds__(kBlock) void k_lv_pass2(DevProblem pb, const double *__restrict__ theta,
                                                     const R *__restrict__ lamD, double *__restrict__ partial,
                                                     R *__restrict__ ckpt)
{
    static_assert(K % 4 == 0, "segments start on a Philox call");
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    LvLds<R> L = carve<R>(pb, lds_raw, pb.nT * pb.nK);
    const int tid = threadIdx.x;
    int64_t p[PPL];
    bool active[PPL];
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
        p[i] = ((int64_t)blockIdx.x * PPL + i) * kBlock + tid;
        active[i] = p[i] < pb.P;
    }
    if constexpr (!FROM_CKPT) save_theta(pb, theta, blockIdx.x);
    for (int i = tid; i < pb.nT * pb.nK; i += kBlock) L.dbl[i] = 0.0;
    for (int i = tid; i < 2 * pb.nK * kBlock; i += kBlock) L.slices[i] = (R)0;
    __syncthreads();

    const R s0 = (R)pb.s0, rh = (R)(pb.rate * pb.h), hh = (R)(0.5 * pb.h), sq = (R)pb.sq, h = (R)pb.h;
    const R K0 = (R)pb.K0, invdK = (R)(1.0 / pb.dK), Klast = (R)(pb.K0 + (pb.nK - 1) * pb.dK);
    const R *strike_r;
    if constexpr (sizeof(R) == 4) strike_r = pb.strike_f;
    else strike_r = pb.strike;

    if constexpr (!FROM_CKPT) {
        // the forward re-run of the paper's step 2, storing every segment's start
        R x[PPL];
#pragma unroll
        for (int i = 0; i < PPL; ++i) x[i] = (R)0;
        const int ncalls = (pb.N + 3) / 4;
        int n0 = 0;
        for (int call = 0; call < ncalls; ++call) {
            if ((call * 4) % K == 0) {
                n0 = call * 4;
                build_window<R>(pb, theta, L, n0);
#pragma unroll
                for (int i = 0; i < PPL; ++i)
                    if (active[i]) ckpt[(int64_t)(n0 / K) * pb.P + p[i]] = x[i];
            }
            R z[PPL][4];
#pragma unroll
            for (int i = 0; i < PPL; ++i)
                normals4<R>((uint32_t)call, (uint32_t)p[i], pb.inst, pb.k0, pb.k1, box_muller_scale<R>(1.0), z[i]);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int n = call * 4 + j;
                if (n < pb.N) {
#pragma unroll
                    for (int i = 0; i < PPL; ++i) {
                        const R S = s0 * exp_t(x[i]);
                        const Cell<R> c = locate<R>(pb, L.rows + (n - n0) * pb.nK, S, K0, invdK, Klast);
                        x[i] = x[i] + (rh - hh * c.sig * c.sig) + (sq * c.sig) * z[i][j];
                    }
                }
            }
        }
    }

    R xb[PPL];
#pragma unroll
    for (int i = 0; i < PPL; ++i) xb[i] = (R)0;
    int cur_a = ldc(pb.step_row, pb.N - 1);
    int dhi = pb.ndates;
    R *my0 = L.slices + tid;   // this lane's column of the slices
    const int rowB = pb.nK * kBlock;
    for (int seg = pb.nseg - 1; seg >= 0; --seg) {
        const int n0 = seg * K;
        build_window<R>(pb, theta, L, n0);
        R x[PPL];
#pragma unroll
        for (int i = 0; i < PPL; ++i)   // inactive lanes run a harmless path
            x[i] = active[i] ? ckpt[(int64_t)seg * pb.P + (active[i] ? p[i] : 0)] : (R)0;
        int dlo = dhi;
        while (dlo > 0 && pb.date_step[dlo - 1] > n0) --dlo;
        int d = dlo;
        int next = d < dhi ? pb.date_step[d] : -1;
        // recompute the segment, keeping per step what the reverse sweep needs,
        // so that it reads no LDS but the slices it adds to:
        //   s_c = d x'/d sigma = -sigma h + sqrt(h) z,  s_d = d sigma/dS * S,
        //   the spot cell b and its weight be, the payoff adjoint injected
        R s_c[PPL][K], s_d[PPL][K], s_be[PPL][K], s_inj[PPL][K];
        int s_b[PPL][K];
        R z[PPL][4];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int n = n0 + j;
#pragma unroll
            for (int i = 0; i < PPL; ++i) s_inj[i][j] = (R)0;
            if (n < pb.N) {
                if (j % 4 == 0) {
#pragma unroll
                    for (int i = 0; i < PPL; ++i)
                        normals4<R>((uint32_t)(n / 4), (uint32_t)p[i], pb.inst, pb.k0, pb.k1,
                                    box_muller_scale<R>(1.0), z[i]);
                }
#pragma unroll
                for (int i = 0; i < PPL; ++i) {
                    const R S = s0 * exp_t(x[i]);
                    const Cell<R> c = locate<R>(pb, L.rows + j * pb.nK, S, K0, invdK, Klast);
                    s_c[i][j] = -c.sig * h + sq * z[i][j % 4];
                    s_d[i][j] = (c.inside ? (c.r1 - c.r0) * invdK : (R)0) * S;
                    s_b[i][j] = c.b;
                    s_be[i][j] = c.be;
                    x[i] = x[i] + (rh - hh * c.sig * c.sig) + (sq * c.sig) * z[i][j % 4];
                }
                if (n + 1 == next) {
#pragma unroll
                    for (int i = 0; i < PPL; ++i) {
                        const R Sn = s0 * exp_t(x[i]);
                        R inj = (R)0;
                        for (int k = pb.date_begin[d]; k < pb.date_begin[d + 1]; ++k)
                            inj += Sn > strike_r[k] ? lamD[k] * Sn : (R)0;
                        s_inj[i][j] = active[i] ? inj : (R)0;
                    }
                    ++d;
                    next = d < dhi ? pb.date_step[d] : -1;
                }
            }
        }
        dhi = dlo;
        // one reverse step of path i: the adjoint of x~ through step n0 + j; its
        // four node adjoints (nodes b, b + 1 of rows a and a + 1) in u[0..3]
        auto reverse_step = [&](int i, int j, R *u) {
            xb[i] += s_inj[i][j];
            const R sbar = xb[i] * s_c[i][j];
            xb[i] = xb[i] + sbar * s_d[i][j];
            const R al = step_al<R>(pb, n0 + j);
            const R w1 = sbar * s_be[i][j], w0 = sbar - w1;
            u[0] = (1 - al) * w0;
            u[1] = (1 - al) * w1;
            u[2] = al * w0;
            u[3] = al * w1;
        };
        // the time cell of the segment's last step (cells do not decrease with n)
        const int a_last = ldc(pb.step_row, min(n0 + K, pb.N) - 1);
        if (a_last != cur_a) {
            flush_cell<R>(pb, L, cur_a);
            cur_a = a_last;
        }
        if (n0 + K <= pb.N && ldc(pb.step_row, n0) == a_last) {
            // a whole segment in one time cell, without tests between the steps.
            // The slice values an update adds to are read one update ahead,
            // before the previous update's writes; where the two share a node the
            // value just written is forwarded instead, so the LDS latency overlaps
            // the arithmetic and the sums are exactly those of one update at a
            // time (updates in the order: step K-1 path 0, path 1, ..., step 0).
            R *col = my0 + s_b[0][K - 1] * kBlock;
            R r0 = col[0], r1 = col[kBlock], r2 = col[rowB], r3 = col[rowB + kBlock];
#pragma unroll
            for (int j = K - 1; j >= 0; --j) {
#pragma unroll
                for (int i = 0; i < PPL; ++i) {
                    R u[4];
                    reverse_step(i, j, u);
                    const bool last = j == 0 && i == PPL - 1;
                    const int inext = i + 1 < PPL ? i + 1 : 0;
                    const int jnext = i + 1 < PPL ? j : j - 1;
                    R q0 = 0, q1 = 0, q2 = 0, q3 = 0;
                    R *ncol = col;
                    if (!last) {   // the next update's slice values, before this update's writes
                        ncol = my0 + s_b[inext][jnext] * kBlock;
                        q0 = ncol[0];
                        q1 = ncol[kBlock];
                        q2 = ncol[rowB];
                        q3 = ncol[rowB + kBlock];
                    }
                    const R v0 = r0 + u[0], v1 = r1 + u[1], v2 = r2 + u[2], v3 = r3 + u[3];
                    col[0] = v0;
                    col[kBlock] = v1;
                    col[rowB] = v2;
                    col[rowB + kBlock] = v3;
                    if (!last) {
                        const int b = s_b[i][j], bn = s_b[inext][jnext];
                        r0 = bn == b ? v0 : (bn == b + 1 ? v1 : q0);
                        r1 = bn == b ? v1 : (bn + 1 == b ? v0 : q1);
                        r2 = bn == b ? v2 : (bn == b + 1 ? v3 : q2);
                        r3 = bn == b ? v3 : (bn + 1 == b ? v2 : q3);
                        col = ncol;
                    }
                }
            }
        } else {
#pragma unroll
            for (int j = K - 1; j >= 0; --j) {
                const int n = n0 + j;
                if (n < pb.N) {
                    const int a = ldc(pb.step_row, n);
                    if (a != cur_a) {
                        flush_cell<R>(pb, L, cur_a);
                        cur_a = a;
                    }
#pragma unroll
                    for (int i = 0; i < PPL; ++i) {
                        R u[4];
                        reverse_step(i, j, u);
                        R *col = my0 + s_b[i][j] * kBlock;
                        col[0] += u[0];
                        col[kBlock] += u[1];
                        col[rowB] += u[2];
                        col[rowB + kBlock] += u[3];
                    }
                }
            }
        }
    }
    flush_cell<R>(pb, L, cur_a);
    const int M = pb.nT * pb.nK;
    for (int i = tid; i < M; i += kBlock) partial[(int64_t)i * gridDim.x + blockIdx.x] = L.dbl[i];
}

template <typename R, int PPL>
hipError_t pass1_p(const DevProblem &pb, bool store, const double *theta, double *partial, void *ckpt, int64_t nb,
                   hipStream_t st)
{
    const size_t lds = lv_lds_bytes(pb, sizeof(R) == 8, 1);
    if (store)
        hipLaunchKernelGGL((k_lv_pass1<R, true, PPL>), dim3((unsigned)nb), dim3(kBlock), lds, st, pb, theta, partial,
                           (R *)ckpt);
    else
        hipLaunchKernelGGL((k_lv_pass1<R, false, PPL>), dim3((unsigned)nb), dim3(kBlock), lds, st, pb, theta,
                           partial, (R *)ckpt);
    return hipGetLastError();
}

template <typename R>
hipError_t pass1_t(const DevProblem &pb, bool store, const double *theta, double *partial, void *ckpt, int64_t nb,
                   hipStream_t st)
{
    switch (pb.ppl) {
    case 1: return pass1_p<R, 1>(pb, store, theta, partial, ckpt, nb, st);
    case 2: return pass1_p<R, 2>(pb, store, theta, partial, ckpt, nb, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename R, int K, int PPL>
hipError_t pass2_k(const DevProblem &pb, bool from_ckpt, const double *theta, const void *lamD, double *partial,
                   void *ckpt, int64_t nb, hipStream_t st)
{
    const size_t lds = lv_lds_bytes(pb, sizeof(R) == 8, 2);
    if (from_ckpt)
        hipLaunchKernelGGL((k_lv_pass2<R, true, K, PPL>), dim3((unsigned)nb), dim3(kBlock), lds, st, pb, theta,
                           (const R *)lamD, partial, (R *)ckpt);
    else
        hipLaunchKernelGGL((k_lv_pass2<R, false, K, PPL>), dim3((unsigned)nb), dim3(kBlock), lds, st, pb, theta,
                           (const R *)lamD, partial, (R *)ckpt);
    return hipGetLastError();
}

template <typename R, int PPL>
hipError_t pass2_p(const DevProblem &pb, bool from_ckpt, const double *theta, const void *lamD, double *partial,
                   void *ckpt, int64_t nb, hipStream_t st)
{
    switch (pb.K) {
    case 8: return pass2_k<R, 8, PPL>(pb, from_ckpt, theta, lamD, partial, ckpt, nb, st);
    case 16: return pass2_k<R, 16, PPL>(pb, from_ckpt, theta, lamD, partial, ckpt, nb, st);
    case 32: return pass2_k<R, 32, PPL>(pb, from_ckpt, theta, lamD, partial, ckpt, nb, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t pass2_t(const DevProblem &pb, bool from_ckpt, const double *theta, const void *lamD, double *partial,
                   void *ckpt, int64_t nb, hipStream_t st)
{
    switch (pb.ppl) {
    case 1: return pass2_p<R, 1>(pb, from_ckpt, theta, lamD, partial, ckpt, nb, st);
    case 2: return pass2_p<R, 2>(pb, from_ckpt, theta, lamD, partial, ckpt, nb, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t lv_lds_bytes(const DevProblem &pb, bool fp64, int pass)
{
    const size_t real = fp64 ? 8 : 4;
    size_t o = sizeof(double) * (pass == 1 ? (size_t)kWavesPerBlock * pb.m : (size_t)pb.nT * pb.nK);
    o += real * (size_t)pb.K * pb.nK;
    o = (o + 15) & ~(size_t)15;
    if (pass == 2) o += real * 2 * (size_t)pb.nK * kBlock;
    return o;
}

hipError_t launch_lv_pass1(const DevProblem &pb, bool fp64, bool store, const double *theta, double *partial,
                           void *ckpt, int64_t nb, hipStream_t st)
{
    return fp64 ? pass1_t<double>(pb, store, theta, partial, ckpt, nb, st)
                : pass1_t<float>(pb, store, theta, partial, ckpt, nb, st);
}

hipError_t launch_lv_pass2(const DevProblem &pb, bool fp64, bool from_ckpt, const double *theta, const void *lamD,
                           double *partial, void *ckpt, int64_t nb, hipStream_t st)
{
    return fp64 ? pass2_t<double>(pb, from_ckpt, theta, lamD, partial, ckpt, nb, st)
                : pass2_t<float>(pb, from_ckpt, theta, lamD, partial, ckpt, nb, st);
}

}  // namespace mcaad
