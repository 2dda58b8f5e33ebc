// Local-volatility model on gfx950: sigma(t, S) bilinear on a grid of node
// values theta[a*nK + k] at times t_nodes[a] and spots K0 + k dK, flat
// outside the grid; log-Euler x' = x + (r - sigma^2/2) h + sigma sqrt(h) z.
//
// The time weights of step n are the same for every path, so the grid is
// interpolated in time once per step for all paths, for the K steps of the
// current checkpoint segment at a time:
// row_n[k] = (1 - al_n) theta[a_n][k] + al_n theta[a_n + 1][k].  A path-step
// then needs its spot cell b, the weight be and the row's nodes b and b + 1:
// pass 1 keeps the K rows in an LDS window, pass 2 in registers spread over
// the lanes of each wave (ds_bpermute fetches a node), so that its LDS holds
// nothing but the node slices below.
//
// Reverse sweep: sigmabar_n = xbar (-sigma h + sqrt(h) z); the node adjoints
// get sigmabar (1-al)(1-be), (1-al) be, al (1-be), al be at (a, b), (a, b+1),
// (a+1, b), (a+1, b+1).  b differs per lane, a and al do not: each lane
// accumulates sum (1-al) w_k and sum al w_k over the steps of one time cell in
// its own LDS slice (in the path precision: FP32, or FP64 in the FP64 mode),
// and when the time cell changes the workgroup sums the slices over lanes in a
// fixed tree and stores the FP64 sums in its partial columns.
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

// time weight al_n of step n in the path precision (host table, uniform)
template <typename R>
__device__ __forceinline__ R step_al(const DevProblem &pb, int n)
{
    if constexpr (sizeof(R) == 4) return ldc(pb.step_al_f, n);
    else return ldc(pb.step_al, n);
}

template <typename R>
struct Cell {
    int b;
    R be, r0, r1, sig;
    bool inside;
};

// The time-interpolated rows of every step, computed once per launch into a
// table (the values build_window computes): rows[n][k].
template <typename R>
__global__ __launch_bounds__(kBlock) void k_lv_rows(DevProblem pb, const double *__restrict__ theta,
                                                    R *__restrict__ rows)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= pb.N * pb.nK) return;
    const int n = i / pb.nK, k = i - n * pb.nK;
    const int a = pb.step_row[n];
    const double al = (double)step_al<R>(pb, n);
    rows[i] = (R)((1.0 - al) * theta[a * pb.nK + k] + al * theta[(a + 1) * pb.nK + k]);
}

// Pass 2 keeps the segment's rows in registers instead of an LDS window:
// lane k < nK of every wave holds node k of each of the K rows, and a
// path-step takes the two nodes of its cell from those lanes with ds_bpermute
// (which moves data between lanes and uses no LDS space).  Each wave loads its
// own copy from the table, so the window needs no barrier and the LDS holds
// only the node slices.
template <typename R, int K>
__device__ __forceinline__ void rows_to_regs(const DevProblem &pb, const R *__restrict__ rows, int n0, R (&v)[K])
{
    const int k = min((int)(threadIdx.x & (kWave - 1)), pb.nK - 1);
#pragma unroll
    for (int j = 0; j < K; ++j) v[j] = rows[min(n0 + j, pb.N - 1) * pb.nK + k];   // rows past N: never read
}

// v of lane `src` of this wave (every lane active)
template <typename R>
__device__ __forceinline__ R lane_value(R v, int src)
{
    if constexpr (sizeof(R) == 4) {
        return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
    } else {
        const long long w = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(w & 0xffffffffll));
        const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(w >> 32));
        return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
    }
}

// locate() with the row held across the wave's lanes
template <typename R>
__device__ __forceinline__ Cell<R> locate_lanes(const DevProblem &pb, R row, R S, R K0, R invdK, R Klast)
{
    Cell<R> c;
    const R u = (S - K0) * invdK;
    int b = (int)floor(u);
    b = b < 0 ? 0 : (b > pb.nK - 2 ? pb.nK - 2 : b);
    R be = u - (R)b;
    be = be < (R)0 ? (R)0 : (be > (R)1 ? (R)1 : be);
    c.b = b;
    c.be = be;
    c.r0 = lane_value(row, b);
    c.r1 = lane_value(row, b + 1);
    c.sig = c.r0 + be * (c.r1 - c.r0);
    c.inside = S >= K0 && S <= Klast;
    return c;
}

// Rows 4 c .. 4 c + 3 (the steps of Philox call c) into registers, node
// `lane` of each, as rows_to_regs.
template <typename R>
__device__ __forceinline__ void call_rows(const DevProblem &pb, const R *__restrict__ rows, int c, R (&v)[4])
{
    const int k = min((int)(threadIdx.x & (kWave - 1)), pb.nK - 1);
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = rows[min(4 * c + j, pb.N - 1) * pb.nK + k];
}

// Pass 1.  A lane runs PPL paths side by side (independent dependency
// chains, which hide each other's latency): path i of the lane in workgroup
// blk is (blk * PPL + i) * kBlock + tid.  The grid rows come from the table
// into registers (see rows_to_regs), those of the next Philox call loaded
// while the current one runs; LDS holds the waves' payoff sums.
template <typename R, bool STORE, int PPL>
__global__ __launch_bounds__(kBlock) void k_lv_pass1(DevProblem pb, const double *__restrict__ theta,
                                                     const R *__restrict__ rowtab, double *__restrict__ partial,
                                                     R *__restrict__ ckpt)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    double *sums = reinterpret_cast<double *>(lds_raw);   // [waves][m]
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
    R rows[4], rows_next[4];
    call_rows<R>(pb, rowtab, 0, rows);
    for (int call = 0; call < ncalls; ++call) {
        call_rows<R>(pb, rowtab, min(call + 1, ncalls - 1), rows_next);
        if constexpr (STORE) {
            if (call % cps == 0) {
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
                    const Cell<R> c = locate_lanes<R>(pb, rows[j], S, K0, invdK, Klast);
                    x[i] = x[i] + (rh - hh * c.sig * c.sig) + (sq * c.sig) * z[i][j];
                }
                if (n + 1 == next) {
#pragma unroll
                    for (int i = 0; i < PPL; ++i) {
                        const double Sd = (double)(s0 * exp_t(x[i]));
                        payoff_sums(pb.strike, pb.disc, Sd, active[i], lane, pb.date_begin[d], pb.date_begin[d + 1],
                                    sums + wave * pb.m, i > 0);
                    }
                    ++d;
                    next = d < pb.ndates ? pb.date_step[d] : -1;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) rows[j] = rows_next[j];
    }
    __syncthreads();
    for (int k = tid; k < pb.m; k += kBlock) {
        double s = sums[k];
#pragma unroll
        for (int w = 1; w < kWavesPerBlock; ++w) s += sums[w * pb.m + k];
        partial[(int64_t)k * gridDim.x + blockIdx.x] = s;
    }
}

// Sum the lane slices of time cell `a` over the workgroup and store the sums
// in this workgroup's partial columns, then clear the slices.  Slice rows
// k < nK hold the weights 1 - al of node (a, k), rows nK + k the weights al of
// node (a + 1, k); a node's two parts go to columns of their own (a * nK + k,
// and M + (a + 1) * nK + k), each written once per workgroup, and the final
// reduction adds them: the FP64 sums need no LDS.  As in flush_slices, wave w
// takes rows w, w + 4, ...; each lane adds four neighbouring columns of the
// row in the slices' precision, the wave sums them along wave_sum's tree.
// Called by every thread (uniform).
template <typename R>
__device__ void flush_cell(const DevProblem &pb, R *slices, int a, double *__restrict__ partial)
{
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const int64_t M = (int64_t)pb.nT * pb.nK;
    __syncthreads();
#pragma unroll 1
    for (int q = wave; q < 2 * pb.nK; q += kWavesPerBlock) {
        R *cell = slices + q * kBlock + 4 * lane;
        double t;
        if constexpr (sizeof(R) == 4) {
            const float4 v = *reinterpret_cast<float4 *>(cell);
            *reinterpret_cast<float4 *>(cell) = make_float4(0.f, 0.f, 0.f, 0.f);
            t = (double)((v.x + v.y) + (v.z + v.w));
        } else {
            const double2 v0 = reinterpret_cast<double2 *>(cell)[0], v1 = reinterpret_cast<double2 *>(cell)[1];
            reinterpret_cast<double2 *>(cell)[0] = make_double2(0.0, 0.0);
            reinterpret_cast<double2 *>(cell)[1] = make_double2(0.0, 0.0);
            t = (v0.x + v0.y) + (v1.x + v1.y);
        }
        t = wave_sum(t);
        if (lane == 0) {
            const int64_t col = q < pb.nK ? (int64_t)a * pb.nK + q : M + (int64_t)(a + 1) * pb.nK + (q - pb.nK);
            partial[col * gridDim.x + blockIdx.x] = t;
        }
    }
    __syncthreads();
}

// Pass 2.  PPL paths per lane side by side, as in pass 1; their node
// adjoints go to the lane's one column of slices, path 0 first at every step.
// LDS holds the slices only ([2 nK][kBlock] in the path precision); the node
// sums go to the partial columns (2 M of them: see flush_cell).
template <typename R, bool FROM_CKPT, int K, int PPL>
__global__ __launch_bounds__(kBlock) void k_lv_pass2(DevProblem pb, const double *__restrict__ theta,
                                                     const R *__restrict__ rowtab, const R *__restrict__ lamD,
                                                     double *__restrict__ partial, R *__restrict__ ckpt)
{
    static_assert(K % 4 == 0, "segments start on a Philox call");
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    R *slices = reinterpret_cast<R *>(lds_raw);
    const int tid = threadIdx.x;
    int64_t p[PPL];
    bool active[PPL];
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
        p[i] = ((int64_t)blockIdx.x * PPL + i) * kBlock + tid;
        active[i] = p[i] < pb.P;
    }
    if constexpr (!FROM_CKPT) save_theta(pb, theta, blockIdx.x);
    // this workgroup's partial columns start at zero (cells no path of it visits)
    for (int i = tid; i < 2 * pb.nT * pb.nK; i += kBlock) partial[(int64_t)i * gridDim.x + blockIdx.x] = 0.0;
    for (int i = tid; i < 2 * pb.nK * kBlock; i += kBlock) slices[i] = (R)0;
    __syncthreads();

    const R s0 = (R)pb.s0, rh = (R)(pb.rate * pb.h), hh = (R)(0.5 * pb.h), sq = (R)pb.sq, h = (R)pb.h;
    const R K0 = (R)pb.K0, invdK = (R)(1.0 / pb.dK), Klast = (R)(pb.K0 + (pb.nK - 1) * pb.dK);
    const R *strike_r;
    if constexpr (sizeof(R) == 4) strike_r = pb.strike_f;
    else strike_r = pb.strike;
    R rows[K];   // the current segment's rows, node `lane` of each (see rows_to_regs)

    if constexpr (!FROM_CKPT) {
        // the forward re-run of the paper's step 2, storing every segment's start
        R x[PPL];
#pragma unroll
        for (int i = 0; i < PPL; ++i) x[i] = (R)0;
        for (int seg = 0; seg < pb.nseg; ++seg) {
            const int n0 = seg * K;
            rows_to_regs<R, K>(pb, rowtab, n0, rows);
#pragma unroll
            for (int i = 0; i < PPL; ++i)
                if (active[i]) ckpt[(int64_t)seg * pb.P + p[i]] = x[i];
            R z[PPL][4];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int n = n0 + j;
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
                        const Cell<R> c = locate_lanes<R>(pb, rows[j], S, K0, invdK, Klast);
                        x[i] = x[i] + (rh - hh * c.sig * c.sig) + (sq * c.sig) * z[i][j % 4];
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
    R *my0 = slices + tid;   // this lane's column of the slices
    const int rowB = pb.nK * kBlock;
    for (int seg = pb.nseg - 1; seg >= 0; --seg) {
        const int n0 = seg * K;
        rows_to_regs<R, K>(pb, rowtab, n0, rows);
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
        //   the spot cell b (four to a register, one byte each) and its
        //   weight be, the payoff adjoint injected
        R s_c[PPL][K], s_d[PPL][K], s_be[PPL][K], s_inj[PPL][K];
        uint32_t s_b4[PPL][(K + 3) / 4];
        R z[PPL][4];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int n = n0 + j;
#pragma unroll
            for (int i = 0; i < PPL; ++i) {
                s_inj[i][j] = (R)0;
                if (j % 4 == 0) s_b4[i][j / 4] = 0u;
            }
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
                    const Cell<R> c = locate_lanes<R>(pb, rows[j], S, K0, invdK, Klast);
                    s_c[i][j] = -c.sig * h + sq * z[i][j % 4];
                    s_d[i][j] = (c.inside ? (c.r1 - c.r0) * invdK : (R)0) * S;
                    s_b4[i][j / 4] |= (uint32_t)c.b << (8 * (j % 4));
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
        auto cell_of = [&](int i, int j) { return (int)((s_b4[i][j / 4] >> (8 * (j % 4))) & 0xffu); };
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
            flush_cell<R>(pb, slices, cur_a, partial);
            cur_a = a_last;
        }
        if (n0 + K <= pb.N && ldc(pb.step_row, n0) == a_last) {
            // a whole segment in one time cell, without tests between the steps.
            // The slice values an update adds to are read one update ahead,
            // before the previous update's writes; where the two share a node the
            // value just written is forwarded instead, so the LDS latency overlaps
            // the arithmetic and the sums are exactly those of one update at a
            // time (updates in the order: step K-1 path 0, path 1, ..., step 0).
            R *col = my0 + cell_of(0, K - 1) * kBlock;
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
                        ncol = my0 + cell_of(inext, jnext) * kBlock;
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
                        const int b = cell_of(i, j), bn = cell_of(inext, jnext);
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
                        flush_cell<R>(pb, slices, cur_a, partial);
                        cur_a = a;
                    }
#pragma unroll
                    for (int i = 0; i < PPL; ++i) {
                        R u[4];
                        reverse_step(i, j, u);
                        R *col = my0 + cell_of(i, j) * kBlock;
                        col[0] += u[0];
                        col[kBlock] += u[1];
                        col[rowB] += u[2];
                        col[rowB + kBlock] += u[3];
                    }
                }
            }
        }
    }
    flush_cell<R>(pb, slices, cur_a, partial);
}

template <typename R, int PPL>
hipError_t pass1_p(const DevProblem &pb, bool store, const double *theta, const void *rows, double *partial,
                   void *ckpt, int64_t nb, hipStream_t st)
{
    const size_t lds = lv_lds_bytes(pb, sizeof(R) == 8, 1);
    if (store)
        hipLaunchKernelGGL((k_lv_pass1<R, true, PPL>), dim3((unsigned)nb), dim3(kBlock), lds, st, pb, theta,
                           (const R *)rows, partial, (R *)ckpt);
    else
        hipLaunchKernelGGL((k_lv_pass1<R, false, PPL>), dim3((unsigned)nb), dim3(kBlock), lds, st, pb, theta,
                           (const R *)rows, partial, (R *)ckpt);
    return hipGetLastError();
}

template <typename R>
hipError_t pass1_t(const DevProblem &pb, bool store, const double *theta, const void *rows, double *partial,
                   void *ckpt, int64_t nb, hipStream_t st)
{
    switch (pb.ppl) {
    case 1: return pass1_p<R, 1>(pb, store, theta, rows, partial, ckpt, nb, st);
    case 2: return pass1_p<R, 2>(pb, store, theta, rows, partial, ckpt, nb, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename R, int K, int PPL>
hipError_t pass2_k(const DevProblem &pb, bool from_ckpt, const double *theta, const void *rows, const void *lamD,
                   double *partial, void *ckpt, int64_t nb, hipStream_t st)
{
    const size_t lds = lv_lds_bytes(pb, sizeof(R) == 8, 2);
    if (from_ckpt)
        hipLaunchKernelGGL((k_lv_pass2<R, true, K, PPL>), dim3((unsigned)nb), dim3(kBlock), lds, st, pb, theta,
                           (const R *)rows, (const R *)lamD, partial, (R *)ckpt);
    else
        hipLaunchKernelGGL((k_lv_pass2<R, false, K, PPL>), dim3((unsigned)nb), dim3(kBlock), lds, st, pb, theta,
                           (const R *)rows, (const R *)lamD, partial, (R *)ckpt);
    return hipGetLastError();
}

template <typename R, int PPL>
hipError_t pass2_p(const DevProblem &pb, bool from_ckpt, const double *theta, const void *rows, const void *lamD,
                   double *partial, void *ckpt, int64_t nb, hipStream_t st)
{
    switch (pb.K) {
    case 8: return pass2_k<R, 8, PPL>(pb, from_ckpt, theta, rows, lamD, partial, ckpt, nb, st);
    case 16: return pass2_k<R, 16, PPL>(pb, from_ckpt, theta, rows, lamD, partial, ckpt, nb, st);
    case 32: return pass2_k<R, 32, PPL>(pb, from_ckpt, theta, rows, lamD, partial, ckpt, nb, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t pass2_t(const DevProblem &pb, bool from_ckpt, const double *theta, const void *rows, const void *lamD,
                   double *partial, void *ckpt, int64_t nb, hipStream_t st)
{
    switch (pb.ppl) {
    case 1: return pass2_p<R, 1>(pb, from_ckpt, theta, rows, lamD, partial, ckpt, nb, st);
    case 2: return pass2_p<R, 2>(pb, from_ckpt, theta, rows, lamD, partial, ckpt, nb, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

namespace {

// One workgroup per node: thread t adds the node's two parts of blocks t,
// t + 256, ... in order, then a fixed tree (the order and tree of
// k_reduce_sorted, over the sum of the two parts of each block).
__global__ __launch_bounds__(kBlock) void k_lv_reduce(const double *__restrict__ partial, int64_t nblocks, int M,
                                                      double *__restrict__ out, int32_t *status)
{
    __shared__ double sh[kBlock];
    const int k = blockIdx.x, tid = threadIdx.x;
    const double *c0 = partial + (int64_t)k * nblocks, *c1 = partial + (int64_t)(M + k) * nblocks;
    double acc = 0.0;
    for (int64_t b = tid; b < nblocks; b += kBlock) acc += c0[b] + c1[b];
    sh[tid] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (tid < s) sh[tid] += sh[tid + s];
        __syncthreads();
    }
    if (tid == 0) {
        out[k] = sh[0];
        if (!isfinite(sh[0])) atomicOr(status, 2);
    }
}

}  // namespace

hipError_t launch_lv_reduce(const double *partial, int64_t nblocks, int32_t M, double *out, int32_t *status,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_lv_reduce, dim3((unsigned)M), dim3(kBlock), 0, st, partial, nblocks, M, out, status);
    return hipGetLastError();
}

size_t lv_lds_bytes(const DevProblem &pb, bool fp64, int pass)
{
    const size_t real = fp64 ? 8 : 4;
    if (pass == 2) return real * 2 * (size_t)pb.nK * kBlock;   // the node slices
    return sizeof(double) * (size_t)kWavesPerBlock * pb.m;      // the waves' payoff sums
}

hipError_t launch_lv_pass1(const DevProblem &pb, bool fp64, bool store, const double *theta, const void *rows,
                           double *partial, void *ckpt, int64_t nb, hipStream_t st)
{
    return fp64 ? pass1_t<double>(pb, store, theta, rows, partial, ckpt, nb, st)
                : pass1_t<float>(pb, store, theta, rows, partial, ckpt, nb, st);
}

hipError_t launch_lv_rows(const DevProblem &pb, bool fp64, const double *theta, void *rows, hipStream_t st)
{
    const unsigned g = (unsigned)((pb.N * pb.nK + kBlock - 1) / kBlock);
    if (fp64) hipLaunchKernelGGL(k_lv_rows<double>, dim3(g), dim3(kBlock), 0, st, pb, theta, (double *)rows);
    else hipLaunchKernelGGL(k_lv_rows<float>, dim3(g), dim3(kBlock), 0, st, pb, theta, (float *)rows);
    return hipGetLastError();
}

hipError_t launch_lv_pass2(const DevProblem &pb, bool fp64, bool from_ckpt, const double *theta, const void *rows,
                           const void *lamD, double *partial, void *ckpt, int64_t nb, hipStream_t st)
{
    return fp64 ? pass2_t<double>(pb, from_ckpt, theta, rows, lamD, partial, ckpt, nb, st)
                : pass2_t<float>(pb, from_ckpt, theta, rows, lamD, partial, ckpt, nb, st);
}

}  // namespace mcaad
