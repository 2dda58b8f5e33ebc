// Black-Scholes with the Euler scheme applied to the SDE as it is written,
// dS = r S dt + sigma S dW (the paper names a standard Euler discretisation;
// section "Test on the Heston SLV model calibration"), on gfx950:
//   S_{n+1} = S_n (1 + r h + sigma z'_n),   z' = sqrt(h) z,
// one path per lane, the spot itself in a VGPR (FP32 or FP64), so a payoff
// needs no exponential.  The step is multiplicative, so the reverse sweep
// carries the spot adjoint a through every step:
//   sigma_bar += a_{n+1} S_n z'_n,   a_n = a_{n+1} (1 + r h + sigma z'_n),
// with lambda_i D_i 1{S > K_i} / P added to a at the maturity steps (the
// payoff's derivative in S is the indicator: no factor S as for log S).
// The step is taken as S + S (r h + sigma z'), one fused multiply-add on an
// increment formed first: in FP32, S (1 + r h + ...) would round 1 + r h
// (relative 2^-24 against r h ~ 1e-4), a bias that compounds over the steps
// (1e-4 on the prices at 256 steps); the adjoint's factor is applied the same way.
// Structure as the log-Euler passes: Philox normals regenerated, the spot
// stored every K steps by a storing pass 1, each K-step segment recomputed
// in pass 2 with (S_n, z'_n) kept in registers, FP32 sums per segment, FP64
// across segments, one wave reduction per workgroup and a fixed-order final sum.
#include <hip/hip_runtime.h>

#include "bse_kernels.hpp"
#include "mc_device.hpp"
#include "models.hpp"

namespace mcaad {
namespace {

// Pass 1 (paper: algorithm step 1): lds holds [kWavesPerBlock][m] payoff sums.
template <typename R, bool STORE>
__global__ __launch_bounds__(kBlock) void k_bse_pass1(DevProblem pb, const double *__restrict__ theta,
                                                      double *__restrict__ partial, R *__restrict__ ckpt)
{
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const int64_t blk = blockIdx.x;
    if (blk == 0 && tid == 0) check_theta<kBS>(pb, theta);   // sigma finite and >= 0
    if constexpr (STORE) save_theta(pb, theta, blk);
    const R rh = (R)(pb.rate * pb.h), sig = (R)theta[0];
    const R bm = box_muller_scale<R>(pb.h);
    const int ncalls = (pb.N + 3) / 4;   // one normal per step, four per Philox call
    const int cps = max(pb.K / 4, 1);    // Philox calls per checkpoint segment
    for (int sp = 0; sp < pb.ppl; ++sp) {
        const int64_t p = (blk * pb.ppl + sp) * kBlock + tid;
        const bool active = p < pb.P;
        R S = (R)pb.s0;
        int d = 0;
        int next = pb.ndates > 0 ? ldc(pb.date_step, 0) : -1;
        R *cp = ckpt + p;
        for (int call = 0; call < ncalls; cp += pb.P) {
            if constexpr (STORE) {
                if (active) cp[0] = S;
            }
            const int cend = min(call + cps, ncalls);
            for (; call < cend; ++call) {
                R z[4];
                normals4<R>((uint32_t)call, (uint32_t)p, pb.inst, pb.k0, pb.k1, bm, z);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int n = call * 4 + j;
                    if (n < pb.N) {
                        S = fma(S, rh + sig * z[j], S);
                        if (n + 1 == next) {
                            payoff_sums(pb.strike, pb.disc, (double)S, active, lane, ldc(pb.date_begin, d),
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

// Pass 2 (paper: algorithm step 2, eq. 0711A): lds holds [kWavesPerBlock]
// FP64 sums, then [K][kBlock] reals, one column per lane, for the payoff
// adjoints of the maturity dates of the current segment.
template <typename R, int K>
constexpr size_t bse_pass2_lds()
{
    return sizeof(double) * kWavesPerBlock + sizeof(R) * K * kBlock;
}

template <typename R, bool FROM_CKPT, int K>
__global__ __launch_bounds__(kBlock) void k_bse_pass2(DevProblem pb, const double *__restrict__ theta,
                                                      const R *__restrict__ lamD, double *__restrict__ partial,
                                                      R *__restrict__ ckpt)
{
    static_assert(K % 4 == 0, "segments start on a Philox call");
    extern __shared__ double lds[];
    R *inj_lds = reinterpret_cast<R *>(lds + kWavesPerBlock);
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const int64_t blk = blockIdx.x;
    if constexpr (!FROM_CKPT) save_theta(pb, theta, blk);
    const R rh = (R)(pb.rate * pb.h), sig = (R)theta[0];
    const R bm = box_muller_scale<R>(pb.h);
    const R *strike_r;
    if constexpr (sizeof(R) == 4) strike_r = pb.strike_f;
    else strike_r = pb.strike;

    double g = 0.0;
    for (int sp = 0; sp < pb.ppl; ++sp) {
        const int64_t p = (blk * pb.ppl + sp) * kBlock + tid;
        const bool active = p < pb.P;
        const uint32_t path = (uint32_t)p;
        if constexpr (!FROM_CKPT) {
            // the forward re-run of the paper's step 2, keeping every segment's start
            R S = (R)pb.s0;
            const int ncalls = (pb.N + 3) / 4;
            for (int call = 0; call < ncalls; ++call) {
                R z[4];
                normals4<R>((uint32_t)call, path, pb.inst, pb.k0, pb.k1, bm, z);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int n = call * 4 + j;
                    if (n < pb.N) {
                        if ((n % K) == 0 && active) ckpt[(int64_t)(n / K) * pb.P + p] = S;
                        S = fma(S, rh + sig * z[j], S);
                    }
                }
            }
        }

        R a = (R)0;                 // adjoint of the spot after the current step
        int dhi = pb.ndates;        // dates with index < dhi mature at or before this segment's end
        for (int seg = pb.nseg - 1; seg >= 0; --seg) {
            const int n0 = seg * K;
            // inactive lanes (past the last path) run a harmless path from S0
            // and add nothing; they read no checkpoint, since in the re-run mode
            // another workgroup may still be writing the one they would share
            // (the index is clamped as well, so the address stays inside the
            // buffer whatever form the compiler gives the selection)
            R S = active ? ckpt[(int64_t)seg * pb.P + (active ? p : 0)] : (R)pb.s0;
            int dlo = dhi;
            while (dlo > 0 && ldc(pb.date_step, dlo - 1) > n0) --dlo;
            int d = dlo;
            int next = d < dhi ? ldc(pb.date_step, d) : -1;

            // recompute the segment keeping S_n and z'_n of every step
            R s_S[K], s_z[K];
            R z[4];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int n = n0 + j;
                s_S[j] = (R)0;
                s_z[j] = (R)0;
                if (n < pb.N) {
                    if (j % 4 == 0) normals4<R>((uint32_t)(n / 4), path, pb.inst, pb.k0, pb.k1, bm, z);
                    s_S[j] = S;
                    s_z[j] = z[j % 4];
                    S = fma(S, rh + sig * z[j % 4], S);
                    if (n + 1 == next) {
                        // payoff adjoints of this date: sum_i lambda_i D_i / P 1{S > K_i}
                        R inj = (R)0;
                        for (int k = ldc(pb.date_begin, d); k < ldc(pb.date_begin, d + 1); ++k)
                            inj += S > ldc(strike_r, k) ? ldc(lamD, k) : (R)0;
                        inj_lds[j * kBlock + tid] = active ? inj : (R)0;
                        ++d;
                        next = d < dhi ? ldc(pb.date_step, d) : -1;
                    }
                }
            }
            dhi = dlo;

            // reverse sweep over the segment; its dates are dlo .. d-1, met last first
            int dr = d - 1;
            int rnext = dr >= dlo ? ldc(pb.date_step, dr) : -1;
            R sb = (R)0;
#pragma unroll
            for (int j = K - 1; j >= 0; --j) {
                if (n0 + j < pb.N) {
                    if (n0 + j + 1 == rnext) {
                        a += inj_lds[j * kBlock + tid];
                        --dr;
                        rnext = dr >= dlo ? ldc(pb.date_step, dr) : -1;
                    }
                    sb += a * (s_S[j] * s_z[j]);
                    a = fma(a, rh + sig * s_z[j], a);
                }
            }
            g += active ? (double)sb : 0.0;
        }
    }

    const double t = wave_sum(g);
    if (lane == 0) lds[wave] = t;
    __syncthreads();
    if (tid == 0) {
        double s = lds[0];
#pragma unroll
        for (int w = 1; w < kWavesPerBlock; ++w) s += lds[w];
        partial[blk] = s;
    }
}

template <typename R>
hipError_t pass1_t(const DevProblem &pb, bool store, const double *theta, double *partial, void *ckpt, int64_t nb,
                   hipStream_t st)
{
    const size_t lds = sizeof(double) * kWavesPerBlock * pb.m;
    if (store)
        hipLaunchKernelGGL((k_bse_pass1<R, true>), dim3((unsigned)nb), dim3(kBlock), lds, st, pb, theta, partial,
                           (R *)ckpt);
    else
        hipLaunchKernelGGL((k_bse_pass1<R, false>), dim3((unsigned)nb), dim3(kBlock), lds, st, pb, theta, partial,
                           (R *)ckpt);
    return hipGetLastError();
}

template <typename R, int K>
hipError_t pass2_k(const DevProblem &pb, bool from_ckpt, const double *theta, const void *lamD, double *partial,
                   void *ckpt, int64_t nb, hipStream_t st)
{
    const size_t lds = bse_pass2_lds<R, K>();
    if (from_ckpt)
        hipLaunchKernelGGL((k_bse_pass2<R, true, K>), dim3((unsigned)nb), dim3(kBlock), lds, st, pb, theta,
                           (const R *)lamD, partial, (R *)ckpt);
    else
        hipLaunchKernelGGL((k_bse_pass2<R, false, K>), dim3((unsigned)nb), dim3(kBlock), lds, st, pb, theta,
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

hipError_t launch_bse_pass1(const DevProblem &pb, bool fp64, bool store, const double *theta, double *partial,
                            void *ckpt, int64_t nb, hipStream_t st)
{
    return fp64 ? pass1_t<double>(pb, store, theta, partial, ckpt, nb, st)
                : pass1_t<float>(pb, store, theta, partial, ckpt, nb, st);
}

hipError_t launch_bse_pass2(const DevProblem &pb, bool fp64, bool from_ckpt, const double *theta, const void *lamD,
                            double *partial, void *ckpt, int64_t nb, hipStream_t st)
{
    return fp64 ? pass2_t<double>(pb, from_ckpt, theta, lamD, partial, ckpt, nb, st)
                : pass2_t<float>(pb, from_ckpt, theta, lamD, partial, ckpt, nb, st);
}

}  // namespace mcaad
