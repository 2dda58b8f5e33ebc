// Kernel-side problem description and launch entry points of the Monte Carlo
// passes (internal to the library; the public boundary is include/mcaad.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcaad {

enum Model { kBS = 0, kHeston = 1, kLV = 2, kSLV = 3 };

// Everything a kernel needs besides theta, passed by value.
struct DevProblem {
    int32_t N;            // Euler steps
    int32_t m;            // instruments
    int32_t M;            // parameters
    int32_t ndates;       // distinct maturity steps
    int32_t nseg;         // checkpoint segments = ceil(N / K)
    int32_t K;            // checkpoint spacing (8, 16, 32)
    int32_t ppl;          // paths per lane, run one after another (1, 2, 4)
    int64_t P;            // paths
    uint32_t k0, k1;      // Philox key
    uint32_t inst;        // Philox counter word 2
    double s0, rate, h, sq;
    const int32_t *date_step;   // [ndates] ascending maturity steps
    const int32_t *date_begin;  // [ndates + 1] ranges into the date-sorted tables
    const double *strike;       // [m] date-sorted strikes
    const float *strike_f;      // [m] the same in FP32
    const double *disc;         // [m] date-sorted discount factors exp(-r n_i h)
    const int32_t *id;          // [m] original index of date-sorted instrument k
    int32_t *status;            // device status bits
    // local volatility: bilinear grid on time nodes t_nodes[nT] and uniformly
    // spaced spot nodes K0 + k dK, k < nK; theta[a*nK + k] is the node value;
    // step n lies in time cell step_row[n] = a (a <= nT - 2) with weight
    // step_al[n] on node row a + 1 (host tables).
    // Stochastic local volatility: the same spot nodes, theta[5 + a*nK + k] is
    // the leverage of time row a, and step n uses row step_row[n].
    int32_t nT, nK;
    double K0, dK;
    const double *t_nodes;
    const int32_t *step_row;    // [N]
    const double *step_al;      // [N] (local volatility)
    const float *step_al_f;     // [N] the same in FP32
    // where a sweep that writes every checkpoint segment (pass 1 storing, pass
    // 2 re-running the forward sweep) leaves a copy of theta (workgroup 0
    // writes it; M doubles); null: no copy
    double *theta_save;
};

// Workgroup 0 of a checkpoint-writing sweep keeps theta beside the buffer.
__device__ __forceinline__ void save_theta(const DevProblem &pb, const double *theta, int64_t blk)
{
    if (blk == 0 && pb.theta_save)
        for (int i = threadIdx.x; i < pb.M; i += blockDim.x) pb.theta_save[i] = theta[i];
}

// One instance of a batch: its problem plus its slices of the batch workspace.
struct BatchInst {
    DevProblem pb;
    double *part_y;    // [m][nblocks]
    double *part_g;    // [M][nblocks]
    void *ckpt;        // [nseg][n_state][P] in the path precision
    void *lamD;        // [m] in the path precision
    int64_t nblocks;
    int32_t y_off;     // first index of this instance in the concatenated C / Ey arrays
    int32_t pad_;
};

// Everything one batched gradient step launches with.
struct BatchLaunch {
    int model;
    bool fp64;
    int K;
    int n_inst;
    int n_items;
    int max_m;
    unsigned grid;             // persistent workgroups
    const BatchInst *insts;    // device [n_inst]
    const int2 *items;         // device [n_items] (instance, block), longest instances first
    unsigned *counters;        // device [2] work-queue heads of the two passes
    const double *theta;       // device [n_inst][M]
    const double *C;           // device, concatenated
    double *Ey;                // device, concatenated
    double *G;                 // device [n_inst]
    double *grad;              // device [n_inst][M]
};

hipError_t launch_batch_step(const BatchLaunch &L, hipStream_t st);
int batch_blocks_per_cu(int model, bool fp64, int K, int max_m);

// Local-volatility passes (lv_kernels.hip).
// rows [N][nK] (path precision): the grid interpolated in time at every step,
// from launch_lv_rows; pass 2's partial: 2 nT nK columns of nblocks (see
// launch_lv_reduce)
hipError_t launch_lv_pass1(const DevProblem &pb, bool fp64, bool store_ckpt, const double *theta, const void *rows,
                           double *partial, void *ckpt, int64_t nblocks, hipStream_t stream);
hipError_t launch_lv_pass2(const DevProblem &pb, bool fp64, bool from_ckpt, const double *theta, const void *rows,
                           const void *lamD, double *partial, void *ckpt, int64_t nblocks, hipStream_t stream);
// rows[n][k] = (1 - al_n) theta[a_n][k] + al_n theta[a_n + 1][k], n < N, k < nK
hipError_t launch_lv_rows(const DevProblem &pb, bool fp64, const double *theta, void *rows, hipStream_t stream);
// pass 2 stores each node's FP64 sums in two partial columns per workgroup
// (the node row's own time cell and the cell below it):
// out[k] = sum over workgroups b of (partial[k][b] + partial[M + k][b]),
// k < M = nT nK, in a fixed order; status bit 2 for a non-finite sum
hipError_t launch_lv_reduce(const double *partial, int64_t nblocks, int32_t M, double *out, int32_t *status,
                            hipStream_t stream);
size_t lv_lds_bytes(const DevProblem &pb, bool fp64, int pass);

// Heston stochastic local volatility passes (slv_kernels.hip).
hipError_t launch_slv_pass1(const DevProblem &pb, bool fp64, bool store_ckpt, const double *theta,
                            double *partial, void *ckpt, int64_t nblocks, hipStream_t stream);
hipError_t launch_slv_pass2(const DevProblem &pb, bool fp64, bool from_ckpt, const double *theta, const void *lamD,
                            double *partial, void *ckpt, int64_t nblocks, hipStream_t stream);
size_t slv_lds_bytes(const DevProblem &pb, bool fp64, int pass);

// All launchers enqueue on `stream` and return hipGetLastError().
hipError_t launch_pass1(const DevProblem &pb, int model, bool fp64, bool store_ckpt, const double *theta,
                        double *partial, void *ckpt, int64_t nblocks, hipStream_t stream);
hipError_t launch_pass2(const DevProblem &pb, int model, bool fp64, bool from_ckpt, const double *theta,
                        const void *lamD, double *partial, void *ckpt, int64_t nblocks, hipStream_t stream);
// ninst instances along the grid's y dimension (theta and partials per instance)
hipError_t launch_tangent(const DevProblem &pb, int model, bool fp64, const double *theta, double *partial,
                          int64_t nblocks, int ninst, hipStream_t stream);
hipError_t launch_reduce_jac(const double *partial, int64_t nblocks, int32_t M, int32_t m, const int32_t *id,
                             double scale, double *Ey, double *J, int32_t *status, int ninst, hipStream_t st);
hipError_t launch_check_theta(const DevProblem &pb, const double *theta, int model, hipStream_t st);
// out[id[k]] = scale * sum_b partial[k*nblocks + b] for k < count (fixed order;
// block partials are stored column by column)
hipError_t launch_reduce_sorted(const double *partial, int64_t nblocks, int32_t count, const int32_t *id,
                                double scale, double *out, int32_t *status, hipStream_t stream);
// r = Ey - C, G = 1/2 sum r^2, lamD[k] = r[id[k]] * disc[k] / P (in FP32 or FP64)
hipError_t launch_residual(const DevProblem &pb, bool fp64, const double *Ey, const double *C, double *G,
                           void *lamD, const double *theta, hipStream_t stream);
// lamD[k] = lambda[id[k]] * disc[k] / P
// saved (may be null): the theta the checkpoints were written with; status
// bit 4 is set when theta differs from it in any bit.
hipError_t launch_lambda(const DevProblem &pb, bool fp64, const double *lambda, void *lamD, const double *saved,
                         const double *theta, hipStream_t stream);
hipError_t launch_philox(const uint32_t *ctr, uint32_t k0, uint32_t k1, int64_t n, uint32_t *out,
                         hipStream_t stream);
hipError_t launch_normals(bool fp64, uint32_t k0, uint32_t k1, uint32_t inst, uint32_t path0, int64_t npaths,
                          uint32_t q0, int32_t nq, void *out, hipStream_t stream);

}  // namespace mcaad
