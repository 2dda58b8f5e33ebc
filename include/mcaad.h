/*
 * mcaad.h - C ABI of the MI355X (gfx950) library for the two-pass Monte Carlo
 * adjoint gradient of the calibration functional
 *
 *     G(theta) = 1/2 sum_{i=1..m} (E y_i(theta) - C_i)^2          (paper, eq. 241118A)
 *
 * where y_i are the m payoffs that the forward algorithm F : R^{M+N} -> R^m
 * produces for one path from M parameters and N random variables (paper,
 * problem statement after eq. 241118A), and E is the Monte Carlo mean over P
 * paths (paper, eq. 1211A).
 *
 * Conventions for every entry point:
 *   - "d_" arguments are device pointers (HIP global memory on the current
 *     device), "h_"/plain struct members are host pointers.
 *   - All device arrays are contiguous, FP64, owned by the caller; the
 *     library never frees or retains them beyond the call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream). Work
 *     is enqueued on it and the call returns without synchronising, except
 *     cal_status and cal_timing_read, which synchronise.
 *   - The context owns all workspace (block partial sums, checkpoints,
 *     sorted instrument tables). It is allocated once in cal_create; the
 *     calibrate_* calls allocate nothing and only launch kernels (no copies,
 *     memsets or synchronisation), so a call can be captured into a HIP graph
 *     (with cal_timing_enable off) and replayed; the graph reads its
 *     arguments' memory at replay time.
 *     One context serves one stream at a time: calls on one context that
 *     overlap on different streams race.
 *   - Return value 0 = success, negative = error (CAL_E*). On error nothing is
 *     enqueued and cal_last_error(ctx) describes it. Nothing throws or aborts
 *     across this boundary.
 *   - Floating point: path state and per-path arithmetic in FP32
 *     (CAL_FP32) or FP64 (CAL_FP64); sums over paths, the residual
 *     E y - C, G and the gradient are always FP64 and are reduced in a fixed
 *     order, so results are bitwise reproducible run to run.
 */
#ifndef MCAAD_H
#define MCAAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* model */
#define CAL_BS 0      /* Black-Scholes GBM, theta = (sigma), log-Euler */
#define CAL_HESTON 1  /* Heston, theta = (kappa, theta_bar, xi, rho, v0), full-truncation log-Euler */
#define CAL_LV 2      /* local volatility, theta = node values of sigma(t, S), bilinear on the nodes */
#define CAL_SLV 3     /* Heston stochastic local volatility (the paper's test model): dS/S = r dt +
                         L(t, S) sqrt(v) dW1, v as Heston; theta = (kappa, theta_bar, xi, rho, v0,
                         L[a][k]); L piecewise constant in t, linear across the spot nodes */
#define CAL_BS_EULER_S 4  /* Black-Scholes GBM, theta = (sigma), with the paper's Euler scheme taken
                             literally on the SDE as written in S (section "Test on the Heston SLV
                             model calibration"): S_{n+1} = S_n (1 + r h + sigma sqrt(h) z_n); forward,
                             gradient and vector-Jacobian product only (no tangent mode, batching or
                             calibrate_gradient_static: CAL_EUNSUPPORTED) */

/* precision of the path state */
#define CAL_FP32 0
#define CAL_FP64 1

/* where the reverse sweep gets its checkpoints */
#define CAL_CKPT_AUTO 0    /* the default: CAL_CKPT_STORE (both modes hold the same
                              [N/K][n_state][P] buffer; storing saves pass 2 its re-run) */
#define CAL_CKPT_RERUN 1   /* pass 2 re-runs the forward sweep and keeps its own checkpoints */
#define CAL_CKPT_STORE 2   /* the pass-1 sweep of calibrate_gradient stores them in HBM */

/* return codes */
#define CAL_OK 0
#define CAL_EINVAL (-1)        /* bad problem or argument */
#define CAL_ENOMEM (-2)        /* device allocation failed */
#define CAL_EHIP (-3)          /* a HIP runtime call failed */
#define CAL_EUNSUPPORTED (-4)  /* valid problem the device path does not implement */

/* device status bits reported by cal_status */
#define CAL_FLAG_THETA 1       /* theta outside the model's domain */
#define CAL_FLAG_NONFINITE 2   /* a non-finite E y, G or gradient was produced */
#define CAL_FLAG_CKPT 4        /* calibrate_vjp_stored got a theta other than the one the
                                  checkpoints were written with (its gradient is invalid) */

typedef struct cal_ctx cal_ctx;

/*
 * Problem description (all pointers are host pointers, read during
 * cal_validate / cal_create only).
 *   model, precision  : see above
 *   n_params (M)      : 1 (BS, BS_EULER_S), 5 (Heston), nT*nK (LV), 5 + nT*nK (SLV)
 *   n_instr  (m)      : number of calls, 1..2048
 *   n_steps  (N)      : Euler steps over [0, t_max], 1..65536
 *   n_paths  (P)      : 1..2^32; path p uses Philox counter word 1 = p
 *   seed              : Philox key (lo, hi words)
 *   inst              : Philox counter word 2 (instance / draw index)
 *   ckpt_every (k)    : 0 = auto, else 8, 16 or 32 steps between checkpoints
 *   paths_per_lane    : 0 = 1, else 1, 2 or 4 paths each lane runs one after
 *                       another (a workgroup then covers 256 x that many
 *                       paths); local volatility takes 1 or 2 and runs
 *                       the two side by side (interleaved, not one after
 *                       the other)
 *   ckpt_mode         : CAL_CKPT_*
 *   s0, rate, t_max   : spot, risk-free rate (drift and discounting), horizon
 *   sqrt_eps          : must be 0 (plain full truncation, s = sqrt(v+)); any
 *                       other finite value >= 0 is refused with CAL_EUNSUPPORTED
 *   instr_step[m]     : maturity step of call i, 1..N (maturity = step * t_max / N)
 *   instr_strike[m]   : strike of call i (>= 0)
 *   n_t_nodes (nT), t_nodes[nT] : LV and SLV time nodes, finite and increasing
 *                       (LV: 2..64, bilinear in t, flat outside; SLV: 1..64,
 *                       step n uses row a = #{t_nodes <= n h}, capped at nT-1)
 *   n_k_nodes (nK), k_nodes[nK] : LV and SLV spot nodes, 2..64, uniformly spaced
 *                       (within 1e-9 relative), linear in S, flat outside;
 *                       theta[(5 +) a*nK + k] is the value at (t_a, K_k);
 *                       LV's reverse pass holds 2*nK*256 values of the path
 *                       precision in one workgroup's LDS, so in FP64 nK is
 *                       at most 40 on a 160 KB device (cal_create refuses
 *                       more with CAL_EUNSUPPORTED)
 * Random numbers: normal q of path p is Box-Muller of the uniforms
 * ((w >> 9) + 0.5) 2^-23 of Philox4x32-10 counter (q/4, p, inst, 0), key
 * (seed lo, seed hi); q = n*d + j for normal j of step n (d = 2 for Heston
 * and SLV, 1 otherwise).
 */
typedef struct {
    int32_t model;
    int32_t precision;
    int32_t n_params;
    int32_t n_instr;
    int32_t n_steps;
    int32_t ckpt_every;
    int64_t n_paths;
    uint64_t seed;
    uint32_t inst;
    int32_t ckpt_mode;
    int32_t max_batch;           /* instances per calibrate_jacobian_batch call (0 = 1) */
    int32_t paths_per_lane;      /* 0 or 1, 2, 4 */
    double s0;
    double rate;
    double t_max;
    double sqrt_eps;
    const int32_t *instr_step;
    const double *instr_strike;
    int32_t n_t_nodes;           /* LV, SLV */
    int32_t n_k_nodes;
    const double *t_nodes;
    const double *k_nodes;
} cal_problem;

/* Host-only check of a problem (no HIP call): CAL_OK or CAL_EINVAL /
 * CAL_EUNSUPPORTED.  `msg` (may be NULL) receives a reason, up to `msg_len`
 * bytes including the terminating NUL. */
int cal_validate(const cal_problem *pb, char *msg, int32_t msg_len);

/* Validate, then allocate the context and all its device workspace on the
 * current device.  *out receives the context (NULL on error).  For LV and
 * SLV it also checks the kernels' LDS need against the current device's
 * per-workgroup limit and returns CAL_EUNSUPPORTED when it does not fit. */
int cal_create(const cal_problem *pb, cal_ctx **out);

/* Free the context and its workspace (synchronises the device first).
 * NULL is accepted. */
int cal_destroy(cal_ctx *ctx);

/* Pass 1 of the paper's algorithm (its step 1, cost eq. 1211A): the forward
 * sweep F_v over all paths and the sample means.
 *   d_theta[M] : parameters (FP64, device)
 *   d_Ey[m]    : out, E y_i = (1/P) sum_p y_i(p) (FP64, device) */
int calibrate_forward(cal_ctx *ctx, const double *d_theta, double *d_Ey, void *stream);

/* Pass 2 alone with a caller-given output adjoint (eq. 0711A summed over
 * paths): d_grad[j] = sum_i lambda_i dE y_i/dtheta_j, where each path runs
 * the forward sweep again and then its reverse sweep seeded with lambda_i/P.
 *   d_lambda[m] : adjoint of E y (FP64, device)
 *   d_grad[M]   : out (FP64, device) */
int calibrate_vjp(cal_ctx *ctx, const double *d_theta, const double *d_lambda, double *d_grad,
                  void *stream);

/* Pass 1 that also keeps the path state at the start of every K-step segment
 * (K = the context's ckpt_every) in the context's checkpoint buffer, the
 * paper's step 2 keeping the results of step 1 in memory; outputs as
 * calibrate_forward.  Afterwards calibrate_vjp_stored can run pass 2 from
 * those checkpoints instead of re-running the forward sweep (a torch.autograd
 * forward/backward pair costs 2 F + R instead of 3 F + R).  Works in either
 * checkpoint mode (the buffer always exists). */
int calibrate_forward_store(cal_ctx *ctx, const double *d_theta, double *d_Ey, void *stream);

/* calibrate_vjp from the checkpoints of the last call on this context whose
 * sweep wrote them: calibrate_forward_store, calibrate_gradient or
 * calibrate_vjp (pass 2 re-running the forward sweep writes them too).
 * d_theta must hold the same values as in that call: the device compares them
 * bit for bit and sets CAL_FLAG_CKPT (see cal_status) if they differ.  Returns
 * CAL_EINVAL when no such call has completed on the context yet. */
int calibrate_vjp_stored(cal_ctx *ctx, const double *d_theta, const double *d_lambda, double *d_grad,
                         void *stream);

/* The paper's full algorithm (its steps 1-3, cost eq. 0711C): pass 1, then
 * r_i = E y_i - C_i and G = 1/2 sum r_i^2 in FP64 on the device, then pass 2
 * seeded with lambda_i = r_i / P per path, summed over paths.
 *   d_C[m]  : targets (FP64, device)
 *   d_Ey[m] : out, E y;  d_G[1] : out, G;  d_grad[M] : out, dG/dtheta */
int calibrate_gradient(cal_ctx *ctx, const double *d_theta, const double *d_C, double *d_Ey,
                       double *d_G, double *d_grad, void *stream);

/* Forward tangent mode over the same paths: d_Ey[m] and the Jacobian
 * d_J[m*M] (row-major, J[i*M + j] = dE y_i/dtheta_j).  Heston and BS (the
 * grid models and CAL_BS_EULER_S return CAL_EUNSUPPORTED).  By
 * the paper's eq. 0711A the same numbers follow from m reverse sweeps; with
 * M < m the tangent sweep is the cheaper route to the whole matrix. */
int calibrate_jacobian(cal_ctx *ctx, const double *d_theta, double *d_Ey, double *d_J, void *stream);

/* calibrate_jacobian for n_inst parameter vectors in one launch (the
 * surrogate's training labels): instance i reads d_theta[i*M .. i*M+M-1],
 * draws its normals with Philox counter word 2 = inst0 + i, and writes
 * d_Ey[i*m ..] and d_J[i*m*M ..].  1 <= n_inst <= the problem's max_batch. */
int calibrate_jacobian_batch(cal_ctx *ctx, const double *d_theta, int32_t n_inst, uint32_t inst0, double *d_Ey,
                             double *d_J, void *stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid allocation): calibrate_gradient for a
 * Black-Scholes or Heston problem without a context.  Every buffer beyond
 * the caller's arrays (instrument tables, block partials, the adjoint seeds,
 * the checkpoints) lives in one static device array of
 * CAL_STATIC_SCRATCH_BYTES per device, which the library holds from the first
 * call on that device until the process ends; the call allocates nothing.
 *   pb        host problem (as for cal_create; models CAL_BS and CAL_HESTON,
 *             else CAL_EUNSUPPORTED); its buffers must fit the array, else
 *             CAL_EINVAL with the bytes needed in cal_last_error(NULL)
 *             (2^20 Heston paths at 256 steps fit at ckpt_every 16)
 *   d_theta [M], d_C [m]   inputs; d_Ey [m], d_G [1], d_grad [M] outputs
 *             (FP64, caller's device memory, as for calibrate_gradient)
 *   d_status  caller's int32 on the device, set to this call's CAL_FLAG_* bits
 * Results are those of calibrate_gradient on a context made from the same
 * problem, bit for bit.  The call uploads the instrument tables (a few KB)
 * and synchronises `stream` once before queuing its kernels; it keeps the
 * array's contents from the last call (nothing in it is read before this
 * call writes it).  Calls that overlap on one device, on any streams or host
 * threads, race on the array: serialise them. */
#define CAL_STATIC_SCRATCH_BYTES ((size_t)160 << 20)
int calibrate_gradient_static(const cal_problem *pb, const double *d_theta, const double *d_C, double *d_Ey,
                              double *d_G, double *d_grad, int32_t *d_status, void *stream);

/* Synchronise `stream` and return the device status bits (CAL_FLAG_*)
 * accumulated since the previous cal_status call (then cleared), or a
 * negative error code. */
int cal_status(cal_ctx *ctx, void *stream);

/* Description of the last error on this context ("" if none). With ctx ==
 * NULL: the last error of cal_create / cal_validate in this thread. */
const char *cal_last_error(const cal_ctx *ctx);

/* Kernel timing with HIP events recorded on the launch stream around the
 * pass-1 kernel (which = 0), the pass-2 kernel (which = 1) and the tangent
 * kernel (which = 2).  cal_timing_enable(ctx, 1) starts recording (and clears
 * earlier records); cal_timing_read synchronises, returns the summed
 * milliseconds and the launch count of kernel `which`. */
int cal_timing_enable(cal_ctx *ctx, int32_t on);
int cal_timing_read(cal_ctx *ctx, int32_t which, double *ms_total, int64_t *launches);

/* Launch geometry the context uses (for reports): threads per block, blocks
 * per pass, checkpoint spacing and mode actually in effect. */
int cal_geometry(const cal_ctx *ctx, int32_t *threads, int64_t *blocks, int32_t *ckpt_every,
                 int32_t *ckpt_mode);

/* Test access to the random stream the kernels use (same device functions).
 *   cal_philox: d_out[4*i..4*i+3] = Philox4x32-10(d_ctr[4*i..4*i+3], key)
 *   cal_normals: for paths path0..path0+n_paths-1 and normals q0..q0+nq-1,
 *     d_out[(p - path0)*nq + (q - q0)] in the given precision (d_out is
 *     float* for CAL_FP32, double* for CAL_FP64). */
int cal_philox(const uint32_t *d_ctr, uint32_t key0, uint32_t key1, int64_t n, uint32_t *d_out,
               void *stream);
int cal_normals(int32_t precision, uint64_t seed, uint32_t inst, uint32_t path0, int64_t n_paths,
                uint32_t q0, int32_t nq, void *d_out, void *stream);

/*
 * Batches: many independent calibration problems of uneven size (m, P, N)
 * computed by one gradient step (the paper's steps 1-3 for every instance).
 * Persistent workgroups take (instance, 256-path block) items from a queue
 * ordered longest instance first, so uneven instances share the GPU; each
 * instance's results are bitwise those of its own cal_create context.
 * All instances share model (BS with log-Euler, or Heston) and precision; checkpoints are
 * stored by pass 1.
 *
 * Device arrays of a batch: d_theta [n_inst * M]; d_C and d_Ey concatenated
 * per instance (instance i at offsets[i] .. offsets[i+1], see calb_offsets,
 * in the instance's own instrument order); d_G [n_inst]; d_grad
 * [n_inst * M].
 */
typedef struct calb_ctx calb_ctx;

/* Validate every problem, allocate all workspace (checkpoints sized for the
 * densest spacing, 8 steps) and upload the tables. */
int calb_create(const cal_problem *problems, int32_t n_inst, calb_ctx **out);
int calb_destroy(calb_ctx *ctx);

/* instr_offsets[n_inst + 1]: start of each instance in d_C / d_Ey. */
int calb_offsets(const calb_ctx *ctx, int64_t *instr_offsets);

/* Checkpoint spacing (8, 16, 32), persistent workgroups per compute unit
 * (0 = as many as fit) and paths per lane (1, 2, 4) for every instance.
 * Synchronises the device and drops a captured graph. */
int calb_configure(calb_ctx *ctx, int32_t ckpt_every, int32_t workgroups_per_cu, int32_t paths_per_lane);
int calb_geometry(const calb_ctx *ctx, int32_t *ckpt_every, int32_t *grid, int32_t *n_items,
                  int32_t *paths_per_lane);

/* One gradient step for all instances, enqueued on `stream`. */
int calibrate_gradient_batch(calb_ctx *ctx, const double *d_theta, const double *d_C, double *d_Ey, double *d_G,
                             double *d_grad, void *stream);

/* Capture one gradient step bound to these arrays into a HIP graph (stream
 * must be a created stream, not the null stream); calb_replay launches it.
 * The step contains no memset nodes: the queue heads are reset by a kernel. */
int calb_capture(calb_ctx *ctx, const double *d_theta, const double *d_C, double *d_Ey, double *d_G,
                 double *d_grad, void *stream);
int calb_replay(calb_ctx *ctx, void *stream);

/* Synchronise `stream`, return and clear the batch's device status bits. */
int calb_status(calb_ctx *ctx, void *stream);
const char *calb_last_error(const calb_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* MCAAD_H */
