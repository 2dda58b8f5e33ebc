"""Algorithmic work per path-step of the Monte Carlo kernels and MI355X peaks.

The path is bound by VALU issue (integer multiplies, transcendentals and
FP32 arithmetic in registers; HBM traffic is only the checkpoints).  Work is
counted from the algorithm, not from compiled code, in VALU issue slots.

Peak: the published FP32 vector rate, 157.3 TFLOP/s = 256 CU x 128 FMA
lanes per clock x 2 flops x 2.4 GHz, i.e. 128 lane-slots per CU per clock,
7.86e13 lane-slots/s.  A throughput probe on gfx950 (independent chains,
4096 x 256 threads) measured, in lane-ops per CU per clock: FP32 mul 104,
FP32 fma 93, xor/shift 103, FP64 fma 52, v_mad_u64_u32 ~32, transcendentals
(v_log/v_sqrt/v_sin/v_rcp/v_exp_f32) 29-30.  Issue costs in slots:
  plain 32-bit VALU op (add, mul, fma, xor3, shift, cvt, cmp, select): 1
  32x32->64 integer multiply (v_mad_u64_u32):                           COST_MAD64 = 4
  transcendental (log2, sqrt, sin, cos, rcp, exp2):                     COST_TRANS = 4

Per path-step, Heston (d = 2 normals per step), FP32 state, counting the
work that differs per lane (the uniform parts of Philox's first rounds run on
the scalar unit and are not counted):
  Philox4x32-10, half a call: counter (call, path, inst, 0) has one varying
    word, so 16 of the 20 wide multiplies and 18 of the 20 three-way xors of
    a call vary per lane                   = 8 mad64 + 9 valu
  two uniforms (align-bit, subtract)       = 4 valu
  Box-Muller pair, scaled by sqrt(h)       = 3 valu + 4 trans
  Euler step on (x~, v): v+, sqrt, w', xi w', x~ (2 fma), v (3)
                                           = 9 valu + 1 trans
  forward step F                           = 8 mad64 + 25 valu + 5 trans  (77 slots)
  reverse step R: v+ = s^2 (1: pass 2 keeps s, not v+, per step of a
    segment), sbar (3), s' (rcp, 1), v+bar (2), the four segment sums (6),
    adjoint of v (3)                       = 17 valu + 1 trans            (21 slots)
  pass 1 (F)                               = F
  pass 2 from stored checkpoints (F + R)   = 8 mad64 + 42 valu + 6 trans  (98 slots)
FP32 flops per path-step, counting every FP32 arithmetic result: add, mul
1, FMA 2, transcendental (log2, sqrt, sin, cos, rcp, exp2) 1:
  F: uniforms 2, Box-Muller 3 + 4 trans, Euler 13 + 1 trans      = 23
  R: 23 + 1 (rcp)                                                  = 24
  pass 2 from checkpoints (F + R)                                  = 47
The flop fraction of the FP32 peak that this work can reach is bounded by
the issue slots it needs: 157.3 TFLOP/s counts two flops per lane-slot
(packed or dual-issued FMA), so a kernel issuing one FP32 op per slot and
nothing else reaches 0.5 of it; pass 2 spends 98 slots on 47 flops, so
its ceiling at full issue is 47 / (2 x 98) = 0.24 of 157.3 TFLOP/s.
"""

CUS = 256
LANE_SLOTS_PER_CU_CLOCK = 128   # 157.3 TFLOP/s / (2 flops x 256 CU x 2.4 GHz)
CLOCK_HZ = 2.4e9
PEAK_SLOTS = CUS * LANE_SLOTS_PER_CU_CLOCK * CLOCK_HZ   # 7.86e13 lane-slots/s
PEAK_FP32_TFLOPS = 157.3        # published FP32 vector peak (FMA = 2 flops)

COST_MAD64 = 4.0
COST_TRANS = 4.0

HESTON_F = {"mad64": 8, "valu": 25, "trans": 5, "flops": 23}
HESTON_R = {"mad64": 0, "valu": 17, "trans": 1, "flops": 24}
BS_F = {"mad64": 4, "valu": 10, "trans": 2, "flops": 7}     # quarter call + one normal per step
BS_R = {"mad64": 0, "valu": 3, "trans": 0, "flops": 3}


def flop_ceiling(op: dict) -> float:
    """Largest fraction of the FP32 peak (two flops per lane-slot) that work
    `op` reaches when every slot issues."""
    return op["flops"] / (2.0 * slots(op))


def slots(op: dict) -> float:
    return op["valu"] + COST_MAD64 * op["mad64"] + COST_TRANS * op["trans"]


def add(a: dict, b: dict) -> dict:
    return {k: a[k] + b[k] for k in a}


def per_path_step(model: str, kernel: str) -> dict:
    """Algorithmic work per path-step of 'pass1' or 'pass2' (from stored
    checkpoints) or 'pass2_rerun' (forward re-run + recompute + reverse)."""
    F, R = (HESTON_F, HESTON_R) if model == "heston" else (BS_F, BS_R)
    if kernel == "pass1":
        return dict(F)
    if kernel == "pass2":
        return add(F, R)
    if kernel == "pass2_rerun":
        return add(add(F, F), R)
    raise ValueError(kernel)


def pass2_bytes(n_paths: int, ckpt_every: int, n_blocks: int, n_instr: int, n_steps: int,
                n_state: int = 2, n_params: int = 5, real_bytes: int = 4) -> int:
    """Algorithmic HBM bytes of one pass-2 launch from stored checkpoints:
    every path's state at the start of each K-step segment is read once, one
    FP64 partial per workgroup and parameter is written, and the m seeds
    lambda_i D_i / P are read."""
    n_seg = -(-n_steps // ckpt_every)
    return n_seg * n_state * n_paths * real_bytes + n_blocks * n_params * 8 + n_instr * real_bytes


def training_step_bytes(batch: int, hidden: int, n_in: int, n_out: int, n_params: int) -> int:
    """Algorithmic HBM bytes of one surrogate training step on the fused
    kernels (network n_in -> H -> H -> H -> n_out, output units padded to
    64): every tensor of the step written once and read once by each of its
    consumers, with R = (n_in + 1) batch activation rows.
      inputs: parameter rows, price and Jacobian labels, Jacobian weights and
        batch indices                                  B (n_in + n_out (1 + n_in) + 2) 4
      layer 1: bf16 activations A1 and FP32 primal pre-activations z1 written
      hidden layers 2, 3, forward: A_{l-1} read; A_l, z_l and the bf16
        tangent pre-activations u_l written
      output layer: A3 read, the bf16 output adjoint G4 written
      weight gradients (three products): both operands read
      input adjoints of layers 3, 2 (fused with the activation adjoint): the
        adjoint above, z_l and u_l read, bf16 Zbar_l written
      layer 1's adjoint: Zbar2 and z1 read
      Adam: parameters, both moments and the gradient read, three written,
        bf16 copies of the three product weights written twice
    Weights read by the products and the per-workgroup partials are left out
    (small next to the activations at B = 4096)."""
    B, H = batch, hidden
    R = (n_in + 1) * B
    act = R * H * 2               # one bf16 activation or adjoint matrix
    z = B * H * 4                 # FP32 primal pre-activations
    u = n_in * B * H * 2          # bf16 tangent pre-activations
    g4 = R * 64 * 2
    inputs = B * (n_in + n_out * (1 + n_in) + 2) * 4
    fwd = (act + z) + 2 * (act + act + z + u) + (act + g4)
    wgrad = (act + g4) + 2 * (act + act)
    bwd = (g4 + z + u + act) + (act + z + u + act) + (act + z)
    adam = n_params * 4 * 7 + 3 * 2 * 2 * H * H
    return inputs + fwd + wgrad + bwd + adam
