"""Benchmark: the two-pass Monte Carlo adjoint gradient on one MI355X.

One step = one calibrate_gradient call on the Heston calibration problem
(2^20 paths x 256 Euler steps, m = 40 calls, M = 5 parameters, FP32 path
state, FP64 sums): pass 1 (forward sweep, E y), residual and G, pass 2
(recompute from checkpoints + reverse sweep), FP64 gradient reduction.
Inputs (theta, targets) are resident in HBM before the timed region.

Prints one JSON line:
  value          paths*steps/s of the gradient (P*N / time per step)
  kr_over_kf     (T_pass2 - T_F)/T_F with T_F the forward pass alone
  roofline       VALU-issue roofline of the dominant kernel (pass 2)
  cpu_baseline   the FP64 CPU oracle on a bounded sample of the same workload
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "paths·steps/s for ∇G (F_v+R_v), K_R/K_F, % FP32 VALU peak; surrogate vs MC step"


def cpu_baseline(pb, theta, C, sample_paths):
    """The oracle, as it stands, on the first `sample_paths` paths."""
    from oracle import build as ob
    ob.build(force=False)
    from oracle import oracle as O
    sub = pb.with_(n_paths=sample_paths)
    t0 = time.perf_counter()
    O.gradient(sub, theta, C)
    dt = time.perf_counter() - t0
    return {"value": sample_paths * pb.n_steps / dt, "unit": "paths*steps/s", "cores": O.get_threads(),
            "kind": "oracle",
            "sample": f"full two-pass gradient (forward, reverse sweep, FP64 sums) on the first {sample_paths} "
                      f"of the {pb.n_paths} paths, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--ckpt-mode", default="store", choices=["store", "rerun"])
    ap.add_argument("--ckpt-every", type=int, default=16)
    ap.add_argument("--cpu-sample-paths", type=int, default=1 << 20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding of "
              f"paths is described in DESIGN.md, not run.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1901_04200_amd import capi, costmodel, roofline
    from paper_1901_04200_amd import workloads as W
    from paper_1901_04200_amd.mc import MonteCarloCalibration

    torch.cuda.set_device(0)
    pb, th0, tht, eps = W.heston_problem()
    P, N = pb.n_paths, pb.n_steps
    # targets: model prices at the target draw (Philox seed 2) plus 0.1 % noise
    gen = MonteCarloCalibration(pb.with_(seed=2), precision=args.precision)
    C = torch.tensor(W.noisy_targets(gen.forward(tht).cpu().numpy(), eps), dtype=torch.float64, device="cuda")
    gen.close()
    mc = MonteCarloCalibration(pb, precision=args.precision, ckpt_every=args.ckpt_every, ckpt_mode=args.ckpt_mode)
    theta = torch.tensor(th0, dtype=torch.float64, device="cuda")
    Ey = torch.empty(pb.n_instr, dtype=torch.float64, device="cuda")
    G = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty(5, dtype=torch.float64, device="cuda")
    ctx = mc.ctx

    def grad_step():
        capi.calibrate_gradient(ctx, theta, C, Ey, G, g)

    def fwd_step():
        capi.calibrate_forward(ctx, theta, Ey)

    for _ in range(args.warmup):
        grad_step()
        fwd_step()
    torch.cuda.synchronize()
    print(f"bench: warmup done ({args.warmup} gradient + forward calls)", file=sys.stderr, flush=True)

    # --- timed region: K gradient steps --------------------------------------
    capi.cal_timing_enable(ctx, True)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        grad_step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = ev0.elapsed_time(ev1) / args.steps
    p1_ms, p1_n = capi.cal_timing_read(ctx, 0)
    p2_ms, p2_n = capi.cal_timing_read(ctx, 1)
    assert mc.status() == 0, "device status flags set"
    print(f"bench: {args.steps} gradient steps, {ms_step:.3f} ms/step (wall {wall:.3f} s)", file=sys.stderr,
          flush=True)

    # --- forward pass alone (T_F) ----------------------------------------------
    capi.cal_timing_enable(ctx, True)
    ev0.record()
    for _ in range(args.steps):
        fwd_step()
    ev1.record()
    torch.cuda.synchronize()
    ms_fwd = ev0.elapsed_time(ev1) / args.steps
    f_ms, f_n = capi.cal_timing_read(ctx, 0)
    capi.cal_timing_enable(ctx, False)

    pass1_avg = p1_ms / max(p1_n, 1)
    pass2_avg = p2_ms / max(p2_n, 1)
    t_f = f_ms / max(f_n, 1)
    kr_kf = costmodel.kr_over_kf(t_f, pass2_avg)
    path_steps = P * N
    model = "heston"
    kern = "pass2" if args.ckpt_mode == "store" else "pass2_rerun"
    w2 = roofline.per_path_step(model, kern)
    slots2 = roofline.slots(w2) * path_steps
    achieved = slots2 / (pass2_avg * 1e-3)
    flops_all = (roofline.per_path_step(model, "pass1")["flops"] + w2["flops"]) * path_steps
    fp32_tflops = flops_all / (ms_step * 1e-3) / 1e12
    geo = mc.geometry()

    out = {
        "metric": METRIC,
        "value": path_steps / (ms_step * 1e-3),
        "unit": "paths*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": "Heston calibration gradient: 2^20 paths x 256 Euler steps, m=40 calls "
                        "(8 strikes x 5 maturities), M=5, full truncation, FP32 state, FP64 sums",
            "n_paths": P, "n_steps": N, "n_instr": pb.n_instr, "n_params": 5,
            "ckpt_every": geo["ckpt_every"], "ckpt_mode": args.ckpt_mode,
            "threads_per_block": geo["threads"], "blocks": geo["blocks"],
        },
        "forward_value": path_steps / (ms_fwd * 1e-3),
        "ms_forward": ms_fwd,
        "ms_pass1_kernel": pass1_avg,
        "ms_pass2_kernel": pass2_avg,
        "kr_over_kf": kr_kf,
        "cost_g_over_cost_f": costmodel.gradient_over_forward(kr_kf),
        "fp32_tflops": fp32_tflops,
        "fp32_valu_peak_frac": fp32_tflops / roofline.PEAK_FP32_TFLOPS,
        "surrogate_vs_mc": None,
        "roofline": {
            "bound": "alu",
            "kernel": "k_pass2 (Heston, FP32, K=%d, %s)" % (geo["ckpt_every"], args.ckpt_mode),
            "achieved": achieved / 1e12,
            "peak": roofline.PEAK_SLOTS / 1e12,
            "unit": "T VALU lane-slots/s",
            "frac": achieved / roofline.PEAK_SLOTS,
            "traffic": None,
        },
    }
    if not args.no_cpu_baseline:
        print("bench: oracle CPU baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(pb, th0, C.cpu().numpy(), args.cpu_sample_paths)
    mc.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
