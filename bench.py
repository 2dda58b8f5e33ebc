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


def cpu_baseline(pb, theta, C, sample_paths, min_seconds):
    """The oracle, as it stands, on the first `sample_paths` paths, repeated
    until at least `min_seconds` have passed."""
    from oracle import build as ob
    ob.build(force=False)
    from oracle import oracle as O
    sub = pb.with_(n_paths=sample_paths)
    reps = 0
    t0 = time.perf_counter()
    while True:
        O.gradient(sub, theta, C)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    return {"value": reps * sample_paths * pb.n_steps / dt, "unit": "paths*steps/s", "cores": O.get_threads(),
            "kind": "oracle",
            "sample": f"full two-pass gradient (forward, reverse sweep, FP64 sums) on the first {sample_paths} "
                      f"of the {pb.n_paths} paths, {reps} time(s), {dt:.1f} s"}


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "mc_kernels_heston_2p20x256_hbm_counters.md")


def code_hash(path):
    """sha256 of a source with comments and whitespace removed."""
    import hashlib
    import re
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return hashlib.sha256(" ".join(text.split()).encode()).hexdigest()


def pass2_traffic(ckpt_every, ppl):
    """HBM bytes per pass-2 launch at this checkpoint spacing and paths per
    lane from the committed counter summary, or None when no figure was taken
    for them or any source of the kernel has changed since."""
    try:
        lines = open(TRAFFIC_PROFILE).read().splitlines()
    except OSError:
        return None
    value, ok = None, True
    for ln in lines:
        f = ln.split()
        if len(f) == 4 and f[0] == "k_pass2_bytes_per_launch" and f[1:3] == [f"K={ckpt_every}", f"ppl={ppl}"]:
            value = float(f[3])
        elif len(f) == 3 and f[0] == "code-sha256":
            ok = ok and os.path.exists(os.path.join(ROOT, f[1])) and code_hash(os.path.join(ROOT, f[1])) == f[2]
    return value if ok else None


GRID_VALU_PROFILE = os.path.join(ROOT, "profiles", "grid_kernels_valu_mix.md")


def counted_slots(model, kernel, ckpt_every):
    """VALU issue slots per path-step of a local-volatility or SLV kernel
    ('pass1' or 'pass2' at this spacing), counted with SQ counters and
    committed with the sources' hashes; None when not counted or stale."""
    try:
        lines = open(GRID_VALU_PROFILE).read().splitlines()
    except OSError:
        return None
    want = [model, kernel, f"K={ckpt_every}" if kernel == "pass2" else "K=-"]
    value, ok = None, True
    for ln in lines:
        f = ln.split()
        if len(f) == 5 and f[0] == "valu_slots_per_path_step" and f[1:4] == want:
            value = float(f[4])
        elif len(f) == 3 and f[0] == "code-sha256":
            ok = ok and os.path.exists(os.path.join(ROOT, f[1])) and code_hash(os.path.join(ROOT, f[1])) == f[2]
    return value if ok else None


def grid_roofline(model, kernel_name, ckpt_every, path_steps, ms_pass2):
    """Issue-slot roofline of a grid model's pass-2 kernel: counted slots per
    path-step x path-steps / the kernel's average duration, against the
    7.86e13 lane-slots/s of the FP32 VALU peak."""
    from paper_1901_04200_amd import roofline
    sl = counted_slots(model, "pass2", ckpt_every)
    achieved = sl * path_steps / (ms_pass2 * 1e-3) * 1e-12 if sl else None
    return {"bound": "alu", "kernel": kernel_name, "achieved": achieved, "peak": roofline.PEAK_SLOTS * 1e-12,
            "unit": "T VALU lane-slots/s", "frac": achieved / (roofline.PEAK_SLOTS * 1e-12) if achieved else None,
            "slots_per_path_step": sl, "work": "VALU issue slots per path-step counted with SQ counters"}


def time_ms(fn, reps):
    import torch
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def e2_sweep(n_paths, reps=5):
    """K_R/K_F over steps N x instruments m (128 steps per year): the paper
    reports its coefficients nearly constant as both grow."""
    import numpy as np
    import torch
    from paper_1901_04200_amd import capi, costmodel
    from paper_1901_04200_amd import workloads as W
    from paper_1901_04200_amd.mc import MonteCarloCalibration
    th = W.heston_draws(2, 10)[9]
    rows = []
    for N in (32, 64, 128, 256, 512):
        for ns, nm in ((8, 1), (8, 5), (24, 5), (40, 5)):
            t_max = N / 128.0
            st, kk = W.heston_instruments(ns, np.linspace(t_max / nm, t_max, nm), 128)
            pb = W.Problem(model=W.MODEL_HESTON, n_params=5, n_steps=N, n_paths=n_paths, t_max=t_max,
                           instr_step=st, instr_strike=kk)
            mc = MonteCarloCalibration(pb)
            C = torch.full((pb.n_instr,), 5.0, dtype=torch.float64, device="cuda")
            thd = torch.tensor(th, device="cuda")
            Ey = torch.empty(pb.n_instr, dtype=torch.float64, device="cuda")
            G = torch.empty(1, dtype=torch.float64, device="cuda")
            g = torch.empty(5, dtype=torch.float64, device="cuda")
            capi.calibrate_gradient(mc.ctx, thd, C, Ey, G, g)
            capi.cal_timing_enable(mc.ctx, True)
            for _ in range(reps):
                capi.calibrate_forward(mc.ctx, thd, Ey)
            tf = capi.cal_timing_read(mc.ctx, 0)
            capi.cal_timing_enable(mc.ctx, True)
            for _ in range(reps):
                capi.calibrate_gradient(mc.ctx, thd, C, Ey, G, g)
            t2 = capi.cal_timing_read(mc.ctx, 1)
            capi.cal_timing_enable(mc.ctx, False)
            mc.close()
            kr = costmodel.kr_over_kf(tf[0] / tf[1], t2[0] / t2[1])
            rows.append({"N": N, "m": pb.n_instr, "kr_over_kf": round(kr, 4)})
    return rows


def slv_leg(reps):
    """Heston stochastic local volatility (the paper's test model): 2^20
    paths x 256 steps, 5 Heston parameters + a 10 x 20 leverage grid, 200
    calls at the grid nodes; gradient and forward throughput, K_R/K_F."""
    import torch
    from paper_1901_04200_amd import capi, costmodel
    from paper_1901_04200_amd import workloads as W
    from paper_1901_04200_amd.mc import MonteCarloCalibration, pick_config
    pb, th0, tht, eps, _ = W.slv_problem()
    gen = MonteCarloCalibration(pb.with_(seed=2))
    C = torch.tensor(W.noisy_targets(gen.forward(tht).cpu().numpy(), eps), device="cuda")
    gen.close()
    (k, ppl), table = pick_config(pb, th0, C, ks=(8, 16), ppls=(1, 2))
    mc = MonteCarloCalibration(pb, ckpt_every=k, ckpt_mode="store", paths_per_lane=ppl)
    th = torch.tensor(th0, device="cuda")
    Ey = torch.empty(pb.n_instr, dtype=torch.float64, device="cuda")
    G = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty(pb.n_params, dtype=torch.float64, device="cuda")
    capi.calibrate_gradient(mc.ctx, th, C, Ey, G, g)
    capi.cal_timing_enable(mc.ctx, True)
    ms_grad = time_ms(lambda: capi.calibrate_gradient(mc.ctx, th, C, Ey, G, g), reps)
    p1 = capi.cal_timing_read(mc.ctx, 0)
    p2 = capi.cal_timing_read(mc.ctx, 1)
    capi.cal_timing_enable(mc.ctx, True)
    ms_fwd = time_ms(lambda: capi.calibrate_forward(mc.ctx, th, Ey), reps)
    f = capi.cal_timing_read(mc.ctx, 0)
    capi.cal_timing_enable(mc.ctx, False)
    status = mc.status()
    mc.close()
    ps = pb.n_paths * pb.n_steps
    t_f, t_2 = f[0] / f[1], p2[0] / p2[1]
    return {"workload": "Heston SLV: 2^20 paths x 256 steps, 5 Heston parameters + 10 x 20 leverage grid "
                        "(piecewise constant in t, linear in S), m = 200 calls, FP32 state, FP64 sums",
            "ckpt_every": k, "paths_per_lane": ppl,
            "tuning_ms": {f"k{kk}_ppl{pp}": t * 1e3 for (kk, pp), t in table}, "status": status,
            "paths_steps_per_s": ps / (ms_grad * 1e-3), "ms_per_step": ms_grad,
            "forward_paths_steps_per_s": ps / (ms_fwd * 1e-3), "ms_forward": ms_fwd,
            "ms_pass1_kernel": p1[0] / p1[1], "ms_pass2_kernel": t_2,
            "kr_over_kf": costmodel.kr_over_kf(t_f, t_2),
            "roofline": grid_roofline("slv", f"k_slv_pass2 (FP32, K={k})", k, ps, t_2)}


def lv_leg(reps):
    """Local volatility (bilinear 10 x 20 grid, M = 200, 200 calls at the grid
    nodes): 2^22 paths x 256 steps over 2 years, FP32 state, checkpoints every
    16 steps.  Times calibrate_gradient, the forward pass, and one step through
    the torch.autograd wrapper (forward keeping checkpoints, G in torch,
    backward = pass 2 from those checkpoints); then the gradient again with the
    spacing (8 or 16) and paths per lane (1 or 2, side by side) picked by
    timing."""
    import torch
    from paper_1901_04200_amd import autograd as AG
    from paper_1901_04200_amd import capi, costmodel
    from paper_1901_04200_amd import workloads as W
    from paper_1901_04200_amd.mc import MonteCarloCalibration
    pb, g0, gt, eps, _ = W.lv_problem()
    gen = MonteCarloCalibration(pb.with_(seed=2))
    C = torch.tensor(W.noisy_targets(gen.forward(gt).cpu().numpy(), eps), device="cuda")
    gen.close()
    k = 16
    mc = MonteCarloCalibration(pb, ckpt_every=k, ckpt_mode="store")
    th = torch.tensor(g0, device="cuda")
    Ey = torch.empty(pb.n_instr, dtype=torch.float64, device="cuda")
    G = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty(pb.n_params, dtype=torch.float64, device="cuda")
    capi.calibrate_gradient(mc.ctx, th, C, Ey, G, g)
    capi.cal_timing_enable(mc.ctx, True)
    ms_grad = time_ms(lambda: capi.calibrate_gradient(mc.ctx, th, C, Ey, G, g), reps)
    p1 = capi.cal_timing_read(mc.ctx, 0)
    p2 = capi.cal_timing_read(mc.ctx, 1)
    capi.cal_timing_enable(mc.ctx, True)
    ms_fwd = time_ms(lambda: capi.calibrate_forward(mc.ctx, th, Ey), reps)
    f = capi.cal_timing_read(mc.ctx, 0)
    capi.cal_timing_enable(mc.ctx, False)
    thg = torch.tensor(g0, device="cuda", requires_grad=True)

    def autograd_step():
        thg.grad = None
        Gt = 0.5 * torch.sum((AG.mc_prices(thg, mc) - C) ** 2)
        Gt.backward()

    autograd_step()
    ms_ag = time_ms(autograd_step, reps)
    agree = float(torch.max(torch.abs(thg.grad - g)) / torch.max(torch.abs(g)))
    status = mc.status()
    mc.close()
    # the same gradient with the checkpoint spacing and paths per lane picked by timing
    from paper_1901_04200_amd.mc import pick_config
    (kt, pplt), table = pick_config(pb, g0, C, ks=(8, 16), ppls=(1, 2))
    mct = MonteCarloCalibration(pb, ckpt_every=kt, ckpt_mode="store", paths_per_lane=pplt)
    capi.calibrate_gradient(mct.ctx, th, C, Ey, G, g)
    capi.cal_timing_enable(mct.ctx, True)
    ms_tuned = time_ms(lambda: capi.calibrate_gradient(mct.ctx, th, C, Ey, G, g), reps)
    p2t = capi.cal_timing_read(mct.ctx, 1)
    status |= mct.status()
    mct.close()
    ps = pb.n_paths * pb.n_steps
    t_f, t_2 = f[0] / f[1], p2[0] / p2[1]
    tuned = {"ckpt_every": kt, "paths_per_lane": pplt,
             "tuning_ms": {f"k{kk}_ppl{pp}": t * 1e3 for (kk, pp), t in table},
             "ms_per_step": ms_tuned, "paths_steps_per_s": ps / (ms_tuned * 1e-3),
             "ms_pass2_kernel": p2t[0] / p2t[1]}
    return {"workload": "local volatility: 2^22 paths x 256 steps over 2 years, bilinear 10 x 20 grid (M = 200), "
                        "m = 200 calls at the grid nodes, FP32 state, FP64 sums",
            "ckpt_every": k, "status": status,
            "paths_steps_per_s": ps / (ms_grad * 1e-3), "ms_per_step": ms_grad,
            "forward_paths_steps_per_s": ps / (ms_fwd * 1e-3), "ms_forward": ms_fwd,
            "ms_pass1_kernel": p1[0] / p1[1], "ms_pass2_kernel": t_2,
            "kr_over_kf": costmodel.kr_over_kf(t_f, t_2),
            "ms_autograd_step": ms_ag, "autograd_vs_gradient_rel_diff": agree,
            "roofline": grid_roofline("lv", f"k_lv_pass2 (FP32, K={k})", k, ps, t_2),
            "tuned": tuned}


def batched_leg(n_inst, reps):
    """The batched workload: n_inst Heston instances with m ~ U{8..120},
    P in {2^14, 2^16, 2^18}, N in {64, 128, 256}; one captured step per
    gradient, autotuned, against the same instances one context at a time."""
    import numpy as np
    import torch
    from paper_1901_04200_amd import capi
    from paper_1901_04200_amd import workloads as W
    from paper_1901_04200_amd.batch import BatchCalibration
    from paper_1901_04200_amd.mc import MonteCarloCalibration
    insts = W.batched_instances(n_inst)
    pbs = [pb for pb, *_ in insts]
    th0 = torch.tensor(np.array([t for _, t, _, _ in insts]), device="cuda")
    tht = torch.tensor(np.array([t for _, _, t, _ in insts]), device="cuda")
    B = BatchCalibration(pbs)
    zero = torch.zeros(int(B.offsets[-1]), dtype=torch.float64, device="cuda")
    Ey_t, _, _ = B.gradient(tht, zero)         # prices at the target draws
    eps = np.concatenate([e for _, _, _, e in insts])
    C = Ey_t.clone() * torch.tensor(1.0 + 1e-3 * eps, device="cuda")
    best, table = B.autotune(th0, C, reps=2)
    ms_graph = time_ms(B.replay, reps)
    flags = B.status()
    path_steps = sum(pb.n_paths * pb.n_steps for pb in pbs)
    Cs = B.split(C)
    mcs = [MonteCarloCalibration(pb, ckpt_every=best[0], paths_per_lane=best[2]) for pb in pbs]
    ths = [th0[i].contiguous() for i in range(n_inst)]
    Cs = [c.contiguous() for c in Cs]
    outs = [(torch.empty(pb.n_instr, dtype=torch.float64, device="cuda"),
             torch.empty(1, dtype=torch.float64, device="cuda"),
             torch.empty(5, dtype=torch.float64, device="cuda")) for pb in pbs]

    def sequential():
        for i, mc in enumerate(mcs):
            capi.calibrate_gradient(mc.ctx, ths[i], Cs[i], *outs[i])

    sequential()
    ms_seq = time_ms(sequential, max(1, reps // 2))
    for mc in mcs:
        mc.close()
    B.close()
    return {"instances": n_inst, "path_steps": path_steps, "status": flags,
            "autotuned": {"ckpt_every": best[0], "workgroups_per_cu": best[1], "paths_per_lane": best[2],
                          "candidates_ms": {f"k{c[0]}_w{c[1]}_ppl{c[2]}": round(t * 1e3, 3) for c, t in table}},
            "ms_graph_step": ms_graph, "paths_steps_per_s": path_steps / (ms_graph * 1e-3),
            "ms_one_context_at_a_time": ms_seq, "speedup": ms_seq / ms_graph,
            "roofline": batched_roofline(path_steps, ms_graph)}


def batched_roofline(path_steps, ms_step):
    """Issue-slot roofline of one captured batched step (pass 1 storing
    checkpoints and pass 2 from them over every instance): the Heston cost
    model's F + (F + R) slots per path-step over the whole step's time."""
    from paper_1901_04200_amd import roofline
    slots = roofline.slots(roofline.per_path_step("heston", "pass1")) + \
        roofline.slots(roofline.per_path_step("heston", "pass2"))
    achieved = slots * path_steps / (ms_step * 1e-3) * 1e-12
    return {"bound": "alu", "kernel": "k_batch_pass1 + k_batch_pass2 (whole step)", "achieved": achieved,
            "peak": roofline.PEAK_SLOTS * 1e-12, "unit": "T VALU lane-slots/s",
            "frac": achieved / (roofline.PEAK_SLOTS * 1e-12), "slots_per_path_step": slots}


def copy_probe(nbytes):
    """A plain device-to-device copy of nbytes (3 launches): what the HBM
    counters read for it scales their readings on the calibration kernels."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").uniform_()
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "launches": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--ckpt-mode", default="store", choices=["store", "rerun"])
    ap.add_argument("--ckpt-every", type=int, default=0, help="8, 16 or 32; 0 = tuned (8 or 16)")
    ap.add_argument("--paths-per-lane", type=int, default=0, help="1, 2 or 4; 0 = tuned (1 or 2)")
    ap.add_argument("--cpu-sample-paths", type=int, default=1 << 20)
    ap.add_argument("--cpu-min-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the extra legs")
    ap.add_argument("--extras", default="slv,lv,e2_sweep,batched,surrogate_vs_mc",
                    help="comma-separated extra legs to run")
    ap.add_argument("--sweep-paths", type=int, default=1 << 20)
    ap.add_argument("--batch-instances", type=int, default=256)
    ap.add_argument("--surrogate-draws", type=int, default=1 << 16)
    ap.add_argument("--surrogate-paths", type=int, default=1 << 16)
    ap.add_argument("--surrogate-epochs", type=int, default=150)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain copy of BYTES (HBM counter scaling) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding of "
              f"paths over GPUs is a design note, not built.", file=sys.stderr)
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
    ckpt_every, ppl, tune_table = args.ckpt_every, args.paths_per_lane, None
    if ckpt_every == 0 or ppl == 0:
        from paper_1901_04200_amd.mc import pick_config
        (ckpt_every, ppl), tune_table = pick_config(pb, th0, C, precision=args.precision,
                                                    ks=(8, 16) if ckpt_every == 0 else (ckpt_every,),
                                                    ppls=(1, 2) if ppl == 0 else (ppl,))
        print(f"bench: checkpoint spacing {ckpt_every}, {ppl} path(s) per lane ({tune_table})", file=sys.stderr,
              flush=True)
    mc = MonteCarloCalibration(pb, precision=args.precision, ckpt_every=ckpt_every, ckpt_mode=args.ckpt_mode,
                               paths_per_lane=ppl)
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
            "paths_per_lane": ppl,
            "tuning_ms": None if tune_table is None else {f"k{k}_ppl{q}": t * 1e3 for (k, q), t in tune_table},
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
            "traffic": pass2_traffic(geo["ckpt_every"], ppl),
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "traffic_algorithmic": roofline.pass2_bytes(pb.n_paths, geo["ckpt_every"], geo["blocks"], pb.n_instr,
                                                        pb.n_steps),
        },
    }
    mc.close()
    if not args.no_extras:
        legs = (("slv", lambda: slv_leg(max(5, args.steps // 2))),
                ("lv", lambda: lv_leg(max(5, args.steps // 2))),
                ("e2_sweep", lambda: e2_sweep(args.sweep_paths)),
                ("batched", lambda: batched_leg(args.batch_instances, max(3, args.steps // 4))),
                ("surrogate_vs_mc", lambda: surrogate_leg(args)))
        chosen = set(args.extras.split(","))
        for name, fn in legs:
            if name not in chosen:
                continue
            print(f"bench: {name} ...", file=sys.stderr, flush=True)
            try:
                out[name] = fn()
            except Exception as exc:   # a failing extra leg must not hide the headline numbers
                out[name] = {"error": f"{type(exc).__name__}: {exc}"}
            print(f"bench: {name} done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("bench: oracle CPU baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(pb, th0, C.cpu().numpy(), args.cpu_sample_paths,
                                           args.cpu_min_seconds)
    print(json.dumps(out), flush=True)


def surrogate_leg(args):
    from paper_1901_04200_amd import surrogate_study
    res = surrogate_study.run(n_train=args.surrogate_draws, train_paths=args.surrogate_paths,
                              epochs=args.surrogate_epochs,
                              log=lambda s: print("bench: " + s, file=sys.stderr, flush=True))
    st = res["step_seconds"]
    gain = res.get("gain") or {}
    gain = {k: v for k, v in gain.items() if k != "per_instance"}
    details = {k: v for k, v in res.items() if k != "gain"}
    return {"grad_rel_err_surrogate": res["surrogate_grad_rel_err"]["median"], "p_star_paths": res["p_star"],
            "us_surrogate_step": st["surrogate"] * 1e6, "us_mc_step_at_p_star": st["mc_at_p_star"] * 1e6,
            "mc_over_surrogate": st["mc_over_surrogate"], "gain_test": gain, "details": details}


if __name__ == "__main__":
    main()
