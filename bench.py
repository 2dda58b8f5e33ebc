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


def host_cpu_model():
    """The host CPU's model name: lscpu's, else /proc/cpuinfo's (with the
    number of sockets and cores per socket lscpu reports, when it does)."""
    import subprocess
    name, extra = None, []
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            k, _, v = ln.partition(":")
            k, v = k.strip(), v.strip()
            if k == "Model name" and not name:
                name = v
            elif k in ("Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU max MHz"):
                extra.append(f"{k} {v}")
    except (OSError, subprocess.SubprocessError):
        pass
    if not name:
        try:
            for ln in open("/proc/cpuinfo"):
                if ln.startswith("model name"):
                    name = ln.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return name if not extra else f"{name} ({', '.join(extra)})"


def oracle_leg(pb, theta, C, got, sample_paths_1t, min_seconds_1t, t_forward_gpu_ms):
    """The FP64 oracle on the timed input: parity of the GPU result `got` =
    (Ey, G, grad) with the oracle's two-pass gradient on all P paths (that
    run, on every host thread, is also the multi-threaded CPU baseline), the
    one-path share of every gradient component, and the oracle on one thread
    on the first `sample_paths_1t` paths (forward alone and the gradient),
    repeated for at least `min_seconds_1t` each: the analogue of the paper's
    Cost(F), from which T_F,GPU / (P Cost_F,1 thread) is the K_F/c proxy."""
    from oracle import build as ob
    ob.build(force=False)
    from oracle import oracle as O
    from oracle import parity as PY
    threads = O.get_threads()
    t0 = time.perf_counter()
    Eo, Go, go = O.gradient(pb, theta, C)
    t_all = time.perf_counter() - t0
    shares = PY.gradient_shares(O, pb, theta, C, Eo)
    Ey, G, g = got
    par = {"theta": [float(v) for v in theta], "paths": pb.n_paths,
           "ey_err": PY.ey_err(Ey, Eo), "grad_err": PY.grad_err(g, go), "grad_err_inf": PY.grad_err_inf(g, go),
           "G_rel_err": abs(G - Go) / max(abs(Go), 1e-300),
           "one_path_share": [float(v) for v in shares],
           "tolerance": {"ey": PY.EY_TOL_FP32, "grad": PY.GRAD_TOL_FP32, "share_gate": PY.SHARE_GATE}}
    par["within_tolerance"] = par["ey_err"] <= PY.EY_TOL_FP32 and par["grad_err"] <= PY.GRAD_TOL_FP32
    par["well_conditioned"] = bool(max(shares) <= PY.SHARE_GATE)
    sub = pb.with_(n_paths=sample_paths_1t)
    O.set_threads(1)
    try:
        rates = {}
        for name, fn in (("forward", lambda: O.forward(sub, theta)), ("gradient", lambda: O.gradient(sub, theta, C))):
            reps, t0 = 0, time.perf_counter()
            while True:
                fn()
                reps += 1
                dt = time.perf_counter() - t0
                if dt >= min_seconds_1t:
                    break
            rates[name] = (reps * sample_paths_1t * pb.n_steps / dt, reps, dt)
    finally:
        O.set_threads(threads)
    cost_f_path_1t = pb.n_steps / rates["forward"][0]   # seconds per path of F, one thread
    base = {"value": pb.n_paths * pb.n_steps / t_all, "unit": "paths*steps/s", "cores": threads,
            "kind": "oracle", "cpu_model": host_cpu_model(),
            "sample": f"full two-pass gradient (forward, reverse sweep, FP64 sums) on all {pb.n_paths} paths of "
                      f"the timed input, once, {t_all:.2f} s on {threads} threads",
            "single_thread": {
                "forward_paths_steps_per_s": rates["forward"][0], "gradient_paths_steps_per_s": rates["gradient"][0],
                "sample": f"first {sample_paths_1t} paths, forward {rates['forward'][1]}x in "
                          f"{rates['forward'][2]:.1f} s, gradient {rates['gradient'][1]}x in "
                          f"{rates['gradient'][2]:.1f} s"},
            "kf_over_c_proxy": (t_forward_gpu_ms * 1e-3) / (pb.n_paths * cost_f_path_1t),
            "kf_over_c_proxy_note": "T_F,GPU / (P Cost_F,oracle 1 thread); the oracle is plain scalar FP64, "
                                    "not an optimised F, so this is a proxy for the paper's K_F/c"}
    return par, base


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


ISSUE_PROFILE = os.path.join(ROOT, "profiles", "mc_kernels_heston_2p20x256_valu_mix.md")


def valu_issue_utilisation(ckpt_every):
    """Measured VALU issue utilisation of the Heston pass-2 kernel at this
    spacing: issue slots counted with SQ counters (SQ_INSTS_VALU, with the
    64-bit integer and transcendental instructions at four slots) over the
    kernel's traced duration x 7.86e13 lane-slots/s, from the committed
    counter summary; None when not taken or stale."""
    try:
        lines = open(ISSUE_PROFILE).read().splitlines()
    except OSError:
        return None
    value, ok = None, True
    for ln in lines:
        f = ln.split()
        if len(f) == 4 and f[0] == "valu_issue_utilisation" and f[1:3] == ["k_pass2", f"K={ckpt_every}"]:
            value = float(f[3])
        elif len(f) == 3 and f[0] == "code-sha256":
            ok = ok and os.path.exists(os.path.join(ROOT, f[1])) and code_hash(os.path.join(ROOT, f[1])) == f[2]
    return value if ok else None


FLOPS_PROFILE = os.path.join(ROOT, "profiles", "mc_kernels_heston_2p20x256_fp32_flops.md")


def counted_flops(ckpt_every, path_steps, ms_pass2):
    """FP32 flops of the Heston pass-2 kernel counted with SQ counters (adds,
    multiplies and transcendentals one each, FMAs two, over 64 lanes) per
    path-step, from the committed counter summary, and what they give over
    the kernel's average duration against 157.3 TFLOP/s (the packed-FP32
    peak) and 78.6 TFLOP/s (one FP32 operation per lane and cycle); None
    when not taken or stale."""
    from paper_1901_04200_amd import roofline
    try:
        lines = open(FLOPS_PROFILE).read().splitlines()
    except OSError:
        return None
    value, ok = None, True
    for ln in lines:
        f = ln.split()
        if len(f) == 4 and f[0] == "fp32_flops_per_path_step" and f[1:3] == ["k_pass2", f"K={ckpt_every}"]:
            value = float(f[3])
        elif len(f) == 3 and f[0] == "code-sha256":
            ok = ok and os.path.exists(os.path.join(ROOT, f[1])) and code_hash(os.path.join(ROOT, f[1])) == f[2]
    if value is None or not ok:
        return None
    tf = value * path_steps / (ms_pass2 * 1e-3) * 1e-12
    return {"flops_per_path_step": value, "achieved_tflops": tf, "frac": tf / roofline.PEAK_FP32_TFLOPS,
            "frac_nonpacked": tf / (roofline.PEAK_FP32_TFLOPS / 2)}


def device_info():
    """Name, architecture and compute units of device 0, and the clock the
    runtime reports for it."""
    import torch
    pr = torch.cuda.get_device_properties(0)
    info = {"name": pr.name, "arch": getattr(pr, "gcnArchName", None), "compute_units": pr.multi_processor_count}
    try:
        import ctypes
        hip = ctypes.CDLL("libamdhip64.so")
        v = ctypes.c_int(0)
        if hip.hipDeviceGetAttribute(ctypes.byref(v), 5, 0) == 0:   # hipDeviceAttributeClockRate (kHz)
            info["clock_khz"] = v.value
    except OSError:
        pass
    return info


GRID_VALU_PROFILE = os.path.join(ROOT, "profiles", "grid_kernels_valu_mix.md")


BATCH_VALU_PROFILE = os.path.join(ROOT, "profiles", "batch_kernels_heston_valu_mix.md")


def counted_slots(model, kernel, ckpt_every, ppl=1, profile=GRID_VALU_PROFILE):
    """VALU issue slots per path-step of a local-volatility or SLV kernel
    ('pass1' or 'pass2' at this spacing) with ppl paths per lane, counted with
    SQ counters and committed with the sources' hashes; None when not counted
    or stale."""
    try:
        lines = open(profile).read().splitlines()
    except OSError:
        return None
    want = [model, kernel, f"K={ckpt_every}" if kernel == "pass2" else "K=-", f"ppl={ppl}"]
    value, ok = None, True
    for ln in lines:
        f = ln.split()
        if len(f) == 6 and f[0] == "valu_slots_per_path_step" and f[1:5] == want:
            value = float(f[5])
        elif len(f) == 3 and f[0] == "code-sha256":
            ok = ok and os.path.exists(os.path.join(ROOT, f[1])) and code_hash(os.path.join(ROOT, f[1])) == f[2]
    return value if ok else None


def grid_roofline(model, kernel_name, ckpt_every, path_steps, ms_pass2, ppl=1):
    """Issue-slot roofline of a grid model's pass-2 kernel: counted slots per
    path-step x path-steps / the kernel's average duration, against the
    7.86e13 lane-slots/s of the FP32 VALU peak."""
    from paper_1901_04200_amd import roofline
    sl = counted_slots(model, "pass2", ckpt_every, ppl)
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


def bs_schemes_leg(reps):
    """Black-Scholes at 2^20 paths x 256 steps (four calls at T = 1, FP32
    state, K = 16) with the paper's Euler scheme on S as the SDE is written
    and with the log-Euler scheme, timed side by side: gradient step,
    forward pass and K_R/K_F of each."""
    import torch
    from paper_1901_04200_amd import capi, costmodel
    from paper_1901_04200_amd import workloads as W
    from paper_1901_04200_amd.mc import MonteCarloCalibration
    out = {"workload": "Black-Scholes: 2^20 paths x 256 steps, 4 calls (K = 80..110, T = 1), FP32 state, "
                       "FP64 sums, K = 16"}
    for name, euler_on_s in (("euler_on_s", True), ("log_euler", False)):
        pb, th, C = W.bs_problem(n_paths=1 << 20, n_steps=256, euler_on_s=euler_on_s)
        mc = MonteCarloCalibration(pb, ckpt_every=16)
        thd = torch.tensor(th, device="cuda")
        Cd = torch.tensor(C, device="cuda")
        Ey = torch.empty(pb.n_instr, dtype=torch.float64, device="cuda")
        G = torch.empty(1, dtype=torch.float64, device="cuda")
        g = torch.empty(1, dtype=torch.float64, device="cuda")
        capi.calibrate_gradient(mc.ctx, thd, Cd, Ey, G, g)
        capi.cal_timing_enable(mc.ctx, True)
        ms = time_ms(lambda: capi.calibrate_gradient(mc.ctx, thd, Cd, Ey, G, g), reps)
        p2 = capi.cal_timing_read(mc.ctx, 1)
        capi.cal_timing_enable(mc.ctx, True)
        ms_f = time_ms(lambda: capi.calibrate_forward(mc.ctx, thd, Ey), reps)
        f = capi.cal_timing_read(mc.ctx, 0)
        capi.cal_timing_enable(mc.ctx, False)
        status = mc.status()
        mc.close()
        t2, tf = p2[0] / p2[1], f[0] / f[1]
        out[name] = {"ms_per_step": ms, "paths_steps_per_s": pb.n_paths * pb.n_steps / (ms * 1e-3),
                     "ms_forward": ms_f, "ms_pass2_kernel": t2, "ms_forward_kernel": tf,
                     "kr_over_kf": costmodel.kr_over_kf(tf, t2), "status": status}
    return out


def slv_calibration(mc, pb, th0, tht):
    """The paper's test: the Heston SLV model calibrated by gradient descent
    (projected L-BFGS on the two-pass gradient) from the first parameter draw
    to prices at the second on the same streams, to G <= 1e-3 G(theta0)."""
    import numpy as np
    from paper_1901_04200_amd import calibrate as K
    from paper_1901_04200_amd import workloads as W
    M = pb.n_params
    lo = np.concatenate([W.HESTON_LO, np.full(M - 5, 0.3)])
    hi = np.concatenate([W.HESTON_HI, np.full(M - 5, 2.0)])
    C = mc.forward(tht).cpu().numpy()
    obj = K.MonteCarloObjective(mc, C)
    G0 = obj.value_and_grad(th0)[0]
    t0 = time.perf_counter()
    r = K.calibrate(obj.value_and_grad, obj.value, th0, lo, hi, g_tol=1e-3 * G0, feller=True, max_iter=300)
    wall = time.perf_counter() - t0
    return {"target": "G <= 1e-3 G(theta0), targets priced at a second parameter draw on the same streams",
            "G0": G0, "G": r.G, "status": r.status, "gradients": r.n_grad, "values": r.n_value,
            "seconds": wall, "ms_per_gradient_call": wall / max(r.n_grad + r.n_value, 1) * 1e3}


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
    calib = slv_calibration(mc, pb, th0, tht)
    status = mc.status()
    mc.close()
    ps = pb.n_paths * pb.n_steps
    t_f, t_2 = f[0] / f[1], p2[0] / p2[1]
    return {"calibration": calib,
            "workload": "Heston SLV: 2^20 paths x 256 steps, 5 Heston parameters + 10 x 20 leverage grid "
                        "(piecewise constant in t, linear in S), m = 200 calls, FP32 state, FP64 sums",
            "ckpt_every": k, "paths_per_lane": ppl,
            "tuning_ms": {f"k{kk}_ppl{pp}": t * 1e3 for (kk, pp), t in table}, "status": status,
            "paths_steps_per_s": ps / (ms_grad * 1e-3), "ms_per_step": ms_grad,
            "forward_paths_steps_per_s": ps / (ms_fwd * 1e-3), "ms_forward": ms_fwd,
            "ms_pass1_kernel": p1[0] / p1[1], "ms_pass2_kernel": t_2,
            "kr_over_kf": costmodel.kr_over_kf(t_f, t_2),
            "roofline": grid_roofline("slv", f"k_slv_pass2 (FP32, K={k}, {ppl} path(s) per lane)", k, ps, t_2,
                                      ppl)}


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
    capi.cal_timing_enable(mct.ctx, True)
    time_ms(lambda: capi.calibrate_forward(mct.ctx, th, Ey), reps)
    ft = capi.cal_timing_read(mct.ctx, 0)
    capi.cal_timing_enable(mct.ctx, False)
    status |= mct.status()
    mct.close()
    ps = pb.n_paths * pb.n_steps
    t_f, t_2 = f[0] / f[1], p2[0] / p2[1]
    tuned = {"ckpt_every": kt, "paths_per_lane": pplt,
             "tuning_ms": {f"k{kk}_ppl{pp}": t * 1e3 for (kk, pp), t in table},
             "ms_per_step": ms_tuned, "paths_steps_per_s": ps / (ms_tuned * 1e-3),
             "ms_pass2_kernel": p2t[0] / p2t[1], "ms_forward_kernel": ft[0] / ft[1],
             "kr_over_kf": costmodel.kr_over_kf(ft[0] / ft[1], p2t[0] / p2t[1]),
             "roofline": grid_roofline("lv", f"k_lv_pass2 (FP32, K={kt}, {pplt} path(s) per lane)", kt, ps,
                                       p2t[0] / p2t[1], pplt)}
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
            "roofline": batched_roofline(path_steps, ms_graph, best[0])}


def batched_roofline(path_steps, ms_step, ckpt_every):
    """Issue-slot roofline of one captured batched step (pass 1 storing
    checkpoints and pass 2 from them over every instance): the slots per
    path-step of both persistent kernels, counted with SQ counters, over the
    whole step's time (the cost model's F + (F + R) when no count is
    committed for these sources)."""
    from paper_1901_04200_amd import roofline
    s1 = counted_slots("batch", "pass1", ckpt_every, "-", BATCH_VALU_PROFILE)
    s2 = counted_slots("batch", "pass2", ckpt_every, "-", BATCH_VALU_PROFILE)
    counted = s1 is not None and s2 is not None
    slots = s1 + s2 if counted else roofline.slots(roofline.per_path_step("heston", "pass1")) + \
        roofline.slots(roofline.per_path_step("heston", "pass2"))
    achieved = slots * path_steps / (ms_step * 1e-3) * 1e-12
    return {"bound": "alu", "kernel": "k_batch_pass1 + k_batch_pass2 (whole step)", "achieved": achieved,
            "peak": roofline.PEAK_SLOTS * 1e-12, "unit": "T VALU lane-slots/s",
            "frac": achieved / (roofline.PEAK_SLOTS * 1e-12), "slots_per_path_step": slots,
            "work": "VALU issue slots per path-step counted with SQ counters" if counted
            else "VALU issue slots per path-step of the cost model"}


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


def timed_gradient(mc, theta_np, C, steps, warmup):
    """Time `steps` calibrate_gradient calls and `steps` calibrate_forward
    calls on one context (inputs resident on the device); returns the
    timings, the library's per-pass kernel averages, the last outputs and
    the spread of single steps (another `steps` steps, each between its own
    events)."""
    import numpy as np
    import torch
    from paper_1901_04200_amd import capi
    ctx = mc.ctx
    theta = torch.tensor(theta_np, dtype=torch.float64, device="cuda")
    Ey = torch.empty(mc.m, dtype=torch.float64, device="cuda")
    G = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty(mc.M, dtype=torch.float64, device="cuda")

    def grad_step():
        capi.calibrate_gradient(ctx, theta, C, Ey, G, g)

    def fwd_step():
        capi.calibrate_forward(ctx, theta, Ey)

    for _ in range(warmup):
        grad_step()
        fwd_step()
    torch.cuda.synchronize()
    capi.cal_timing_enable(ctx, True)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        grad_step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = ev0.elapsed_time(ev1) / steps
    p1_ms, p1_n = capi.cal_timing_read(ctx, 0)
    p2_ms, p2_n = capi.cal_timing_read(ctx, 1)
    got = (Ey.cpu().numpy().copy(), float(G.item()), g.cpu().numpy().copy())
    capi.cal_timing_enable(ctx, True)
    ev0.record()
    for _ in range(steps):
        fwd_step()
    ev1.record()
    torch.cuda.synchronize()
    ms_fwd = ev0.elapsed_time(ev1) / steps
    f_ms, f_n = capi.cal_timing_read(ctx, 0)
    capi.cal_timing_enable(ctx, False)
    # the spread of single steps: each step of another `steps` bracketed by its own events
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in evs:
        a.record()
        grad_step()
        b.record()
    torch.cuda.synchronize()
    one = sorted(a.elapsed_time(b) for a, b in evs)
    stats = {"n": steps, "median": float(np.median(one)), "min": one[0], "max": one[-1]}
    status = mc.status()
    return {"ms_step": ms_step, "wall": wall, "ms_fwd": ms_fwd, "pass1_avg": p1_ms / max(p1_n, 1),
            "pass2_avg": p2_ms / max(p2_n, 1), "t_f": f_ms / max(f_n, 1), "status": status, "got": got,
            "step_stats": stats}


def theta0_leg(pb, th0, C, ckpt_every, ppl, steps, warmup):
    """The first draw of the Heston box (2 kappa theta_bar << xi^2): the FP32
    gradient timed there and compared with the oracle, and the FP64 path at
    the same point (its prices are the parity-checked ones there)."""
    from oracle import parity as PY
    from oracle import oracle as O
    from paper_1901_04200_amd.mc import MonteCarloCalibration
    out = {"theta": [float(v) for v in th0], "feller_ratio": float(2 * th0[0] * th0[1] / th0[2] ** 2)}
    Eo, Go, go = O.gradient(pb, th0, C.cpu().numpy())
    shares = PY.gradient_shares(O, pb, th0, C.cpu().numpy(), Eo)
    out["one_path_share"] = [float(v) for v in shares]
    for prec, k in (("fp32", ckpt_every), ("fp64", 8)):
        mc = MonteCarloCalibration(pb, precision=prec, ckpt_every=k, ckpt_mode="store",
                                   paths_per_lane=ppl if prec == "fp32" else 1)
        r = timed_gradient(mc, th0, C, max(3, steps // 2), warmup)
        mc.close()
        Ey, G, g = r["got"]
        out[prec] = {"ms_per_step": r["ms_step"], "paths_steps_per_s": pb.n_paths * pb.n_steps / (r["ms_step"] * 1e-3),
                     "ckpt_every": k, "status": r["status"],
                     "ey_err": PY.ey_err(Ey, Eo), "grad_err": PY.grad_err(g, go),
                     "grad_err_inf": PY.grad_err_inf(g, go), "G_rel_err": abs(G - Go) / abs(Go),
                     "ey_within_tolerance": PY.ey_err(Ey, Eo) <= PY.EY_TOL_FP32}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--theta", default="feller", choices=["feller", "first"],
                    help="timed parameter vector: the tenth draw of the Heston box (2 kappa theta_bar > xi^2, "
                         "the full-size parity test's) or the first draw (Feller's condition badly violated)")
    ap.add_argument("--ckpt-mode", default="store", choices=["store", "rerun"])
    ap.add_argument("--ckpt-every", type=int, default=0, help="8, 16 or 32; 0 = tuned (8 or 16)")
    ap.add_argument("--paths-per-lane", type=int, default=0, help="1, 2 or 4; 0 = tuned (1 or 2)")
    ap.add_argument("--cpu-sample-paths", type=int, default=1 << 13,
                    help="paths of the single-thread oracle timing")
    ap.add_argument("--cpu-min-seconds", type=float, default=4.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the extra legs")
    ap.add_argument("--extras", default="theta0,rerun,bs_schemes,slv,lv,e2_sweep,batched,surrogate_vs_mc",
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

    import torch

    from paper_1901_04200_amd import costmodel, roofline
    from paper_1901_04200_amd import workloads as W
    from paper_1901_04200_amd.mc import MonteCarloCalibration

    torch.cuda.set_device(0)
    pb, th0, tht, eps = W.heston_problem()
    th_feller = W.heston_draws(2, 10)[9]
    theta_np = th_feller if args.theta == "feller" else th0
    P, N = pb.n_paths, pb.n_steps
    # targets: model prices at the target draw (Philox seed 2) plus 0.1 % noise
    gen = MonteCarloCalibration(pb.with_(seed=2), precision=args.precision)
    C = torch.tensor(W.noisy_targets(gen.forward(tht).cpu().numpy(), eps), dtype=torch.float64, device="cuda")
    gen.close()
    ckpt_every, ppl, tune_table = args.ckpt_every, args.paths_per_lane, None
    if ckpt_every == 0 or ppl == 0:
        from paper_1901_04200_amd.mc import pick_config
        (ckpt_every, ppl), tune_table = pick_config(pb, theta_np, C, precision=args.precision,
                                                    ks=(8, 16) if ckpt_every == 0 else (ckpt_every,),
                                                    ppls=(1, 2) if ppl == 0 else (ppl,))
        print(f"bench: checkpoint spacing {ckpt_every}, {ppl} path(s) per lane ({tune_table})", file=sys.stderr,
              flush=True)
    mc = MonteCarloCalibration(pb, precision=args.precision, ckpt_every=ckpt_every, ckpt_mode=args.ckpt_mode,
                               paths_per_lane=ppl)
    geo = mc.geometry()
    r = timed_gradient(mc, theta_np, C, args.steps, args.warmup)
    mc.close()
    assert r["status"] == 0, "device status flags set"
    ms_step = r["ms_step"]
    print(f"bench: {args.steps} gradient steps, {ms_step:.3f} ms/step (wall {r['wall']:.3f} s)", file=sys.stderr,
          flush=True)

    pass2_avg, t_f = r["pass2_avg"], r["t_f"]
    kr_kf = costmodel.kr_over_kf(t_f, pass2_avg)
    path_steps = P * N
    model = "heston"
    kern = "pass2" if args.ckpt_mode == "store" else "pass2_rerun"
    w2 = roofline.per_path_step(model, kern)
    flops2 = w2["flops"] * path_steps                      # FP32 flops of one pass-2 launch
    achieved = flops2 / (pass2_avg * 1e-3) / 1e12          # TFLOP/s
    slots_frac = roofline.slots(w2) * path_steps / (pass2_avg * 1e-3) / roofline.PEAK_SLOTS
    flops_all = (roofline.per_path_step(model, "pass1")["flops"] + w2["flops"]) * path_steps
    fp32_tflops = flops_all / (ms_step * 1e-3) / 1e12

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
            "theta": [float(v) for v in theta_np],
            "theta_draw": "tenth draw of the Heston box (rng 2), 2 kappa theta_bar > xi^2" if args.theta == "feller"
                          else "first draw of the Heston box (rng 2), 2 kappa theta_bar << xi^2",
            "n_paths": P, "n_steps": N, "n_instr": pb.n_instr, "n_params": 5,
            "ckpt_every": geo["ckpt_every"], "ckpt_mode": args.ckpt_mode,
            "paths_per_lane": ppl,
            "tuning_ms": None if tune_table is None else {f"k{k}_ppl{q}": t * 1e3 for (k, q), t in tune_table},
            "threads_per_block": geo["threads"], "blocks": geo["blocks"],
        },
        "ms_per_step_single": r["step_stats"],
        "device": device_info(),
        "forward_value": path_steps / (r["ms_fwd"] * 1e-3),
        "ms_forward": r["ms_fwd"],
        "ms_pass1_kernel": r["pass1_avg"],
        "ms_pass2_kernel": pass2_avg,
        "kr_over_kf": kr_kf,
        "cost_g_over_cost_f": costmodel.gradient_over_forward(kr_kf),
        "fp32_tflops_whole_step": fp32_tflops,
        "fp32_peak_frac_whole_step": fp32_tflops / roofline.PEAK_FP32_TFLOPS,
        "parity": None,
        "surrogate_vs_mc": None,
        "roofline": {
            "bound": "alu",
            "kernel": "k_pass2 (Heston, FP32, K=%d, %s)" % (geo["ckpt_every"], args.ckpt_mode),
            "achieved": achieved,
            "peak": roofline.PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / roofline.PEAK_FP32_TFLOPS,
            "flops_per_path_step": w2["flops"],
            "frac_ceiling_at_full_issue": roofline.flop_ceiling(w2),
            "issue_slots_per_path_step": roofline.slots(w2),
            "issue_frac_cost_model": slots_frac,
            "issue_frac_counters": valu_issue_utilisation(geo["ckpt_every"]),
            "counted_fp32": counted_flops(geo["ckpt_every"], path_steps, pass2_avg),
            "traffic": pass2_traffic(geo["ckpt_every"], ppl),
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "traffic_algorithmic": roofline.pass2_bytes(pb.n_paths, geo["ckpt_every"], geo["blocks"], pb.n_instr,
                                                        pb.n_steps),
        },
    }
    if not args.no_cpu_baseline:
        print("bench: oracle parity of the timed input and CPU baseline ...", file=sys.stderr, flush=True)
        out["parity"], out["cpu_baseline"] = oracle_leg(pb, theta_np, C.cpu().numpy(), r["got"],
                                                        args.cpu_sample_paths, args.cpu_min_seconds, t_f)
        print(f"bench: parity {out['parity']['ey_err']:.2e} (E y) {out['parity']['grad_err']:.2e} (grad)",
              file=sys.stderr, flush=True)
    if not args.no_extras:
        legs = (("theta0", lambda: theta0_leg(pb, th0, C, ckpt_every, ppl, args.steps, args.warmup)),
                ("rerun", lambda: rerun_leg(pb, theta_np, C, ckpt_every, ppl, args.steps, args.warmup, t_f)),
                ("bs_schemes", lambda: bs_schemes_leg(max(5, args.steps // 2))),
                ("slv", lambda: slv_leg(max(5, args.steps // 2))),
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
    print(json.dumps(out), flush=True)


def rerun_leg(pb, theta_np, C, ckpt_every, ppl, steps, warmup, t_f):
    """The paper's memory-lean case: pass 2 re-runs the forward sweep itself
    (Cost(G) = (2 K_F + K_R)/c per path), beside the stored-checkpoint default."""
    from paper_1901_04200_amd import costmodel
    from paper_1901_04200_amd.mc import MonteCarloCalibration
    mc = MonteCarloCalibration(pb, ckpt_every=ckpt_every, ckpt_mode="rerun", paths_per_lane=ppl)
    r = timed_gradient(mc, theta_np, C, steps, warmup)
    mc.close()
    return {"ckpt_mode": "rerun", "ckpt_every": ckpt_every, "ms_per_step": r["ms_step"],
            "paths_steps_per_s": pb.n_paths * pb.n_steps / (r["ms_step"] * 1e-3),
            "ms_pass1_kernel": r["pass1_avg"], "ms_pass2_kernel": r["pass2_avg"], "status": r["status"],
            "cost_g_over_cost_f": (r["pass1_avg"] + r["pass2_avg"]) / t_f,
            "kr_over_kf": costmodel.kr_over_kf(t_f, r["pass2_avg"] - t_f)}


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
            "mc_grad_rel_err_at_p_star": res["mc_grad_rel_err_at_p_star"],
            "us_surrogate_step": st["surrogate"] * 1e6, "us_mc_step_at_p_star": st["mc_at_p_star"] * 1e6,
            "mc_over_surrogate": st["mc_over_surrogate"], "gain_test": gain, "details": details}


if __name__ == "__main__":
    main()
