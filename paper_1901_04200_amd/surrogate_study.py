"""The surrogate against the plain Monte Carlo adjoint step, on one GPU.

  1. labels: E y and dE y/dtheta for n_train parameter draws (each draw its
     own Philox instance), by the Monte Carlo tangent kernel;
  2. training: the differential loss, bf16 MFMA kernels, Adam;
  3. accuracy: on held-out draws, the surrogate's gradient of
     G = 1/2 |y - C|^2 against a Monte Carlo reference gradient at
     ref_paths paths gives eps_s (median relative error);
  4. the Monte Carlo gradient's own error at P paths (independent seeds,
     the same held-out draws, the same reference) falls like P^-1/2; P* is
     where it equals eps_s;
  5. cost of one gradient step: surrogate (network forward, batch 1) vs the
     Monte Carlo adjoint (calibrate_gradient) at P* paths;
  6. gain test: on n_gain calibration instances (start and target draws),
     wall time and Monte Carlo gradient calls to bring G below
     g_frac G(theta0) by Monte Carlo projected L-BFGS alone and by the
     surrogate-assisted trust-region iteration (surrogate model, Monte Carlo
     judge), both at the benchmark's 2^20 paths.
Everything is on the Feller-satisfying part of the Heston box, where the
pathwise gradient is well conditioned.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import capi
from . import surrogate as S
from . import workloads as W
from .mc import MonteCarloCalibration


def _time_call(fn, reps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def _heldout_errors(net, ref, ho, C):
    """Relative gradient errors of the network on the held-out draws ho
    against the Monte Carlo reference context ref; returns (errors, g_ref)."""
    import torch
    g_ref = []
    for th in ho:
        _, _, g = ref.gradient(th, C)
        g_ref.append(g.cpu().numpy())
    g_ref = np.array(g_ref)
    _, g_s = net.calibration_gradient(torch.as_tensor(ho, dtype=torch.float32, device="cuda"), C)
    g_s = g_s.cpu().numpy()
    return np.linalg.norm(g_s - g_ref, axis=1) / np.linalg.norm(g_ref, axis=1), g_ref


def _mc_errors(pb, P, ho, g_ref, C, seeds):
    """Relative gradient errors of the P-path Monte Carlo gradient (Philox
    seeds 1000.., one context per seed) on the held-out draws."""
    errs = []
    for s_ in range(seeds):
        mc = MonteCarloCalibration(pb.with_(n_paths=P, seed=1000 + s_))
        for k in range(len(ho)):
            _, _, g = mc.gradient(ho[k], C)
            errs.append(np.linalg.norm(g.cpu().numpy() - g_ref[k]) / np.linalg.norm(g_ref[k]))
        mc.close()
    return np.array(errs)


def run(n_train=1 << 14, train_paths=1 << 14, n_heldout=64, ref_paths=1 << 26, epochs=200, batch=4096,
        lr=2e-3, lr_final=5e-5, w=1.0, seeds_mc=4, n_gain=16, g_frac=1e-3, max_iter=200, uniform_variant=True,
        log=print):
    import torch
    out = {}
    pb, th0, tht, eps = W.heston_problem()

    # ---- 1.-2. labels and training ------------------------------------------
    net, info = train_surrogate(pb, n_train, train_paths, epochs, batch=batch, lr=lr, lr_final=lr_final, w=w,
                                log=log)
    out.update(info)

    # ---- 3. accuracy on held-out draws -------------------------------------
    # targets: prices at the target draw (seed 2) plus 0.1 % noise
    gen = MonteCarloCalibration(pb.with_(seed=2))
    C = torch.as_tensor(W.noisy_targets(gen.forward(tht).cpu().numpy(), eps), device="cuda")
    gen.close()
    ho = W.heston_feller_draws(99, n_heldout)
    # held-out draws where Feller's condition fails (uniform box draws of rng(98))
    box = W.heston_draws(98, 8 * n_heldout)
    ho_nf = box[2 * box[:, 0] * box[:, 1] < box[:, 2] ** 2][:n_heldout]
    ref = MonteCarloCalibration(pb.with_(n_paths=ref_paths, seed=7))
    err_s, g_ref = _heldout_errors(net, ref, ho, C)
    err_nf, g_ref_nf = _heldout_errors(net, ref, ho_nf, C)
    eps_s = float(np.median(err_s))
    out["surrogate_grad_rel_err"] = {"median": eps_s, "p90": float(np.quantile(err_s, 0.9)),
                                     "heldout": n_heldout, "ref_paths": ref_paths,
                                     "non_feller_median": float(np.median(err_nf)),
                                     "non_feller_p90": float(np.quantile(err_nf, 0.9))}
    log(f"surrogate: held-out gradient error median {eps_s:.3g} (Feller draws), {np.median(err_nf):.3g} "
        f"(non-Feller draws), vs MC at {ref_paths} paths")

    # ---- 4. Monte Carlo gradient error vs paths -----------------------------
    # every held-out draw, seeds 1000.., against the same reference
    curve = []
    for lp in range(10, 19, 2):
        P = 1 << lp
        curve.append((P, float(np.median(_mc_errors(pb, P, ho, g_ref, C, seeds_mc)))))
    out["mc_grad_rel_err_vs_paths"] = curve
    # err = a P^-1/2 fitted on the points with P >= 2^14 (below that the
    # relative error is no longer small), then solved for eps_s; the error at
    # P* is then measured there directly
    a = float(np.median([e * math.sqrt(P) for P, e in curve if P >= 1 << 14]))
    p_fit = max(256, int(round((a / eps_s) ** 2)))
    err_fit = float(np.median(_mc_errors(pb, p_fit, ho, g_ref, C, seeds_mc)))
    # one correction with the error measured at the fitted point (error ~ P^-1/2)
    p_star = max(256, int(round(p_fit * (err_fit / eps_s) ** 2)))
    err_star = float(np.median(_mc_errors(pb, p_star, ho, g_ref, C, seeds_mc)))
    out["mc_err_coefficient"] = a
    out["reference_rel_err_estimate"] = a / math.sqrt(ref_paths)
    out["p_fit"] = p_fit
    out["mc_grad_rel_err_at_p_fit"] = err_fit
    out["p_star"] = p_star
    out["mc_grad_rel_err_at_p_star"] = err_star
    log(f"surrogate: MC gradient error ~ {a:.3g}/sqrt(P) (reference ~{a / math.sqrt(ref_paths):.2g}); "
        f"equal to eps_s at {p_fit} paths by the fit, measured there {err_fit:.3g}; corrected P* = {p_star}, "
        f"measured there {err_star:.3g}")

    # ---- 5. step costs ------------------------------------------------------
    th1 = torch.as_tensor(ho[:1], dtype=torch.float32, device="cuda")
    bufs = net.calibration_buffers(1)

    def sur_step():
        net.calibration_gradient(th1, C, out=bufs)

    t_sur = _time_call(sur_step, 50)
    mcs = MonteCarloCalibration(pb.with_(n_paths=p_star))
    t_mc = _time_call(lambda: mcs.gradient(ho[0], C), 20)
    mcs.close()
    out["step_seconds"] = {"surrogate": t_sur, "mc_at_p_star": t_mc, "p_star_paths_timed": p_star,
                           "mc_over_surrogate": t_mc / t_sur}
    log(f"surrogate: step {t_sur * 1e6:.1f} us vs MC adjoint at {p_star} paths {t_mc * 1e6:.1f} us")

    # ---- 6. gain test ---------------------------------------------------------
    if n_gain > 0:
        out["gain"] = gain_test(net, pb, n_gain, g_frac, max_iter, log)
    net.close()

    # ---- 7. the literal training set: uniform draws over the whole box -------
    if uniform_variant:
        net_u, info_u = train_surrogate(pb, n_train, train_paths, epochs, batch=batch, lr=lr, lr_final=lr_final,
                                        w=w, log=log, region="box")
        e_f, _ = _heldout_errors(net_u, ref, ho, C)
        e_nf, _ = _heldout_errors(net_u, ref, ho_nf, C)
        out["uniform_training"] = {"loss_last": info_u["training"]["loss_last"],
                                   "grad_rel_err_median_feller": float(np.median(e_f)),
                                   "grad_rel_err_median_non_feller": float(np.median(e_nf))}
        log(f"surrogate (trained on uniform box draws): held-out gradient error median {np.median(e_f):.3g} "
            f"(Feller), {np.median(e_nf):.3g} (non-Feller)")
        net_u.close()
    ref.close()
    return out


def train_surrogate(pb, n_train, train_paths, epochs, batch=4096, lr=2e-3, lr_final=5e-5, w=1.0, log=print,
                    region="feller"):
    """Labels (E y and dE y/dtheta by the Monte Carlo tangent kernel, each of
    n_train draws its own Philox instance, seed 4) and the network trained on
    them with the differential loss; returns (net, timings and losses).
    region: "feller" (draws where 2 kappa theta_bar >= xi^2) or "box"
    (uniform over the whole Heston box)."""
    import torch
    lo, hi = W.HESTON_LO, W.HESTON_HI
    out = {}
    draws = W.surrogate_draws(n_train, rng_seed=6) if region == "feller" else W.heston_draws(6, n_train)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Ey, J = S.generate_labels(pb, draws, n_paths=train_paths, seed=4, chunk=256)
    torch.cuda.synchronize()
    t_lab = time.perf_counter() - t0
    out["labels"] = {"draws": n_train, "paths_per_draw": train_paths, "seconds": t_lab,
                     "path_steps_per_s": n_train * train_paths * pb.n_steps / t_lab}
    log(f"surrogate: labels for {n_train} draws x {train_paths} paths in {t_lab:.2f} s")
    net = S.MLP(5, 256, pb.n_instr, max_batch=batch)
    net.init_params(0)
    sh, sc, mu, sd = S.standard_scaling(lo, hi, Ey.cpu().numpy())
    net.set_scaling(sh, sc, mu, sd)
    thd = torch.as_tensor(draws, dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    jw = None
    if region != "feller":
        # Jacobian labels only where Feller's condition holds: elsewhere the
        # pathwise Jacobian is heavy-tailed (a few paths near zero variance
        # decide it) and those samples train on their prices alone
        feller = 2.0 * draws[:, 0] * draws[:, 1] >= draws[:, 2] ** 2
        jw = torch.as_tensor(feller.astype(np.float32), device="cuda")
        J = torch.where(jw[:, None, None] > 0, J, torch.zeros_like(J))
        out["jacobian_labels_kept"] = float(feller.mean())
    hist = S.fit(net, thd, Ey.float(), J.float(), epochs=epochs, batch=min(batch, n_train), lr=lr,
                 lr_final=lr_final, w=w, log_every=max(1, epochs // 10), jw=jw)
    t_fit = time.perf_counter() - t0
    steps = epochs * (n_train // min(batch, n_train))
    # useful GEMM work of one step: forward, input gradient and weight gradient
    # of the layers 256x256, 256x256 and 256xm over the primal and 5 tangent row
    # blocks (the 5x256 first layer is elementwise)
    rows = 6 * min(batch, n_train)
    flops = 3 * 2 * rows * (2 * 256 * 256 + 256 * pb.n_instr)
    # epochs after the second logged one replay the captured epoch: their rate
    # is the steady training step (the first epoch runs eagerly, the second is captured)
    spe = n_train // min(batch, n_train)
    replay = None
    if len(hist) >= 3 and hist[-1].epoch > hist[1].epoch:
        replay = (hist[-1].seconds - hist[1].seconds) / ((hist[-1].epoch - hist[1].epoch) * spe) * 1e3
    out["training"] = {"epochs": epochs, "seconds": t_fit, "loss_first": hist[0].loss, "loss_last": hist[-1].loss,
                       "steps": steps, "ms_per_step_replayed": replay, "gemm_flop_per_step": flops,
                       "gemm_tflops": flops * steps / t_fit * 1e-12,
                       "bf16_peak_frac": flops * steps / t_fit / 2.5e15}
    log(f"surrogate: {epochs} epochs in {t_fit:.2f} s, loss {hist[0].loss:.4g} -> {hist[-1].loss:.4g}")
    return net, out


def gain_instances(pb, n_inst, g_frac=1e-3, rng_seed=11, margin=2.0):
    """Calibration instances for the gain test: pairs (theta0, theta_target)
    of Feller draws of rng(rng_seed) with targets priced at theta_target
    (Philox seed 2) times 1 + 1e-3 eps (eps from rng(rng_seed + 1)), in draw
    order, keeping those whose target level g_frac G(theta0) lies above
    margin G(theta_target): G cannot go much below what the target
    parameters themselves reach (the targets carry noise and another seed's
    paths), so a pair with a lower target level does not test speed.
    Returns [(theta0, theta_target, C, G0, G_target)]."""
    gen = MonteCarloCalibration(pb.with_(seed=2))
    mc = MonteCarloCalibration(pb)
    rng = np.random.default_rng(rng_seed + 1)
    pool = W.heston_feller_draws(rng_seed, 16 * n_inst)
    out, k = [], 0
    try:
        while len(out) < n_inst and 2 * k + 1 < len(pool):
            th0, tht = pool[2 * k], pool[2 * k + 1]
            eps = rng.standard_normal(pb.n_instr)
            k += 1
            C = W.noisy_targets(gen.forward(tht).cpu().numpy(), eps)
            G0 = float(mc.gradient(th0, C)[1].item())
            Gt = float(mc.gradient(tht, C)[1].item())
            if g_frac * G0 > margin * Gt:
                out.append((th0, tht, C, G0, Gt))
    finally:
        gen.close()
        mc.close()
    return out


def gain_test(net, pb, n_inst, g_frac, max_iter, log=print, instances=None):
    """Calibrate n_inst instances (gain_instances) to G <= g_frac G(theta0)
    by Monte Carlo projected L-BFGS alone and by the surrogate-assisted
    trust-region iteration (surrogate model, Monte Carlo judge), both on the
    same 2^20-path Monte Carlo gradient; wall time and Monte Carlo gradient
    calls each."""
    import torch
    from .calibrate import MonteCarloObjective, calibrate
    lo, hi = W.HESTON_LO, W.HESTON_HI
    if instances is None:
        instances = gain_instances(pb, n_inst, g_frac)
    mc = MonteCarloCalibration(pb)
    rows = []
    # one warm-up calibration of each kind (first-call costs out of the timings)
    th0, tht, C, G0, Gt = instances[0]
    calibrate(MonteCarloObjective(mc, C).value_and_grad, None, th0, lo, hi, max_iter=2, feller=True)
    S.surrogate_calibration(net, mc, C, th0, lo, hi, iters=2, feller=True)
    for th0, tht, C, G0, Gt in instances:
        g_tol = g_frac * G0
        obj = MonteCarloObjective(mc, C)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = calibrate(obj.value_and_grad, obj.value, th0, lo, hi, max_iter=max_iter, g_tol=g_tol, feller=True)
        t_mc = time.perf_counter() - t0
        mc_calls = obj.n_grad + obj.n_value
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        th_s, recs = S.surrogate_calibration(net, mc, C, th0, lo, hi, iters=max_iter, feller=True, g_stop=g_tol)
        t_s = time.perf_counter() - t0
        G_s = recs[-1].G_mc if recs else G0
        rows.append({"G0": G0, "G_target": Gt,
                     "mc": {"reached": r.G <= g_tol, "G": r.G, "seconds": t_mc, "mc_calls": mc_calls,
                            "iters": len(r.history), "status": r.status},
                     "surrogate": {"reached": G_s <= g_tol, "G": G_s, "seconds": t_s,
                                   "mc_calls": 1 + sum(x.mc_calls for x in recs), "iters": len(recs),
                                   "accepted": sum(1 for x in recs if x.accepted_surrogate),
                                   "surrogate_launches": sum(x.inner_launches + 1 for x in recs)}})
    mc.close()
    both = [r_ for r_ in rows if r_["mc"]["reached"] and r_["surrogate"]["reached"]]
    med = lambda key, sub: float(np.median([r_[sub][key] for r_ in both])) if both else None
    summ = {"instances": len(rows), "g_frac": g_frac, "paths": pb.n_paths,
            "selection": "Feller pairs of rng(11) in draw order with g_frac G(theta0) > 2 G(theta_target)",
            "reached_mc": sum(r_["mc"]["reached"] for r_ in rows),
            "reached_surrogate": sum(r_["surrogate"]["reached"] for r_ in rows),
            "median_seconds_mc": med("seconds", "mc"), "median_seconds_surrogate": med("seconds", "surrogate"),
            "median_mc_calls_mc": med("mc_calls", "mc"), "median_mc_calls_surrogate": med("mc_calls", "surrogate"),
            "per_instance": rows}
    if both:
        summ["median_speedup"] = float(np.median([r_["mc"]["seconds"] / r_["surrogate"]["seconds"] for r_ in both]))
        summ["median_mc_call_ratio"] = float(np.median([r_["mc"]["mc_calls"] / r_["surrogate"]["mc_calls"]
                                                        for r_ in both]))
    log(f"surrogate: gain test reached {summ['reached_mc']}/{len(rows)} (MC L-BFGS) and "
        f"{summ['reached_surrogate']}/{len(rows)} (surrogate-assisted); median seconds {summ['median_seconds_mc']} vs "
        f"{summ['median_seconds_surrogate']}, MC calls {summ['median_mc_calls_mc']} vs "
        f"{summ['median_mc_calls_surrogate']}")
    return summ
