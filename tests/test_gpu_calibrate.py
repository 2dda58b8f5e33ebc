"""Calibration by gradient descent on the HIP gradient (the use the paper's
title names), and what the learned surrogate gains over the Monte Carlo
adjoint alone.

* Black-Scholes (sigma, FP64, 2^14 paths): projected L-BFGS on the library's
  two-pass gradient follows the oracle-driven run iterate by iterate and
  reaches the sigma the targets were priced at (0.25).
* Heston (FP64, small): the same, five parameters.
* Heston (FP32, the benchmark's 2^20 x 256 workload): L-BFGS brings G below
  1e-3 G(theta0) on a calibration instance, monotonically.
* Heston SLV, the paper's own test (calibrating the leverage grid and the
  five Heston parameters by gradient descent): FP64 on a small grid follows
  the oracle-driven run iterate by iterate; FP32 on the 2^20 x 256 workload
  brings G below 1e-3 G(theta0) from targets priced at a second parameter
  draw on the same streams (so the exact optimum has G = 0).
* Gain: a surrogate trained on Monte Carlo labels, used as the model of a
  trust-region iteration judged by the Monte Carlo gradient, reaches the
  same G level on at least 12 of 16 instances with at least half the Monte
  Carlo gradient calls and half the wall time (medians) of Monte Carlo
  L-BFGS alone.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1901_04200_amd import calibrate as K
from paper_1901_04200_amd import workloads as W
from paper_1901_04200_amd.mc import MonteCarloCalibration

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda", 0)


class OracleObjective:
    def __init__(self, orc, pb, C):
        self.orc, self.pb, self.C = orc, pb, np.asarray(C)

    def value_and_grad(self, th):
        Ey, G, g = self.orc.gradient(self.pb, th, self.C)
        return G, g

    def value(self, th):
        return 0.5 * float(np.sum((self.orc.forward(self.pb, th) - self.C) ** 2))


def _both(orc, pb, th0, C, lo, hi, precision, **kw):
    mc = MonteCarloCalibration(pb, precision=precision)
    obj = K.MonteCarloObjective(mc, C)
    r_gpu = K.calibrate(obj.value_and_grad, obj.value, th0, lo, hi, **kw)
    assert mc.status() == 0
    mc.close()
    o = OracleObjective(orc, pb, C)
    r_orc = K.calibrate(o.value_and_grad, o.value, th0, lo, hi, **kw)
    return r_gpu, r_orc


def test_bs_calibration_on_hip_gradient(orc):
    pb, th, C = W.bs_problem()
    say("bs fp64 2^14 paths: L-BFGS on the HIP gradient and on the oracle")
    r_gpu, r_orc = _both(orc, pb, th, C, [0.05], [1.0], "fp64", max_iter=30, pg_tol=1e-10)
    say(f"  sigma {r_gpu.theta[0]:.10f} (oracle {r_orc.theta[0]:.10f}), {r_gpu.n_grad} gradients, {r_gpu.status}")
    assert len(r_gpu.iterates) == len(r_orc.iterates)
    for a, b in zip(r_gpu.iterates, r_orc.iterates):
        assert abs(a[0] - b[0]) <= 1e-10
    assert abs(r_gpu.theta[0] - 0.25) < 0.01      # the targets were priced at sigma = 0.25
    g = MonteCarloCalibration(pb, precision="fp64")
    _, _, gg = g.gradient(r_gpu.theta, C)
    _, _, g0 = g.gradient(th, C)
    g.close()
    assert abs(float(gg[0])) < 1e-6 * abs(float(g0[0]))


def test_heston_fp64_calibration_iterates(orc):
    pb, _, _, eps = W.heston_problem(n_paths=4096 + 5, n_steps=64)
    a, b = W.heston_feller_draws(11, 2)
    C = W.noisy_targets(orc.forward(pb.with_(seed=2), b), eps)
    say("heston fp64 4101 paths x 64 steps: 8 L-BFGS iterations on the HIP gradient and on the oracle")
    r_gpu, r_orc = _both(orc, pb, a, C, W.HESTON_LO, W.HESTON_HI, "fp64", max_iter=8, feller=True)
    n = min(len(r_gpu.iterates), len(r_orc.iterates))
    dev = max(float(np.max(np.abs((x - y) / (W.HESTON_HI - W.HESTON_LO))))
              for x, y in zip(r_gpu.iterates[:n], r_orc.iterates[:n]))
    say(f"  {n} iterates, largest difference {dev:.2e} of the box; G {r_gpu.G:.6g} vs {r_orc.G:.6g}")
    assert n >= 8 and dev <= 1e-7
    assert abs(r_gpu.G - r_orc.G) <= 1e-8 * r_orc.G


def test_heston_fp32_calibration_converges():
    """The benchmark's workload: L-BFGS on the FP32 two-pass gradient brings G
    below 1e-3 G(theta0) on the first gain-test instance, G never rising."""
    from paper_1901_04200_amd import surrogate_study as SS
    pb, _, _, _ = W.heston_problem()
    th0, tht, C, G0, Gt = SS.gain_instances(pb, 1)[0]
    mc = MonteCarloCalibration(pb)
    obj = K.MonteCarloObjective(mc, C)
    r = K.calibrate(obj.value_and_grad, obj.value, th0, W.HESTON_LO, W.HESTON_HI, g_tol=1e-3 * G0, feller=True,
                    max_iter=200)
    assert mc.status() == 0
    mc.close()
    Gs = [h.G for h in r.history] + [r.G]
    say(f"heston fp32 2^20 x 256: G {G0:.4g} -> {r.G:.4g} in {r.n_grad} gradients ({r.status}); "
        f"G(target) {Gt:.3g}")
    assert r.status == "converged"
    assert all(y <= x for x, y in zip(Gs, Gs[1:]))


def _slv_box(M):
    """The Heston box for the first five parameters, [0.3, 2] for the leverage nodes."""
    return (np.concatenate([W.HESTON_LO, np.full(M - 5, 0.3)]), np.concatenate([W.HESTON_HI, np.full(M - 5, 2.0)]))


def test_slv_fp64_calibration_iterates(orc):
    pb, th0, tht, _, _ = W.slv_problem(n_paths=2048 + 3, n_steps=64, n_t=4, n_k=6)
    C = orc.forward(pb, tht)
    lo, hi = _slv_box(pb.n_params)
    say(f"slv fp64 {pb.n_paths} paths x 64 steps, {pb.n_params} parameters: 8 L-BFGS iterations on the HIP "
        "gradient and on the oracle")
    r_gpu, r_orc = _both(orc, pb, th0, C, lo, hi, "fp64", max_iter=8, feller=True)
    n = min(len(r_gpu.iterates), len(r_orc.iterates))
    dev = max(float(np.max(np.abs((x - y) / (hi - lo)))) for x, y in zip(r_gpu.iterates[:n], r_orc.iterates[:n]))
    say(f"  {n} iterates, largest difference {dev:.2e} of the box; G {r_gpu.G:.6g} vs {r_orc.G:.6g}")
    assert n >= 8 and dev <= 1e-7
    assert abs(r_gpu.G - r_orc.G) <= 1e-8 * r_orc.G


def test_slv_fp32_calibration_converges():
    """The Heston SLV workload (2^20 paths x 256 steps, 5 + 200 parameters,
    m = 200): L-BFGS on the FP32 two-pass gradient from the first parameter
    draw to targets priced at the second on the same streams brings G below
    1e-3 G(theta0), G never rising."""
    pb, th0, tht, _, _ = W.slv_problem()
    lo, hi = _slv_box(pb.n_params)
    mc = MonteCarloCalibration(pb)
    C = mc.forward(tht).cpu().numpy()
    obj = K.MonteCarloObjective(mc, C)
    G0 = obj.value_and_grad(th0)[0]
    r = K.calibrate(obj.value_and_grad, obj.value, th0, lo, hi, g_tol=1e-3 * G0, feller=True, max_iter=300)
    assert mc.status() == 0
    mc.close()
    Gs = [h.G for h in r.history] + [r.G]
    say(f"slv fp32 2^20 x 256: G {G0:.4g} -> {r.G:.4g} in {r.n_grad} gradients ({r.status})")
    assert r.status == "converged"
    assert all(y <= x for x, y in zip(Gs, Gs[1:]))


def test_surrogate_gain():
    """The surrogate (5 -> 256 -> 256 -> 256 -> 40, trained on 2^16 label
    draws at 2^14 paths each) against Monte Carlo L-BFGS alone on 16
    calibration instances of the 2^20 x 256 workload."""
    from paper_1901_04200_amd import surrogate_study as SS
    pb, _, _, _ = W.heston_problem()
    net, info = SS.train_surrogate(pb, 1 << 16, 1 << 14, 150, log=say)
    res = SS.gain_test(net, pb, 16, 1e-3, 200, log=say)
    net.close()
    for r in res["per_instance"]:
        say("  G0 %.3g: MC %s %d calls %.1f ms | surrogate %s %d calls %.1f ms" % (
            r["G0"], r["mc"]["reached"], r["mc"]["mc_calls"], 1e3 * r["mc"]["seconds"], r["surrogate"]["reached"],
            r["surrogate"]["mc_calls"], 1e3 * r["surrogate"]["seconds"]))
    say(f"  medians: MC calls {res['median_mc_calls_mc']} vs {res['median_mc_calls_surrogate']}, "
        f"seconds {res['median_seconds_mc']:.4f} vs {res['median_seconds_surrogate']:.4f}, "
        f"speedup {res.get('median_speedup')}")
    assert res["instances"] == 16
    assert res["reached_surrogate"] >= 12 and res["reached_mc"] >= 12
    assert res["median_mc_call_ratio"] >= 2.0
    assert res["median_speedup"] >= 2.0
