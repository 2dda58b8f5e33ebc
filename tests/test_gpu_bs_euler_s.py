"""GPU parity of the Black-Scholes passes with the Euler scheme on S (the SDE
as written, model CAL_BS_EULER_S) against the FP64 CPU oracle on identical
random streams.

Tolerances as in test_gpu_parity.py (oracle.parity): E y within 1e-12 (FP64
state) and 1e-5 (FP32 state) of max(|E y_i|, 1e-2); the gradient per
component within 1e-10 (FP64) and 1e-4 (FP32).  The one-parameter gradient
of this workload is a sum of smooth per-path terms (no path carries more
than a fraction of a percent of it), so no conditioning gate is needed.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import parity as PY
from paper_1901_04200_amd import capi
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
    capi.lib()


def run(pb, th, C, precision, **kw):
    mc = MonteCarloCalibration(pb, precision=precision, **kw)
    Ey_f = mc.forward(th).cpu().numpy()
    Ey, G, g = mc.gradient(th, C)
    out = dict(Ey_f=Ey_f, Ey=Ey.cpu().numpy(), G=float(G.item()), g=g.cpu().numpy())
    assert mc.status() == 0
    mc.close()
    return out


@pytest.mark.parametrize("precision,k", [("fp64", 8), ("fp64", 16), ("fp32", 16), ("fp32", 8)])
def test_matches_oracle(orc, precision, k):
    """The Black-Scholes workload (2^14 paths, 16 steps, m = 4) in both
    checkpoint modes; forward-only and gradient prices are the same sums."""
    pb, th, C = W.bs_problem(euler_on_s=True)
    Eo, Go, go = orc.gradient(pb, th, C)
    for mode in ("store", "rerun"):
        say(f"bs euler-on-S {precision} K={k} {mode}")
        r = run(pb, th, C, precision, ckpt_every=k, ckpt_mode=mode)
        ey, eg = PY.ey_err(r["Ey"], Eo), PY.grad_err(r["g"], go)
        say(f"  Ey {ey:.2e} grad {eg:.2e} G {abs(r['G'] - Go) / Go:.2e}")
        np.testing.assert_array_equal(r["Ey_f"], r["Ey"])
        if precision == "fp64":
            assert ey <= 1e-12 and eg <= 1e-10
        else:
            assert ey <= 1e-5 and eg <= 1e-4


def test_full_size_fp32(orc):
    """2^20 paths x 256 steps (the log-Euler bound's workload scaled up):
    FP32 state within the Monte Carlo bounds of the oracle."""
    pb, th, C = W.bs_problem(n_paths=1 << 20, n_steps=256, euler_on_s=True)
    Eo, Go, go = orc.gradient(pb, th, C)
    r = run(pb, th, C, "fp32", ckpt_every=16)
    ey, eg = PY.ey_err(r["Ey"], Eo), PY.grad_err(r["g"], go)
    say(f"bs euler-on-S full size fp32: Ey {ey:.2e} grad {eg:.2e}")
    assert ey <= 1e-5 and eg <= 1e-4


@pytest.mark.parametrize("P,N,steps,k", [
    (1, 16, [16, 16, 8], 8),
    (63, 3, [1, 2, 3, 3], 8),
    (257, 37, [37, 5, 20, 5, 1], 16),
    (1000, 40, [40, 33, 17], 32),
])
def test_edge_shapes_fp64(orc, P, N, steps, k):
    """Ragged path counts, step counts that are not a multiple of the
    checkpoint spacing or of the Philox call, unsorted maturities, and one,
    two or four paths per lane."""
    steps = np.array(steps, dtype=np.int32)
    pb = W.Problem(model=W.MODEL_BS_S, n_params=1, n_steps=N, n_paths=P, t_max=N / 64.0, instr_step=steps,
                   instr_strike=np.linspace(85.0, 115.0, len(steps)), seed=77, inst=2)
    th = np.array([0.3])
    C = np.linspace(3.0, 9.0, len(steps))
    Eo, Go, go = orc.gradient(pb, th, C)
    for ppl in (1, 2, 4):
        for mode in ("store", "rerun"):
            say(f"bs euler-on-S edge P={P} N={N} K={k} ppl={ppl} {mode}")
            r = run(pb, th, C, "fp64", ckpt_every=k, ckpt_mode=mode, paths_per_lane=ppl)
            assert PY.ey_err(r["Ey"], Eo) <= 1e-12
            assert PY.grad_err(r["g"], go) <= 1e-10


def test_sigma_zero_is_deterministic():
    """sigma = 0: every path is S0 (1 + r h)^n, so the prices are the
    discounted intrinsic values of that forward (FP64 state)."""
    pb, _, C = W.bs_problem(n_paths=1000, n_steps=16, euler_on_s=True)
    h = pb.t_max / pb.n_steps
    SN = pb.s0 * (1.0 + pb.rate * h) ** pb.n_steps
    ref = math.exp(-pb.rate * pb.t_max) * np.maximum(SN - pb.instr_strike, 0.0)
    r = run(pb, np.array([0.0]), C, "fp64")
    np.testing.assert_allclose(r["Ey"], ref, rtol=1e-13, atol=1e-13)


def test_vjp_and_stored_checkpoints(orc):
    """calibrate_vjp and calibrate_vjp_stored (after a storing forward) give
    the oracle's vector-Jacobian product."""
    pb, th, _ = W.bs_problem(euler_on_s=True)
    lam = np.array([1.0, -2.0, 0.5, 3.0])
    go = orc.vjp(pb, th, lam)
    mc = MonteCarloCalibration(pb, precision="fp64", ckpt_every=8)
    g1 = mc.vjp(th, lam).cpu().numpy()
    mc.forward_store(th)
    g2 = mc.vjp_stored(th, lam).cpu().numpy()
    assert mc.status() == 0
    mc.close()
    np.testing.assert_array_equal(g1, g2)
    assert abs(g1[0] - go[0]) <= 1e-10 * abs(go[0])


def test_unsupported_entry_points_refuse():
    """Tangent mode, batching and the allocation-free entry point serve the
    log-Euler Black-Scholes and Heston models only."""
    pb, th, C = W.bs_problem(euler_on_s=True)
    mc = MonteCarloCalibration(pb, precision="fp64")
    with pytest.raises(capi.CalError) as e:
        mc.jacobian(th)
    assert e.value.code == capi.CAL_EUNSUPPORTED
    mc.close()
    dev = torch.device("cuda", 0)
    t = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64), device=dev)
    Ey, G, g = t(np.zeros(4)), t(np.zeros(1)), t(np.zeros(1))
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    with pytest.raises(capi.CalError) as e:
        capi.calibrate_gradient_static(pb, t(th), t(C), Ey, G, g, status, precision=capi.CAL_FP64)
    assert e.value.code == capi.CAL_EUNSUPPORTED


def test_autograd_backward_is_the_adjoint():
    """theta.grad of G = 1/2 |Ey - C|^2 through the torch.autograd wrapper
    equals calibrate_gradient's gradient on the same context (FP32)."""
    from paper_1901_04200_amd import autograd as AG
    pb, th0, C = W.bs_problem(n_paths=(1 << 16) + 5, n_steps=64, euler_on_s=True)
    mc = AG.make(pb, "fp32")
    th = torch.tensor(th0, dtype=torch.float64, device="cuda", requires_grad=True)
    Ct = torch.as_tensor(C, device="cuda")
    G = 0.5 * torch.sum((AG.mc_prices(th, mc) - Ct) ** 2)
    G.backward()
    _, G2, g2 = mc.gradient(th0, Ct)
    assert mc.status() == 0
    mc.close()
    assert abs(G.item() - G2.item()) <= 1e-12 * G2.item()
    assert abs(th.grad.item() - g2.item()) <= 1e-12 * abs(g2.item())
