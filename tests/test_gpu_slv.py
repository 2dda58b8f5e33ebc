"""Heston stochastic local volatility on the GPU (the paper's test model:
5 Heston parameters + a 10 x 20 leverage grid, 200 calls at the grid nodes)
against the FP64 oracle on the same streams.

Bounds as for local volatility: E y 1e-5 (FP32) / 1e-12 (FP64); gradient,
per component, 1e-4 (FP32) / 1e-9 (FP64: path state, leverage-node slices
and sums all in FP64).  Heston parameters come from the Feller part of
the box, where the pathwise gradient is well conditioned.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1901_04200_amd import autograd as AG
from oracle import parity as PY
from paper_1901_04200_amd import workloads as W
from paper_1901_04200_amd.mc import MonteCarloCalibration

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


ey_err = PY.ey_err
g_err = PY.grad_err          # per component: max_j |dg_j| / max(|g_j|, 1e-3 max|g|)


def run(pb, th, C, precision, **kw):
    mc = MonteCarloCalibration(pb, precision=precision, **kw)
    Ey_f = mc.forward(th).cpu().numpy()
    Ey, G, g = mc.gradient(th, C)
    st = mc.status()
    mc.close()
    assert st == 0
    return Ey_f, Ey.cpu().numpy(), float(G.item()), g.cpu().numpy()


@pytest.fixture(scope="module")
def slv_small(orc):
    pb, th0, tht, eps, coords = W.slv_problem(n_paths=(1 << 14) + 37)
    C = W.noisy_targets(orc.forward(pb, tht), eps)
    return pb, th0, tht, C, coords


def test_slv_fp32_matches_oracle(orc, slv_small):
    pb, th0, tht, C, _ = slv_small
    say("slv fp32 P=2^14+37 N=256 M=205")
    Ey_f, Ey, G, g = run(pb, th0, C, "fp32")
    Eo, Go, go = orc.gradient(pb, th0, C)
    say(f"  errors Ey {ey_err(Ey, Eo):.2e} grad {g_err(g, go):.2e} (Heston part {g_err(g[:5], go[:5]):.2e})")
    assert ey_err(Ey_f, Eo) <= 1e-5 and ey_err(Ey, Eo) <= 1e-5
    assert abs(G - Go) <= 1e-4 * Go
    assert g_err(g, go) <= 1e-4


def test_slv_fp64_matches_oracle(orc):
    pb, th0, tht, eps, _ = W.slv_problem(n_paths=4096 + 3, n_steps=64)
    C = W.noisy_targets(orc.forward(pb, tht), eps)
    say("slv fp64 P=4099 N=64")
    Eo, Go, go = orc.gradient(pb, th0, C)
    for mode in ("store", "rerun"):
        Ey_f, Ey, G, g = run(pb, th0, C, "fp64", ckpt_mode=mode)
        say(f"  {mode}: errors Ey {ey_err(Ey, Eo):.2e} grad {g_err(g, go):.2e} "
            f"(Heston part {g_err(g[:5], go[:5]):.2e})")
        assert ey_err(Ey, Eo) <= 1e-12
        assert g_err(g, go) <= 1e-9


def test_slv_checkpoint_spacings(slv_small):
    pb, th0, tht, C, _ = slv_small
    res = {}
    for mode in ("store", "rerun"):
        for k in (8, 16, 32):
            res[(mode, k)] = run(pb, th0, C, "fp32", ckpt_every=k, ckpt_mode=mode)
    base = res[("store", 8)]
    for key, r in res.items():
        np.testing.assert_array_equal(r[1], base[1])
        assert g_err(r[3], base[3]) <= 1e-5, key
    for k in (8, 16, 32):
        np.testing.assert_array_equal(res[("store", k)][3], res[("rerun", k)][3])


def test_slv_edge_shapes(orc):
    """One leverage row, a single path, ragged segment ends (N not a
    multiple of the spacing) and a call maturing at the first step, FP64."""
    for n_t, P, N, k in ((1, 1, 21, 8), (2, 63, 37, 16), (3, 257, 50, 32)):
        pb, th0, tht, eps, _ = W.slv_problem(n_paths=P, n_steps=N, n_t=n_t, n_k=4)
        pb = pb.with_(instr_step=np.concatenate([[1], pb.instr_step[1:]]).astype(np.int32))
        C = np.linspace(2.0, 9.0, pb.n_instr)
        Ey_f, Ey, G, g = run(pb, th0, C, "fp64", ckpt_every=k)
        Eo, Go, go = orc.gradient(pb, th0, C)
        say(f"  nT={n_t} P={P} N={N} K={k}: Ey {ey_err(Ey, Eo):.2e} grad {g_err(g, go):.2e}")
        assert ey_err(Ey, Eo) <= 1e-12
        assert g_err(g, go) <= 1e-9


def test_slv_invalid_theta_sets_status(slv_small):
    pb, th0, tht, C, _ = slv_small
    bad = th0.copy()
    bad[7] = -0.5     # a negative leverage node
    mc = MonteCarloCalibration(pb, precision="fp32")
    mc.forward(bad)
    assert mc.status() & 1
    mc.close()


def test_slv_autograd_backward_is_the_adjoint(slv_small):
    pb, th0, tht, C, _ = slv_small
    mc = AG.make(pb, "fp32")
    th = torch.tensor(th0, dtype=torch.float64, device="cuda", requires_grad=True)
    Ct = torch.as_tensor(C, device="cuda")
    Ey = AG.mc_prices(th, mc)
    G = 0.5 * torch.sum((Ey - Ct) ** 2)
    G.backward()
    _, G2, g2 = mc.gradient(th0, Ct)
    assert abs(G.item() - G2.item()) <= 1e-12 * G2.item()
    np.testing.assert_allclose(th.grad.cpu().numpy(), g2.cpu().numpy(), rtol=0, atol=1e-6 * g2.abs().max().item())
    mc.close()


def test_slv_full_size_oracle_and_fd(orc):
    """2^20 paths x 256 steps (the benchmark's SLV workload): FP32 gradient
    against the oracle; FP64 gradient against central differences of the FP64
    device forward (h = 1e-6, common random numbers) on 10 random
    coordinates at 2^16 paths."""
    pb, th0, tht, eps, coords = W.slv_problem()
    say("slv full size: oracle targets (2^20 paths, seed 2)")
    C = W.noisy_targets(orc.forward(pb.with_(seed=2), tht), eps)
    say("slv full size: device gradient")
    Ey_f, Ey, G, g = run(pb, th0, C, "fp32")
    say("slv full size: oracle gradient")
    Eo, Go, go = orc.gradient(pb, th0, C)
    say(f"  full size errors Ey {ey_err(Ey, Eo):.2e} grad {g_err(g, go):.2e}")
    assert ey_err(Ey, Eo) <= 1e-5
    assert g_err(g, go) <= 1e-4
    sub = pb.with_(n_paths=1 << 16)
    mc = MonteCarloCalibration(sub, precision="fp64")
    Ct = torch.as_tensor(C, device="cuda")
    _, _, g64 = mc.gradient(th0, Ct)
    g64 = g64.cpu().numpy()
    h = 1e-6
    worst = 0.0
    for j in coords:
        e = np.zeros(pb.n_params)
        e[j] = h
        Gp = 0.5 * torch.sum((mc.forward(th0 + e) - Ct) ** 2).item()
        Gm = 0.5 * torch.sum((mc.forward(th0 - e) - Ct) ** 2).item()
        fd = (Gp - Gm) / (2 * h)
        worst = max(worst, abs(fd - g64[j]) / np.max(np.abs(g64)))
        say(f"  coordinate {j}: fd {fd:.8g} adjoint {g64[j]:.8g}")
    say(f"  worst |fd - adjoint| / max|g| = {worst:.2e}")
    assert worst <= 1e-5
    mc.close()


def test_slv_paths_per_lane(orc):
    pb, th0, tht, eps, _ = W.slv_problem(n_paths=2 * 256 + 5, n_steps=48)
    C = np.linspace(2.0, 9.0, pb.n_instr)
    Eo, Go, go = orc.gradient(pb, th0, C)
    for ppl, k in ((2, 8), (4, 8), (2, 16), (2, 32)):
        for prec, tol_y, tol_g in (("fp64", 1e-12, 1e-9), ("fp32", 1e-5, 1e-4)):
            Ey_f, Ey, G, g = run(pb, th0, C, prec, paths_per_lane=ppl, ckpt_every=k)
            say(f"  ppl={ppl} K={k} {prec}: Ey {ey_err(Ey, Eo):.2e} grad {g_err(g, go):.2e}")
            assert ey_err(Ey, Eo) <= tol_y
            assert g_err(g, go) <= tol_g


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_unit_leverage_is_heston(slv_small, precision):
    """Two independent kernels on the same streams: with every leverage node
    at 1 the SLV sweep is the Heston sweep operation for operation (L s z1'
    = s z1', (h/2) L^2 v+ = (h/2) v+, no spot slope), so the prices are
    bitwise Heston's, and the Heston part of the gradient differs only by the
    association of the reverse step's terms (1e-12 FP64, 1e-6 FP32
    relative per component; both at K = 8, so the FP32 segment sums cover the
    same steps)."""
    pb, th0, _, C, _ = slv_small
    th = np.concatenate([th0[:5], np.ones(pb.n_params - 5)])
    hp = pb.with_(model=W.MODEL_HESTON, n_params=5, t_nodes=None, k_nodes=None)
    say(f"slv with unit leverage vs heston, {precision}")
    _, Ey_s, G_s, g_s = run(pb, th, C, precision, ckpt_every=8)
    _, Ey_h, G_h, g_h = run(hp, th[:5], C, precision, ckpt_every=8)
    np.testing.assert_array_equal(Ey_s, Ey_h)
    eg = g_err(g_s[:5], g_h)
    say(f"  Heston part of the gradient: {eg:.2e}")
    assert eg <= (1e-12 if precision == "fp64" else 1e-6)


def test_slv_longest_time_grid(orc):
    """64 leverage rows (the limit) over 256 steps: the row changes every 4
    steps, inside every checkpoint segment; FP64 against the oracle in both
    checkpoint modes."""
    pb, th0, tht, eps, _ = W.slv_problem(n_paths=1000, n_steps=256, n_t=64, n_k=6)
    C = np.linspace(2.0, 9.0, pb.n_instr)
    Eo, Go, go = orc.gradient(pb, th0, C)
    for k in (8, 32):
        for mode in ("store", "rerun"):
            say(f"  slv nT=64 nK=6 fp64 K={k} {mode}")
            Ey_f, Ey, G, g = run(pb, th0, C, "fp64", ckpt_every=k, ckpt_mode=mode)
            assert ey_err(Ey_f, Eo) <= 1e-12 and ey_err(Ey, Eo) <= 1e-12
            assert g_err(g, go) <= 1e-9
