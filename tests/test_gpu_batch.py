"""Batched instances of uneven size in one step (persistent work queue),
its HIP-graph capture and the autotuner.

Each instance's result must be bitwise the one its own context gives (same
per-block code, same fixed-order reductions); against the FP64 oracle the
usual bounds hold (FP64 path: 1e-12 on E y, 1e-9 on the gradient, on
well-conditioned draws).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1901_04200_amd import workloads as W
from paper_1901_04200_amd.batch import BatchCalibration
from paper_1901_04200_amd.mc import MonteCarloCalibration

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def targets_for(insts):
    # smooth synthetic targets: parity does not need market-like ones
    return [np.linspace(2.0, 12.0, pb.n_instr) for pb, *_ in insts]


@pytest.fixture(scope="module")
def batch12():
    insts = W.batched_instances(12)
    Cs = targets_for(insts)
    th = np.array([t for _, t, _, _ in insts])
    return insts, Cs, th


def single(pb, th, C, precision="fp32", k=16, ppl=1):
    mc = MonteCarloCalibration(pb, precision=precision, ckpt_every=k, ckpt_mode="store", paths_per_lane=ppl)
    Ey, G, g = mc.gradient(th, C)
    out = Ey.cpu().numpy(), float(G.item()), g.cpu().numpy()
    mc.close()
    return out


def test_batch_matches_single_instances(batch12):
    insts, Cs, th = batch12
    say("batch of 12: m", [pb.n_instr for pb, *_ in insts], "P", [pb.n_paths for pb, *_ in insts],
        "N", [pb.n_steps for pb, *_ in insts])
    B = BatchCalibration([pb for pb, *_ in insts])
    thd = torch.tensor(th, device="cuda")
    Cd = torch.tensor(np.concatenate(Cs), device="cuda")
    Ey, G, g = B.gradient(thd, Cd)
    assert B.status() == 0
    Ey = B.split(Ey.cpu().numpy())
    G, g = G.cpu().numpy(), g.cpu().numpy()
    for i, (pb, t, _, _) in enumerate(insts):
        e1, G1, g1 = single(pb, t, Cs[i])
        np.testing.assert_array_equal(Ey[i], e1)
        assert G[i] == G1
        np.testing.assert_array_equal(g[i], g1)
    B.close()


def test_batch_graph_replays(batch12):
    insts, Cs, th = batch12
    B = BatchCalibration([pb for pb, *_ in insts])
    thd = torch.tensor(th, device="cuda")
    Cd = torch.tensor(np.concatenate(Cs), device="cuda")
    Ey, G, g = B.gradient(thd, Cd)
    ref = (Ey.clone(), G.clone(), g.clone())
    torch.cuda.synchronize()
    B.capture(thd, Cd)
    other = MonteCarloCalibration(insts[0][0], precision="fp32")
    for r in range(3):
        B.Ey.zero_()
        B.G.zero_()
        B.grad.zero_()
        B.replay()
        torch.cuda.synchronize()
        assert torch.equal(B.Ey, ref[0]) and torch.equal(B.G, ref[1]) and torch.equal(B.grad, ref[2]), r
        other.gradient(insts[0][1], Cs[0])   # eager work between replays
        torch.cuda.synchronize()
    other.close()
    assert B.status() == 0
    B.close()


def test_batch_configure_and_autotune(batch12):
    insts, Cs, th = batch12
    sub = insts[:5]
    B = BatchCalibration([pb for pb, *_ in sub])
    thd = torch.tensor(th[:5], device="cuda")
    Cd = torch.tensor(np.concatenate(Cs[:5]), device="cuda")
    for k, w, ppl in ((8, 1, 1), (32, 2, 2), (16, 0, 4)):
        B.configure(k, w, ppl)
        assert B.geometry()["paths_per_lane"] == ppl
        Ey, G, g = B.gradient(thd, Cd)
        Ey = B.split(Ey.cpu().numpy())
        for i in (0, 4):
            e1, G1, g1 = single(sub[i][0], sub[i][1], Cs[i], k=k, ppl=ppl)
            np.testing.assert_array_equal(Ey[i], e1)
            np.testing.assert_array_equal(g.cpu().numpy()[i], g1)
    best, table = B.autotune(thd, Cd, ks=(8, 16), wpcs=(0, 2), ppls=(1, 2), reps=2)
    say("autotune:", best, [(c, round(t * 1e3, 3)) for c, t in table])
    assert best in [c for c, _ in table]
    B.replay()
    torch.cuda.synchronize()
    e1, G1, g1 = single(sub[1][0], sub[1][1], Cs[1], k=best[0], ppl=best[2])
    np.testing.assert_array_equal(B.split(B.Ey.cpu().numpy())[1], e1)
    B.close()


def test_batch_fp64_against_oracle(orc):
    draws = W.heston_feller_draws(17, 3)
    pbs = []
    for i, (P, N, m) in enumerate(((4096 + 11, 64, 12), (3000, 128, 40), (513, 32, 8))):
        st, kk = W.heston_instruments(int(np.ceil(m / 5)), np.linspace(0.4, 2.0, 5), N / 2.0)
        pbs.append(W.Problem(model=W.MODEL_HESTON, n_params=5, n_steps=N, n_paths=P, t_max=2.0,
                             instr_step=st[:m], instr_strike=kk[:m], seed=1, inst=i))
    Cs = [np.linspace(3.0, 9.0, pb.n_instr) for pb in pbs]
    B = BatchCalibration(pbs, precision="fp64")
    Ey, G, g = B.gradient(torch.tensor(draws, device="cuda"), torch.tensor(np.concatenate(Cs), device="cuda"))
    Ey = B.split(Ey.cpu().numpy())
    for i, pb in enumerate(pbs):
        Eo, Go, go = orc.gradient(pb, draws[i], Cs[i])
        ey = np.max(np.abs(Ey[i] - Eo) / np.maximum(np.abs(Eo), 1e-2))
        eg = np.max(np.abs(g.cpu().numpy()[i] - go)) / np.max(np.abs(go))
        say(f"  instance {i}: Ey {ey:.2e} grad {eg:.2e}")
        assert ey <= 1e-12 and eg <= 1e-9
    B.close()


def test_batch_fp32_workload_sample_against_oracle(orc):
    """The batched workload itself (256 instances, uniform parameter draws,
    FP32 state) in one step; eight instances (every 32nd) against the FP64
    oracle.  E y is asserted at 1e-5 where Feller's condition holds (below it
    FP32 state cannot reach 1e-5: tests/test_precision_floor.py); gradient
    components at 1e-4 where no path carries more than 2% of the component
    (the one-path share); the rest are stated."""
    from oracle import parity as PY
    insts = W.batched_instances(256)
    Cs = targets_for(insts)
    th = np.array([t for _, t, _, _ in insts])
    B = BatchCalibration([pb for pb, *_ in insts])
    Ey, G, g = B.gradient(torch.tensor(th, device="cuda"), torch.tensor(np.concatenate(Cs), device="cuda"))
    assert B.status() == 0
    Ey = B.split(Ey.cpu().numpy())
    g = g.cpu().numpy()
    B.close()
    asserted = 0
    for i in range(0, 256, 32):
        pb = insts[i][0]
        Eo, Go, go = orc.gradient(pb, th[i], Cs[i])
        share = PY.gradient_shares(orc, pb, th[i], Cs[i], Eo)
        feller = 2 * th[i][0] * th[i][1] >= th[i][2] ** 2
        ey = PY.ey_err(Ey[i], Eo)
        scale = np.maximum(np.abs(go), 1e-3 * np.max(np.abs(go)))
        rel = np.abs(g[i] - go) / scale
        ok = share <= PY.SHARE_GATE
        say(f"  instance {i}: P={pb.n_paths} N={pb.n_steps} m={pb.n_instr} feller={feller} Ey {ey:.2e}; "
            f"grad per component {np.array2string(rel, precision=2)} shares {np.array2string(share, precision=3)}")
        if feller:
            assert ey <= PY.EY_TOL_FP32
        assert np.all(rel[ok] <= PY.GRAD_TOL_FP32)
        assert np.all(np.isfinite(g[i]))
        asserted += int(ok.sum())
    assert asserted >= 10
