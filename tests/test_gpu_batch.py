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
