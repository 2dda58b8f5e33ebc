"""Brute-force pin: on tiny inputs (3 paths, 3 steps) the calibration
functional is evaluated in 50-digit arithmetic from the same normals and
differentiated by central differences with h = 1e-20; the oracle's reverse
sweep must agree to FP64 round-off."""
import math

import mpmath as mp
import numpy as np

from paper_1901_04200_amd import workloads as W

mp.mp.dps = 50


def _G_bs(sig, z, pb, C):
    h = mp.mpf(pb.t_max) / pb.n_steps
    sq = mp.sqrt(h)
    r = mp.mpf(pb.rate)
    Ey = [mp.mpf(0)] * pb.n_instr
    for p in range(pb.n_paths):
        x = mp.mpf(0)
        for n in range(pb.n_steps):
            x = x + (r - sig * sig / 2) * h + sig * sq * mp.mpf(z[p][n])
            for i in range(pb.n_instr):
                if pb.instr_step[i] == n + 1:
                    S = pb.s0 * mp.exp(x)
                    Ey[i] += mp.exp(-r * (n + 1) * h) * max(S - mp.mpf(pb.instr_strike[i]), 0)
    return sum((e / pb.n_paths - mp.mpf(c)) ** 2 for e, c in zip(Ey, C)) / 2


def _G_heston(th, z, pb, C):
    kap, thb, xi, rho, v0 = th
    h = mp.mpf(pb.t_max) / pb.n_steps
    sq = mp.sqrt(h)
    r = mp.mpf(pb.rate)
    rhop = mp.sqrt(1 - rho * rho)
    Ey = [mp.mpf(0)] * pb.n_instr
    for p in range(pb.n_paths):
        x, v = mp.mpf(0), v0
        for n in range(pb.n_steps):
            z1, z2 = mp.mpf(z[p][2 * n]), mp.mpf(z[p][2 * n + 1])
            vp = v if v > 0 else mp.mpf(0)
            s = mp.sqrt(vp)
            w = rho * z1 + rhop * z2
            x, v = x + (r - vp / 2) * h + s * sq * z1, v + kap * (thb - vp) * h + xi * s * sq * w
            for i in range(pb.n_instr):
                if pb.instr_step[i] == n + 1:
                    S = pb.s0 * mp.exp(x)
                    Ey[i] += mp.exp(-r * (n + 1) * h) * max(S - mp.mpf(pb.instr_strike[i]), 0)
    return sum((e / pb.n_paths - mp.mpf(c)) ** 2 for e, c in zip(Ey, C)) / 2


def test_bs_bruteforce(orc):
    pb = W.Problem(model=W.MODEL_BS, n_params=1, n_steps=3, n_paths=3, t_max=0.5,
                   instr_step=np.array([2, 3], dtype=np.int32), instr_strike=np.array([97.0, 103.0]), seed=21)
    C = np.array([5.0, 3.0])
    sig = 0.35
    z = [orc.normals(pb.seed, 0, p, 0, pb.n_steps) for p in range(pb.n_paths)]
    _, G, g = orc.gradient(pb, np.array([sig]), C)
    hh = mp.mpf("1e-20")
    s = mp.mpf(sig)
    ref = (_G_bs(s + hh, z, pb, C) - _G_bs(s - hh, z, pb, C)) / (2 * hh)
    assert abs(G - float(_G_bs(s, z, pb, C))) <= 1e-14 * abs(G)
    assert abs(g[0] - float(ref)) <= 1e-13 * abs(float(ref))


def test_heston_bruteforce(orc):
    pb = W.Problem(model=W.MODEL_HESTON, n_params=5, n_steps=3, n_paths=3, t_max=0.75,
                   instr_step=np.array([2, 3, 3], dtype=np.int32),
                   instr_strike=np.array([98.0, 95.0, 104.0]), seed=5)
    C = np.array([4.0, 8.0, 3.0])
    th = np.array([1.3, 0.05, 0.6, -0.55, 0.045])
    z = [orc.normals(pb.seed, 0, p, 0, 2 * pb.n_steps) for p in range(pb.n_paths)]
    _, G, g = orc.gradient(pb, th, C)
    thm = [mp.mpf(t) for t in th]
    assert abs(G - float(_G_heston(thm, z, pb, C))) <= 1e-14 * abs(G)
    hh = mp.mpf("1e-20")
    for j in range(5):
        tp = list(thm)
        tm = list(thm)
        tp[j] += hh
        tm[j] -= hh
        ref = float((_G_heston(tp, z, pb, C) - _G_heston(tm, z, pb, C)) / (2 * hh))
        assert abs(g[j] - ref) <= 1e-12 * max(abs(ref), 1e-3 * np.max(np.abs(g))), (j, g[j], ref)
    assert math.isfinite(G)
