"""How well FP32 path state can reproduce the local-volatility gradient.

A plain numpy implementation of the local-volatility sweep and its
pathwise reverse sweep (log-Euler, sigma bilinear on the node grid, flat
outside, payoff adjoints at the maturity dates), written here for this test
only and sharing nothing with the library or the oracle, runs twice on the
same normals: in float64 and in float32.  With a smooth node surface the
two gradients agree to ~1e-6 per component; with independent U(0.1, 0.5)
node values the slope of sigma in S jumps by up to 0.08 per unit of spot
between cells, the reverse sweep multiplies the adjoint of x by about
1 + sbar dsigma/dS S per step (factors far from 1), and float32 rounding is
amplified: the per-component error (relative, floor 1e-3 of the largest
component) is ~1e-3 in the median, far above 1e-4, in any FP32
implementation of the exact pathwise gradient.  CPU only; no GPU involved.
"""
import numpy as np

from paper_1901_04200_amd import workloads as W


def lv_gradient(pb, theta, C, dt, Z):
    P, N = Z.shape
    nT, nK = len(pb.t_nodes), len(pb.k_nodes)
    h = pb.t_max / N
    sq = np.sqrt(h)
    K0, dK = pb.k_nodes[0], pb.k_nodes[1] - pb.k_nodes[0]
    tn = pb.t_nodes
    th = np.asarray(theta).reshape(nT, nK)
    f = lambda v: np.asarray(v, dtype=dt)
    cell, al = np.zeros(N, int), np.zeros(N)
    for n in range(N):       # time cell of step n and the weight on its upper row
        t, a = n * h, 0
        while a + 1 < nT - 1 and tn[a + 1] <= t:
            a += 1
        cell[n], al[n] = a, min(max((t - tn[a]) / (tn[a + 1] - tn[a]), 0.0), 1.0)
    dates = set(int(s) for s in pb.instr_step)
    x = np.zeros(P, dt)
    tape, S_at = [], {}
    for n in range(N):
        row = f((1 - al[n]) * th[cell[n]] + al[n] * th[cell[n] + 1])
        S = f(pb.s0) * np.exp(x)
        u = (S - f(K0)) / f(dK)
        b = np.clip(np.floor(u).astype(int), 0, nK - 2)
        be = np.clip(u - b.astype(dt), 0, 1).astype(dt)
        sig = row[b] + be * (row[b + 1] - row[b])
        inside = (S >= K0) & (S <= K0 + (nK - 1) * dK)
        tape.append((S, b, be, sig, np.where(inside, (row[b + 1] - row[b]) / f(dK), f(0))))
        x = x + (f(pb.rate * h) - f(0.5 * h) * sig * sig) + f(sq) * sig * f(Z[:, n])
        if n + 1 in dates:
            S_at[n + 1] = f(pb.s0) * np.exp(x)
    disc = np.exp(-pb.rate * pb.instr_step * h)
    Ey = np.array([np.mean(d * np.maximum(S_at[int(s)].astype(np.float64) - k, 0.0))
                   for s, k, d in zip(pb.instr_step, pb.instr_strike, disc)])
    lam = (Ey - C) / P
    grad = np.zeros(nT * nK)
    xb = np.zeros(P, dt)
    for n in range(N - 1, -1, -1):
        if n + 1 in dates:
            for i in np.where(pb.instr_step == n + 1)[0]:
                Sd = S_at[n + 1]
                xb = xb + np.where(Sd > f(pb.instr_strike[i]), f(lam[i] * disc[i]) * Sd, f(0))
        S, b, be, sig, slope = tape[n]
        sbar = xb * (-sig * f(h) + f(sq) * f(Z[:, n]))
        xb = xb + sbar * slope * S
        w1 = sbar * be
        w0 = sbar - w1
        for a, wa in ((cell[n], 1 - al[n]), (cell[n] + 1, al[n])):
            np.add.at(grad, a * nK + b, (f(wa) * w0).astype(np.float64))
            np.add.at(grad, a * nK + b + 1, (f(wa) * w1).astype(np.float64))
    return Ey, grad


def errors(surface, paths=1 << 14):
    pb, g0, gt, eps, _ = W.lv_problem(n_paths=paths, surface=surface)
    Z = np.random.default_rng(0).standard_normal((pb.n_paths, pb.n_steps))
    C = np.linspace(2.0, 20.0, pb.n_instr)
    E64, g64 = lv_gradient(pb, g0, C, np.float64, Z)
    E32, g32 = lv_gradient(pb, g0, C, np.float32, Z)
    rel = np.abs(g32 - g64) / np.maximum(np.abs(g64), 1e-3 * np.max(np.abs(g64)))
    ey = np.max(np.abs(E32 - E64) / np.maximum(np.abs(E64), 1e-2))
    return ey, rel


def test_smooth_surface_fp32_meets_the_bound():
    ey, rel = errors("smooth")
    assert ey < 1e-5
    assert np.median(rel) < 1e-5 and np.max(rel) < 1e-3


def test_iid_nodes_fp32_cannot():
    ey, rel = errors("iid")
    print(f"iid: E y {ey:.2e}, gradient per component median {np.median(rel):.2e} max {np.max(rel):.2e}")
    assert ey < 1e-5                       # prices are fine
    assert np.median(rel) > 1e-4 and np.max(rel) > 0.1   # the gradient is not, in FP32
