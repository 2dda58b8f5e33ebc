"""Pins for the oracle on Heston stochastic local volatility.

With the leverage function identically c the model is Heston with
(kappa, c^2 theta_bar, c xi, rho, c^2 v0) path by path (v scales by c^2, the
spot's diffusion L sqrt(v) stays the same), so prices match the oracle's
independent Heston sweep and the derivatives follow by the chain rule (the
leverage weights of a step sum to one, so the node derivatives sum to
d/dc).  A leverage that varies only in time gives, at xi = 0 and v0 =
theta_bar, Gaussian log-prices with a known variance (Black-Scholes at the
integrated variance).  The piecewise-constant time rows and the linear spot
weights are checked on one step against their definition; the derivatives
agree with the complex step, tangent mode and central differences.
"""
import math

import numpy as np
import pytest

from paper_1901_04200_amd import workloads as W


def _small_slv(n_paths=1 << 11, n_t=3, n_k=5, seed=3):
    t_nodes = np.array([0.25, 0.5, 1.0])[:n_t]
    k_nodes = np.linspace(70.0, 130.0, n_k)
    N = 32
    steps = np.array([8, 16, 32], dtype=np.int32)
    strikes = np.array([80.0, 95.0, 100.0, 110.0, 125.0])
    pb = W.Problem(model=W.MODEL_SLV, n_params=5 + n_t * n_k, n_steps=N, n_paths=n_paths, t_max=1.0,
                   instr_step=np.repeat(steps, len(strikes)), instr_strike=np.tile(strikes, len(steps)),
                   seed=seed, t_nodes=t_nodes, k_nodes=k_nodes)
    hd = W.heston_feller_draws(31, 2)
    rng = np.random.default_rng(32)
    lev0 = rng.uniform(0.7, 1.3, n_t * n_k)
    lev1 = rng.uniform(0.7, 1.3, n_t * n_k)
    return pb, np.concatenate([hd[0], lev0]), np.concatenate([hd[1], lev1])


def _heston_of(pb):
    return pb.with_(model=W.MODEL_HESTON, n_params=5, t_nodes=None, k_nodes=None)


@pytest.mark.parametrize("c", [1.0, 0.8, 1.3])
def test_constant_leverage_is_heston(orc, c):
    pb, th, _ = _small_slv(n_paths=1 << 12)
    kap, thb, xi, rho, v0 = th[:5]
    slv = np.concatenate([th[:5], np.full(pb.n_params - 5, c)])
    hes = np.array([kap, c * c * thb, c * xi, rho, c * c * v0])
    Ey_s, J_s = orc.jacobian(pb, slv)
    Ey_h, J_h = orc.jacobian(_heston_of(pb), hes)
    np.testing.assert_allclose(Ey_s, Ey_h, rtol=1e-11, atol=1e-12)
    scale = np.max(np.abs(J_h))
    # Heston columns by the chain rule through (c^2 theta_bar, c xi, c^2 v0)
    ref = np.stack([J_h[:, 0], c * c * J_h[:, 1], c * J_h[:, 2], J_h[:, 3], c * c * J_h[:, 4]], axis=1)
    assert np.max(np.abs(J_s[:, :5] - ref)) <= 1e-9 * scale
    # the node columns sum to d/dc
    dc = 2 * c * thb * J_h[:, 1] + xi * J_h[:, 2] + 2 * c * v0 * J_h[:, 4]
    assert np.max(np.abs(J_s[:, 5:].sum(axis=1) - dc)) <= 1e-9 * scale


def test_time_only_leverage_matches_black_scholes(orc):
    """xi = 0, v0 = theta_bar: v stays theta_bar, the spot's volatility is
    L_a sqrt(theta_bar) on row a's time, so prices are Black-Scholes at the
    integrated variance (4 standard errors)."""
    pb, _, _ = _small_slv(n_paths=1 << 16)
    rows = np.array([0.9, 1.25, 0.7])
    thb = 0.05
    th = np.concatenate([[2.0, thb, 0.0, -0.5, thb], np.repeat(rows, len(pb.k_nodes))])
    Ey, yp = orc.forward(pb, th, per_path=True)
    se = yp.std(axis=0, ddof=1) / math.sqrt(pb.n_paths)
    h = pb.t_max / pb.n_steps
    tn = np.arange(pb.n_steps) * h
    a = np.minimum(np.searchsorted(pb.t_nodes, tn, side="right"), len(rows) - 1)
    cum = np.concatenate([[0.0], np.cumsum(rows[a] ** 2 * thb * h)])
    ref = np.array([W.bs_call(pb.s0, K, pb.rate, st * h, math.sqrt(cum[st] / (st * h)))
                    for K, st in zip(pb.instr_strike, pb.instr_step)]).ravel()
    assert np.all(np.abs(Ey - ref) < 4 * se), np.abs(Ey - ref) / se


@pytest.mark.parametrize("t_first,s0", [(0.0, 83.0), (0.05, 100.0), (0.1, 112.5), (0.3, 60.0), (0.6, 140.0),
                                         (1.0, 130.0)])
def test_leverage_weights_one_step(orc, t_first, s0):
    """One step starting at t = t_first (the first node shifted so that the
    step's time is t_first relative to it), a call struck at ~0: the node
    columns of the Jacobian, normalised, are the row's linear weights at S0."""
    t_nodes = np.array([0.2, 0.5, 0.9]) - t_first
    k_nodes = np.array([70.0, 85.0, 100.0, 115.0, 130.0])
    pb = W.Problem(model=W.MODEL_SLV, n_params=5 + 15, n_steps=1, n_paths=1, t_max=0.01,
                   instr_step=np.array([1], dtype=np.int32), instr_strike=np.array([1e-9]),
                   s0=s0, seed=5, t_nodes=t_nodes, k_nodes=k_nodes)
    lev = np.random.default_rng(2).uniform(0.7, 1.3, 15)
    th = np.concatenate([[2.0, 0.05, 0.3, -0.5, 0.04], lev])
    _, J = orc.jacobian(pb, th)
    w = J[0, 5:] / J[0, 5:].sum()
    a = min(int(np.sum(t_nodes <= 0.0)), 2)
    Sc = np.clip(s0, k_nodes[0], k_nodes[-1])
    b = min(max(int(np.searchsorted(k_nodes, Sc, side="right")) - 1, 0), 3)
    be = (Sc - k_nodes[b]) / (k_nodes[b + 1] - k_nodes[b])
    ref = np.zeros(15)
    ref[a * 5 + b] += 1 - be
    ref[a * 5 + b + 1] += be
    np.testing.assert_allclose(w, ref, atol=1e-12)


def test_adjoint_matches_complex_step(orc):
    pb, th, tt = _small_slv()
    C = orc.forward(pb, tt)
    Ey, G, g = orc.gradient(pb, th, C)
    for j in range(pb.n_params):
        re, im = orc.forward_cstep(pb, th, j, 1e-30)
        gcs = np.sum((Ey - C) * im / 1e-30)
        assert abs(g[j] - gcs) <= 1e-11 * np.max(np.abs(g)), (j, g[j], gcs)


def test_gradient_identity_with_tangent_mode(orc):
    pb, th, tt = _small_slv()
    C = orc.forward(pb, tt)
    Ey, G, g = orc.gradient(pb, th, C)
    Ey2, J = orc.jacobian(pb, th)
    np.testing.assert_allclose(Ey2, Ey, rtol=1e-13, atol=1e-15)
    assert np.max(np.abs(g - (Ey - C) @ J)) <= 1e-12 * np.max(np.abs(g))


def test_central_fd_common_random_numbers(orc):
    """h = 1e-7 central differences on the Heston parameters and 6 nodes.
    The sample functional has kinks (payoffs, the truncation of v, the
    leverage's slope changes at spot nodes) that a wider step straddles on
    some paths (at h = 1e-5 the theta_bar column is off by 0.2%); at 1e-7 the
    differences agree with the adjoint to 5e-8 of the largest component."""
    pb, th, tt = _small_slv(n_paths=1 << 12)
    C = orc.forward(pb, tt)
    _, _, g = orc.gradient(pb, th, C)
    coords = list(range(5)) + list(5 + np.random.default_rng(5).choice(pb.n_params - 5, size=6, replace=False))
    for j in coords:
        e = np.zeros(pb.n_params)
        e[j] = 1e-7
        fd = (0.5 * np.sum((orc.forward(pb, th + e) - C) ** 2)
              - 0.5 * np.sum((orc.forward(pb, th - e) - C) ** 2)) / 2e-7
        assert abs(fd - g[j]) < 1e-5 * np.max(np.abs(g)), (j, fd, g[j])
