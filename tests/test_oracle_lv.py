"""Pins for the oracle on the local-volatility problem (bilinear grid in (t, S)).

A constant grid reproduces the Black-Scholes paths exactly and its node
derivatives sum to the Black-Scholes sigma derivative (bilinear weights are
a partition of unity); a grid that varies only in t gives Gaussian log-prices
with a known variance; the interpolation weights agree with scipy's
RegularGridInterpolator; derivatives agree with the complex step, forward
tangent mode and central differences.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

from paper_1901_04200_amd import workloads as W


def _small_lv(n_paths=1 << 12, n_t=4, n_k=6, seed=3):
    t_nodes = np.linspace(0.25, 1.0, n_t)
    k_nodes = np.linspace(70.0, 130.0, n_k)
    N = 32
    steps = np.array([8, 16, 24, 32], dtype=np.int32)
    strikes = np.array([80.0, 95.0, 100.0, 110.0, 125.0])
    pb = W.Problem(model=W.MODEL_LV, n_params=n_t * n_k, n_steps=N, n_paths=n_paths, t_max=1.0,
                   instr_step=np.repeat(steps, len(strikes)), instr_strike=np.tile(strikes, len(steps)),
                   seed=seed, t_nodes=t_nodes, k_nodes=k_nodes)
    rng = np.random.default_rng(11)
    return pb, rng.uniform(0.1, 0.5, n_t * n_k), rng.uniform(0.1, 0.5, n_t * n_k)


def test_constant_grid_reproduces_black_scholes(orc):
    pb, _, _ = _small_lv(n_paths=1 << 13)
    sig = 0.27
    grid = np.full(pb.n_params, sig)
    bs = pb.with_(model=W.MODEL_BS, n_params=1, t_nodes=None, k_nodes=None)
    np.testing.assert_allclose(orc.forward(pb, grid), orc.forward(bs, np.array([sig])), rtol=1e-13, atol=1e-14)
    C = np.linspace(5.0, 20.0, pb.n_instr)
    _, _, g_lv = orc.gradient(pb, grid, C)
    _, _, g_bs = orc.gradient(bs, np.array([sig]), C)
    assert abs(g_lv.sum() - g_bs[0]) < 1e-12 * abs(g_bs[0])


def test_time_only_grid_matches_black_scholes(orc):
    pb, _, _ = _small_lv(n_paths=1 << 16)
    rows = np.array([0.15, 0.35, 0.22, 0.4])
    grid = np.repeat(rows, len(pb.k_nodes))
    Ey, yp = orc.forward(pb, grid, per_path=True)
    se = yp.std(axis=0, ddof=1) / math.sqrt(pb.n_paths)
    h = pb.t_max / pb.n_steps
    sig_n = np.interp(np.arange(pb.n_steps) * h, pb.t_nodes, rows)
    cum = np.concatenate([[0.0], np.cumsum(sig_n ** 2 * h)])
    ref = np.array([W.bs_call(pb.s0, K, pb.rate, st * h, math.sqrt(cum[st] / (st * h)))
                    for K, st in zip(pb.instr_strike, pb.instr_step)]).ravel()
    assert np.all(np.abs(Ey - ref) < 4 * se), np.abs(Ey - ref) / se


@pytest.mark.parametrize("s0", [50.0, 70.0, 83.0, 100.0, 112.5, 129.9, 130.0, 160.0])
def test_interpolation_weights_match_scipy(orc, s0):
    """One path, one step, a call struck at ~0: row j of the Jacobian is the
    node weight of sigma(0, S0) times a common factor."""
    t_nodes = np.array([-0.5, 0.3, 1.0])
    k_nodes = np.array([70.0, 85.0, 100.0, 115.0, 130.0])
    pb = W.Problem(model=W.MODEL_LV, n_params=15, n_steps=1, n_paths=1, t_max=0.1,
                   instr_step=np.array([1], dtype=np.int32), instr_strike=np.array([1e-9]),
                   s0=s0, seed=5, t_nodes=t_nodes, k_nodes=k_nodes)
    grid = np.random.default_rng(2).uniform(0.1, 0.5, 15)
    _, J = orc.jacobian(pb, grid)
    w = J[0] / J[0].sum()
    q = np.array([[np.clip(0.0, t_nodes[0], t_nodes[-1]), np.clip(s0, k_nodes[0], k_nodes[-1])]])
    ref = np.array([RegularGridInterpolator((t_nodes, k_nodes), np.eye(15)[j].reshape(3, 5))(q)[0]
                    for j in range(15)])
    np.testing.assert_allclose(w, ref, atol=1e-13)


def test_adjoint_matches_complex_step(orc):
    pb, grid, gt = _small_lv(n_paths=1 << 11)
    C = orc.forward(pb, gt)
    Ey, G, g = orc.gradient(pb, grid, C)
    for j in (0, 5, 7, 13, 20, 23):
        re, im = orc.forward_cstep(pb, grid, j, 1e-30)
        gcs = np.sum((Ey - C) * im / 1e-30)
        assert abs(g[j] - gcs) <= 1e-12 * np.max(np.abs(g)), (j, g[j], gcs)


def test_gradient_identity_with_tangent_mode(orc):
    pb, grid, gt = _small_lv(n_paths=1 << 11)
    C = orc.forward(pb, gt)
    Ey, G, g = orc.gradient(pb, grid, C)
    Ey2, J = orc.jacobian(pb, grid)
    np.testing.assert_allclose(Ey2, Ey, rtol=1e-13, atol=1e-15)
    assert np.max(np.abs(g - (Ey - C) @ J)) <= 1e-12 * np.max(np.abs(g))


def test_central_fd_common_random_numbers(orc):
    """h = 1e-4 central differences on 10 random nodes, same seed."""
    pb, grid, gt = _small_lv(n_paths=1 << 13)
    C = orc.forward(pb, gt)
    _, _, g = orc.gradient(pb, grid, C)
    coords = np.random.default_rng(5).choice(pb.n_params, size=10, replace=False)
    for j in coords:
        e = np.zeros(pb.n_params)
        e[j] = 1e-4
        fd = (0.5 * np.sum((orc.forward(pb, grid + e) - C) ** 2)
              - 0.5 * np.sum((orc.forward(pb, grid - e) - C) ** 2)) / 2e-4
        assert abs(fd - g[j]) < 1e-3 * np.max(np.abs(g)), (j, fd, g[j])
