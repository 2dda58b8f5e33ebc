"""Pins for the oracle on the Heston problem (M = 5, m = 40).

Forward: at xi = 0 the log-Euler scheme is exactly Gaussian, so prices are
Black-Scholes prices at the integrated variance; at xi > 0 the prices match
Heston's characteristic-function price within Monte Carlo error once the
time step is fine.  Derivatives: complex step, forward tangent mode,
central differences, zero residual.
"""
import math

import numpy as np
import pytest

from paper_1901_04200_amd import workloads as W
from tests import pin_helpers as H


def _eff_vol(th, pb):
    """Integrated variance of the deterministic (xi = 0) variance recursion."""
    kap, thb, _, _, v0 = th
    h = pb.t_max / pb.n_steps
    v = v0
    cum = [0.0]
    for n in range(pb.n_steps):
        vp = max(v, 0.0)
        cum.append(cum[-1] + vp * h)
        v = v + kap * (thb - vp) * h
    T = pb.instr_step * h
    return np.sqrt(np.array([cum[s] for s in pb.instr_step]) / T), T


def _bs_eff(th, pb):
    sig, T = _eff_vol(th, pb)
    return np.array([W.bs_call(pb.s0, K, pb.rate, t, s) for K, t, s in zip(pb.instr_strike, T, sig)]).ravel()


def test_xi_zero_prices_match_black_scholes(orc):
    pb, _, _, _ = W.heston_problem(n_paths=1 << 16)
    th = np.array([1.5, 0.06, 0.0, -0.5, 0.03])
    Ey, yp = orc.forward(pb, th, per_path=True)
    se = yp.std(axis=0, ddof=1) / math.sqrt(pb.n_paths)
    ref = _bs_eff(th, pb)
    assert np.all(np.abs(Ey - ref) < 4 * se + 1e-12), np.abs(Ey - ref) / se


def test_xi_zero_jacobian_matches_chain_rule(orc):
    pb, _, _, _ = W.heston_problem(n_paths=1 << 15)
    th = np.array([1.5, 0.06, 0.0, -0.5, 0.03])
    Ey, J, yp, dyp = orc.jacobian(pb, th, per_path=True)
    se = dyp.std(axis=0, ddof=1) / math.sqrt(pb.n_paths)
    for j in (0, 1, 4):   # kappa, theta_bar, v0 act through the integrated variance
        e = np.zeros(5)
        e[j] = 1e-6
        ref = (_bs_eff(th + e, pb) - _bs_eff(th - e, pb)) / 2e-6
        assert np.all(np.abs(J[:, j] - ref) < 4 * se[:, j] + 1e-6), (j, np.abs(J[:, j] - ref) / se[:, j])
    # rho only enters through xi * s * q * w, so its derivative vanishes at xi = 0
    assert np.all(J[:, 3] == 0.0)


def test_xi_positive_prices_match_characteristic_function(orc):
    th = np.array([2.0, 0.04, 0.3, -0.7, 0.04])
    zs = {}
    for N in (64, 256):
        pb, _, _, _ = W.heston_problem(n_paths=1 << 18, n_steps=N)
        Ey, yp = orc.forward(pb, th, per_path=True)
        se = yp.std(axis=0, ddof=1) / math.sqrt(pb.n_paths)
        h = pb.t_max / N
        ref = np.array([H.heston_call(pb.s0, K, pb.rate, st * h, *th)
                        for K, st in zip(pb.instr_strike, pb.instr_step)])
        zs[N] = (Ey - ref) / se
    # at 128 steps per year the Euler bias is inside the Monte Carlo band;
    # at 32 steps per year it is not, and it shrinks as the step is refined
    assert np.abs(zs[256]).max() < 4.0, zs[256]
    assert np.abs(zs[64]).max() > np.abs(zs[256]).max()


@pytest.fixture(scope="module")
def c2_small():
    pb, th0, tht, eps = W.heston_problem(n_paths=1 << 12)
    return pb, th0, tht, eps


def test_adjoint_matches_complex_step(orc, c2_small):
    pb, th0, tht, eps = c2_small
    C = W.noisy_targets(orc.forward(pb, tht), eps)
    Ey, G, g = orc.gradient(pb, th0, C)
    hc = 1e-30
    gcs = np.empty(5)
    for j in range(5):
        re, im = orc.forward_cstep(pb, th0, j, hc)
        np.testing.assert_allclose(re, Ey, rtol=1e-13, atol=1e-15)
        gcs[j] = np.sum((Ey - C) * im / hc)
    assert np.max(np.abs(g - gcs)) <= 1e-12 * np.max(np.abs(gcs)), (g, gcs)
    np.testing.assert_allclose(g, gcs, rtol=1e-10)


def test_gradient_identity_with_tangent_mode(orc, c2_small):
    pb, th0, tht, eps = c2_small
    C = W.noisy_targets(orc.forward(pb, tht), eps)
    Ey, G, g = orc.gradient(pb, th0, C)
    Ey2, J = orc.jacobian(pb, th0)
    np.testing.assert_allclose(Ey2, Ey, rtol=1e-13, atol=1e-15)
    ref = (Ey - C) @ J
    assert np.max(np.abs(g - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_vjp_columns_equal_jacobian_rows(orc, c2_small):
    """calibrate_vjp with lambda = e_i returns row i of the Jacobian."""
    pb, th0, _, _ = c2_small
    _, J = orc.jacobian(pb, th0)
    for i in (0, 13, 39):
        lam = np.zeros(pb.n_instr)
        lam[i] = 1.0
        g = orc.vjp(pb, th0, lam)
        np.testing.assert_allclose(g, J[i], rtol=1e-11, atol=1e-12 * np.abs(J[i]).max())


def test_central_fd_common_random_numbers(orc, c2_small):
    """Central differences with the same seed at a draw that satisfies
    Feller's condition (2 kappa theta_bar > xi^2), where the pathwise
    derivative is well conditioned.  (Where the condition fails badly, a few
    paths whose variance nears zero dominate the exact pathwise gradient and
    no finite difference resolves it; the complex-step pin covers that case.)"""
    pb, th0, tht, eps = c2_small
    pb = pb.with_(n_paths=1 << 14)
    C = W.noisy_targets(orc.forward(pb, th0), eps)
    th = tht
    assert 2 * th[0] * th[1] > th[2] ** 2
    _, _, g = orc.gradient(pb, th, C)
    for j in range(5):
        h = 1e-4 * max(abs(th[j]), 1e-2)
        e = np.zeros(5)
        e[j] = h
        Gp = 0.5 * np.sum((orc.forward(pb, th + e) - C) ** 2)
        Gm = 0.5 * np.sum((orc.forward(pb, th - e) - C) ** 2)
        fd = (Gp - Gm) / (2 * h)
        assert abs(fd - g[j]) < 1e-3 * np.max(np.abs(g)), (j, fd, g[j])


def test_smoothed_square_root_matches_complex_step(orc, c2_small):
    """The optional C1 square root below eps is differentiated consistently."""
    pb, th0, tht, eps = c2_small
    pb = pb.with_(sqrt_eps=1e-3)
    C = W.noisy_targets(orc.forward(pb, tht), eps)
    Ey, G, g = orc.gradient(pb, th0, C)
    gcs = np.array([np.sum((Ey - C) * orc.forward_cstep(pb, th0, j, 1e-30)[1] / 1e-30) for j in range(5)])
    assert np.max(np.abs(g - gcs)) <= 1e-12 * np.max(np.abs(gcs))
    # eps only changes paths whose variance falls below it
    Ey0 = orc.forward(pb.with_(sqrt_eps=0.0), th0)
    assert np.max(np.abs(Ey - Ey0)) < 1e-2 * np.max(Ey0)


def test_zero_residual(orc, c2_small):
    pb, th0, _, _ = c2_small
    Ey = orc.forward(pb, th0)
    _, G, g = orc.gradient(pb, th0, Ey)
    assert G == 0.0
    assert np.all(g == 0.0)
