"""Pins for the oracle on the Black-Scholes problem (sigma only, m = 4).

Each pin compares the oracle with something it does not contain:
closed-form prices and vegas, the closed-form calibration gradient, the
complex-step derivative, forward tangent mode, central finite differences
with common random numbers, and the paper's appendix algorithm.
"""
import math

import numpy as np
import pytest

from paper_1901_04200_amd import workloads as W
from tests import pin_helpers as H


@pytest.fixture(scope="module")
def c1():
    return W.bs_problem()


def test_prices_match_closed_form(orc, c1):
    pb, th, _ = c1
    pb = pb.with_(n_paths=1 << 20)
    Ey, yp = orc.forward(pb, th, per_path=True)
    se = yp.std(axis=0, ddof=1) / math.sqrt(pb.n_paths)
    ref = W.bs_call(100.0, pb.instr_strike, 0.02, 1.0, 0.20)
    assert np.all(np.abs(Ey - ref) < 4 * se), (Ey, ref, se)
    # the published-value check at the stated size, 2^14 paths
    Ey14, yp14 = orc.forward(c1[0], th, per_path=True)
    se14 = yp14.std(axis=0, ddof=1) / math.sqrt(c1[0].n_paths)
    assert np.all(np.abs(Ey14 - ref) < 4 * se14)


def test_vega_matches_closed_form(orc, c1):
    pb, th, _ = c1
    pb = pb.with_(n_paths=1 << 18)
    Ey, J, yp, dyp = orc.jacobian(pb, th, per_path=True)
    se = dyp[:, :, 0].std(axis=0, ddof=1) / math.sqrt(pb.n_paths)
    vega = W.bs_vega(100.0, pb.instr_strike, 0.02, 1.0, 0.20)
    assert np.all(np.abs(J[:, 0] - vega) < 4 * se), (J[:, 0], vega, se)


def test_calibration_gradient_matches_closed_form(orc, c1):
    """dG/dsigma = sum_i (BS_i(0.2) - C_i) vega_i(0.2) (paper: gradient formula
    with E outside the derivative), within a delta-method 4-SE band."""
    pb, th, C = c1
    pb = pb.with_(n_paths=1 << 18)
    Ey, G, g = orc.gradient(pb, th, C)
    ref_r = W.bs_call(100.0, pb.instr_strike, 0.02, 1.0, 0.20) - C
    ref = float(np.sum(ref_r * W.bs_vega(100.0, pb.instr_strike, 0.02, 1.0, 0.20)))
    assert abs(ref - (-216.2078591017)) < 1e-6
    _, J, yp, dyp = orc.jacobian(pb, th, per_path=True)
    r = Ey - C
    infl = (yp - Ey) @ J[:, 0] + (dyp[:, :, 0] - J[:, 0]) @ r
    se = infl.std(ddof=1) / math.sqrt(pb.n_paths)
    assert abs(g[0] - ref) < 4 * se, (g[0], ref, se)
    assert abs(G - 0.5 * np.sum(r * r)) < 1e-12 * G


def test_adjoint_matches_complex_step(orc, c1):
    pb, th, C = c1
    Ey, G, g = orc.gradient(pb, th, C)
    hc = 1e-30
    re, im = orc.forward_cstep(pb, th, 0, hc)
    np.testing.assert_allclose(re, Ey, rtol=1e-14, atol=0)
    g_cs = float(np.sum((Ey - C) * im / hc))
    assert abs(g[0] - g_cs) <= 1e-12 * abs(g_cs)


def test_gradient_identity_with_tangent_mode(orc, c1):
    """grad G = sum_i (Ey_i - C_i) grad Ey_i, with grad Ey from tangent mode."""
    pb, th, C = c1
    Ey, G, g = orc.gradient(pb, th, C)
    Ey2, J = orc.jacobian(pb, th)
    np.testing.assert_allclose(Ey2, Ey, rtol=1e-14)
    assert abs(g[0] - (Ey - C) @ J[:, 0]) <= 1e-12 * abs(g[0])


def test_central_fd_common_random_numbers(orc, c1):
    """Central differences of G with the same seed.  With strikes far below
    the spot the payoffs are smooth and the error falls as h^2; at the real
    strikes a path whose S crosses K inside [sigma-h, sigma+h] adds an O(1/P)
    jump, so only agreement at h = 1e-4 is asserted there."""
    pb, th, C = c1
    smooth = pb.with_(instr_strike=np.array([1e-6, 1e-3, 0.1, 1.0]))
    Cs = np.array([90.0, 95.0, 99.0, 101.0])
    _, _, gs = orc.gradient(smooth, th, Cs)
    errs = []
    for h in (1e-2, 1e-3, 1e-4):
        Gp = 0.5 * np.sum((orc.forward(smooth, th + h) - Cs) ** 2)
        Gm = 0.5 * np.sum((orc.forward(smooth, th - h) - Cs) ** 2)
        errs.append(abs((Gp - Gm) / (2 * h) - gs[0]) / abs(gs[0]))
    assert errs[0] / errs[1] > 50 and errs[1] / errs[2] > 50, errs
    assert errs[2] < 1e-8
    _, _, g = orc.gradient(pb, th, C)
    h = 1e-4
    Gp = 0.5 * np.sum((orc.forward(pb, th + h) - C) ** 2)
    Gm = 0.5 * np.sum((orc.forward(pb, th - h) - C) ** 2)
    assert abs((Gp - Gm) / (2 * h) - g[0]) < 1e-4 * abs(g[0])


def test_zero_residual(orc, c1):
    pb, th, _ = c1
    Ey = orc.forward(pb, th)
    Ey2, G, g = orc.gradient(pb, th, Ey)
    assert G == 0.0
    assert g[0] == 0.0


def test_vjp_is_linear_in_lambda(orc, c1):
    pb, th, _ = c1
    lam1 = np.array([1.0, -2.0, 0.5, 3.0])
    lam2 = np.array([0.0, 1.0, 0.0, -1.0])
    g1 = orc.vjp(pb, th, lam1)
    g2 = orc.vjp(pb, th, lam2)
    g12 = orc.vjp(pb, th, 2 * lam1 + lam2)
    assert abs(g12[0] - (2 * g1[0] + g2[0])) < 1e-12 * abs(g12[0])


def test_fries_expected_backward_ad(orc):
    """The two-pass gradient equals the appendix algorithm (expected
    backward AD over an operator list) on a tiny case."""
    P, N = 8, 3
    pb = W.Problem(model=W.MODEL_BS, n_params=1, n_steps=N, n_paths=P, t_max=0.75,
                   instr_step=np.array([2, 3, 3], dtype=np.int32),
                   instr_strike=np.array([95.0, 90.0, 105.0]), seed=9)
    sig = 0.3
    C = np.array([6.0, 11.0, 4.0])
    Ey, G, g = orc.gradient(pb, np.array([sig]), C)
    h = pb.t_max / N
    z = np.stack([orc.normals(pb.seed, 0, p, 0, N) for p in range(P)])  # [P, N]
    T = H.Tape(P)
    s = T.var(sig)
    x = T.const(0.0)
    ys = {}
    for n in range(N):
        drift = T.scale(T.shift(T.scale(T.mul(s, s), -0.5), pb.rate), h)
        diff = T.mul(s, T.const(math.sqrt(h) * z[:, n]))
        x = T.add(T.add(x, drift), diff)
        for i in np.nonzero(pb.instr_step == n + 1)[0]:
            S = T.scale(T.exp(x), pb.s0)
            pay = T.relu(T.shift(S, -pb.instr_strike[i]))
            ys[i] = T.scale(pay, math.exp(-pb.rate * (n + 1) * h))
    Gn = T.const(0.0)
    for i in range(3):
        e = T.shift(T.expect(ys[i]), -C[i])
        Gn = T.add(Gn, T.scale(T.mul(e, e), 0.5))
    assert abs(T.vals[Gn][0] - G) < 1e-12 * G
    (gf,) = T.grad(Gn, [s])
    assert abs(gf - g[0]) < 1e-12 * abs(g[0])
