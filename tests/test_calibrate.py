"""The calibration-step drivers, run against the CPU oracle or closed-form
functions as objectives (no GPU): projected L-BFGS and plain projected
descent recover the Black-Scholes sigma that zeroes the sample gradient and
the minimiser of functions whose minimiser is known, box and Feller
projections hold, failures are reported; the surrogate-assisted trust-region
iteration converges with a deliberately wrong model and never accepts a step
that raises G."""
import numpy as np
import pytest

from paper_1901_04200_amd import calibrate as K
from paper_1901_04200_amd import workloads as W


class OracleObjective:
    def __init__(self, orc, pb, C):
        self.orc, self.pb, self.C = orc, pb, np.asarray(C)

    def value_and_grad(self, th):
        Ey, G, g = self.orc.gradient(self.pb, th, self.C)
        return G, g

    def value(self, th):
        return 0.5 * float(np.sum((self.orc.forward(self.pb, th) - self.C) ** 2))


@pytest.mark.parametrize("method", ["lbfgs", "gd"])
def test_bs_calibration_reaches_stationary_point(orc, method):
    pb, th, C = W.bs_problem(n_paths=1 << 12)
    obj = OracleObjective(orc, pb, C)
    res = K.calibrate(obj.value_and_grad, obj.value, th, [0.05], [1.0], max_iter=40, method=method)
    assert res.status in ("stalled", "max_iter", "converged", "stationary")
    _, _, g = orc.gradient(pb, res.theta, C)
    _, _, g0 = orc.gradient(pb, th, C)
    assert abs(g[0]) < 1e-3 * abs(g0[0])
    assert 0.22 < res.theta[0] < 0.28          # targets were priced at sigma = 0.25
    Gs = [h.G for h in res.history]
    assert all(b <= a for a, b in zip(Gs, Gs[1:]))   # monotone descent


@pytest.mark.parametrize("method", ["lbfgs", "gd"])
def test_quadratic_with_box(method):
    target = np.array([2.0, -3.0])
    f = lambda th: 0.5 * float(np.sum((th - target) ** 2))
    fg = lambda th: (f(th), th - target)
    res = K.calibrate(fg, f, [0.0, 0.0], [-1.0, -1.0], [1.0, 1.0], max_iter=100, method=method)
    np.testing.assert_allclose(res.theta, [1.0, -1.0], atol=1e-9)


def test_lbfgs_rosenbrock():
    """An ill-conditioned curved valley (Rosenbrock, minimiser (1, 1) inside
    the box): L-BFGS reaches it to 1e-6 where plain descent does not in the
    same number of gradients."""
    f = lambda t: float(100.0 * (t[1] - t[0] ** 2) ** 2 + (1.0 - t[0]) ** 2)
    g = lambda t: np.array([-400.0 * t[0] * (t[1] - t[0] ** 2) - 2.0 * (1.0 - t[0]), 200.0 * (t[1] - t[0] ** 2)])
    fg = lambda t: (f(t), g(t))
    res = K.calibrate(fg, f, [-1.2, 1.0], [-2.0, -2.0], [2.0, 2.0], max_iter=300, g_tol=1e-14)
    np.testing.assert_allclose(res.theta, [1.0, 1.0], atol=1e-6)
    gd = K.calibrate(fg, f, [-1.2, 1.0], [-2.0, -2.0], [2.0, 2.0], max_iter=300, g_tol=1e-14, method="gd")
    assert res.n_grad < 150 and gd.G > 1e3 * res.G


def test_lbfgs_bound_constrained_least_squares():
    """A linear least-squares problem whose unconstrained minimiser leaves
    the box: the driver stops at the box-constrained minimiser, which
    scipy's bounded least-squares solver (a library routine) gives."""
    from scipy.optimize import lsq_linear
    rng = np.random.default_rng(3)
    A = rng.standard_normal((30, 5)) @ np.diag([1, 3, 10, 30, 100.0])
    b = rng.standard_normal(30) * 50
    lo, hi = -np.ones(5) * 0.2, np.ones(5) * 0.3
    fg = lambda t: (0.5 * float((A @ t - b) @ (A @ t - b)), A.T @ (A @ t - b))
    res = K.calibrate(fg, None, np.zeros(5), lo, hi, max_iter=500, pg_tol=1e-12)
    ref = lsq_linear(A, b, bounds=(lo, hi), tol=1e-14, method="bvls").x
    np.testing.assert_allclose(res.theta, ref, atol=1e-7)
    assert res.status in ("stationary", "stalled")


def test_heston_oracle_calibration_lbfgs(orc):
    """Heston (64 steps, 2^14 paths, oracle objective): from the first of a
    pair of Feller draws to targets priced at the second, L-BFGS lowers G
    by three orders of magnitude in a few dozen gradients, monotonically."""
    pb, _, _, eps = W.heston_problem(n_paths=1 << 14, n_steps=64)
    a, b = W.heston_feller_draws(11, 2)
    C = W.noisy_targets(orc.forward(pb.with_(seed=2), b), eps)
    obj = OracleObjective(orc, pb, C)
    G0 = obj.value_and_grad(a)[0]
    res = K.calibrate(obj.value_and_grad, obj.value, a, W.HESTON_LO, W.HESTON_HI, g_tol=1e-3 * G0, feller=True,
                      max_iter=60)
    assert res.status == "converged" and res.n_grad <= 40, (res.status, res.n_grad)
    Gs = [h.G for h in res.history] + [res.G]
    assert all(y <= x for x, y in zip(Gs, Gs[1:]))


def test_feller_projection():
    lo, hi = W.HESTON_LO, W.HESTON_HI
    th = np.array([1.0, 0.02, 0.9, -0.5, 0.05])
    p = K.project(th, lo, hi, feller=True)
    assert 2 * p[0] * p[1] >= p[2] ** 2 - 1e-15
    assert np.all(p >= lo) and np.all(p <= hi)
    np.testing.assert_array_equal(np.delete(p, 2), np.delete(th, 2))


def test_non_finite_gradient_stops():
    fg = lambda th: (1.0, np.array([np.nan]))
    res = K.calibrate(fg, lambda th: 1.0, [0.5], [0.0], [1.0])
    assert res.status == "non_finite"


@pytest.mark.parametrize("method", ["lbfgs", "gd"])
def test_line_search_failure_reported(method):
    # gradient points uphill: no step satisfies Armijo
    fg = lambda th: (float(th[0] ** 2), np.array([-1.0]))
    res = K.calibrate(fg, lambda th: float(th[0] ** 2), [0.5], [0.0], [1.0], method=method)
    assert res.status == "line_search_failed"


class ToyPricing:
    """Prices y(t) = A tanh(t) + B t^2 (40 instruments, 5 parameters) and a
    deliberately wrong model of them: 2 % too large plus a smooth parameter-
    dependent offset (the surrogate's role)."""

    def __init__(self, seed=0):
        rng = np.random.default_rng(seed)
        self.A = rng.standard_normal((40, 5))
        self.B = 0.3 * rng.standard_normal((40, 5))
        self.t_target = rng.uniform(-0.5, 0.5, 5)
        self.C = self.prices(self.t_target) + 1e-3 * rng.standard_normal(40)
        self.theta0 = rng.uniform(-0.9, 0.9, 5)
        self.calls = 0

    def prices(self, t):
        return self.A @ np.tanh(t) + self.B @ (t ** 2)

    def jac(self, t):
        return self.A * (1 - np.tanh(t) ** 2)[None, :] + self.B * (2 * t)[None, :]

    def mc(self, t):
        self.calls += 1
        y = self.prices(t)
        return y, 0.5 * float((y - self.C) @ (y - self.C)), self.jac(t).T @ (y - self.C)

    def sur_prices(self, t):
        return 1.02 * self.prices(t) + 0.05 * np.sin(3 * t).sum()

    def sur_jac(self, t):
        return 1.02 * self.jac(t) + 0.05 * 3 * np.cos(3 * t)[None, :] * np.ones((40, 1))

    def sur_eval(self, ts, Cp):
        Y = np.array([self.sur_prices(t) for t in ts])
        J = np.array([self.sur_jac(t) for t in ts])
        r = Y - Cp[None, :]
        return Y, J, 0.5 * np.sum(r * r, axis=1), np.einsum("bij,bi->bj", J, r)


def test_trust_region_with_wrong_model_converges():
    from paper_1901_04200_amd import surrogate as S
    T = ToyPricing()
    lo, hi = -np.ones(5), np.ones(5)
    G0 = T.mc(T.theta0)[1]
    T.calls = 0
    th, recs = S.trust_region_calibration(T.mc, T.sur_eval, T.C, T.theta0, lo, hi, iters=40, g_stop=1e-5 * G0,
                                          feller=False)
    Gs = [G0] + [r.G_mc for r in recs]
    assert Gs[-1] <= 1e-5 * G0
    assert all(y <= x for x, y in zip(Gs, Gs[1:]))        # the judge never accepts a rise
    res = K.calibrate(lambda t: T.mc(t)[1:], None, T.theta0, lo, hi, g_tol=1e-5 * G0, max_iter=200)
    assert T.calls - res.n_grad < res.n_grad               # fewer Monte Carlo calls than L-BFGS alone


def test_trust_region_first_step_uses_exact_gradient():
    """With a model that is useless (constant prices, zero Jacobian), the
    corrected model is the linearisation of G at the current point: every
    accepted step still lowers G, as projected gradient steps would, and the
    Monte Carlo L-BFGS fallback takes over after rejections."""
    from paper_1901_04200_amd import surrogate as S
    T = ToyPricing(1)
    lo, hi = -np.ones(5), np.ones(5)

    def flat(ts, Cp):
        Y = np.zeros((len(ts), 40))
        return Y, np.zeros((len(ts), 40, 5)), np.full(len(ts), 0.5 * float(Cp @ Cp)), np.zeros((len(ts), 5))

    G0 = T.mc(T.theta0)[1]
    th, recs = S.trust_region_calibration(T.mc, flat, T.C, T.theta0, lo, hi, iters=30, feller=False)
    Gs = [G0] + [r.G_mc for r in recs]
    assert Gs[-1] < 0.5 * G0 and all(y <= x for x, y in zip(Gs, Gs[1:]))
