"""Pins for the surrogate oracle: the input Jacobian against central
differences of the forward, and the double-backprop weight gradient against
torch.autograd in FP64 on the CPU (a library routine) and central
differences of the loss."""
import numpy as np
import pytest

from oracle import mlp_oracle as MO

SIZES = [5, 16, 12, 9, 7]


@pytest.fixture(scope="module")
def case():
    rng = np.random.default_rng(1)
    params = MO.init_params(SIZES, 3)
    params = [(W, rng.normal(0, 0.1, b.shape)) for W, b in params]
    X = rng.uniform(-1, 1, (6, 5))
    Yl = rng.normal(0, 1, (6, 7))
    Jl = rng.normal(0, 1, (6, 7, 5))
    return params, X, Yl, Jl


def test_silu_derivatives():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    np.testing.assert_allclose(MO.dsilu(z), (MO.silu(z + h) - MO.silu(z - h)) / (2 * h), atol=1e-9)
    np.testing.assert_allclose(MO.d2silu(z), (MO.dsilu(z + h) - MO.dsilu(z - h)) / (2 * h), atol=1e-8)


def test_jacobian_matches_central_differences(case):
    params, X, _, _ = case
    Y, J = MO.forward_tangent(params, X)
    h = 1e-6
    for j in range(5):
        e = np.zeros(5)
        e[j] = h
        fd = (MO.forward_tangent(params, X + e)[0] - MO.forward_tangent(params, X - e)[0]) / (2 * h)
        np.testing.assert_allclose(J[:, :, j], fd, atol=1e-8)


@pytest.mark.parametrize("weighted", [False, True])
def test_grads_match_torch_autograd(case, weighted):
    """Unweighted, and with per-sample Jacobian-term weights (some zero)."""
    torch = pytest.importorskip("torch")
    params, X, Yl, Jl = case
    w = 0.7
    jw = np.array([1.0, 0.0, 0.5, 1.0, 0.0, 2.0]) if weighted else None
    L, g = MO.grads(params, X, Yl, Jl, w, jw=jw)
    tp = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in params]
    Xt = torch.tensor(X, requires_grad=True)

    def net(x):
        h = x
        for l, (W, b) in enumerate(tp):
            h = h @ W + b
            if l < len(tp) - 1:
                h = torch.nn.functional.silu(h)
        return h

    Y = net(Xt)
    cols = [torch.autograd.grad(Y[:, i].sum(), Xt, create_graph=True)[0] for i in range(Y.shape[1])]
    J = torch.stack(cols, dim=1)                       # [B, m, n_in]
    c = torch.ones(len(X), dtype=torch.float64) if jw is None else torch.tensor(jw)
    Lt = torch.mean((Y - torch.tensor(Yl)) ** 2) + w * torch.mean(c[:, None, None] * (J - torch.tensor(Jl)) ** 2)
    Lt.backward()
    assert abs(L - Lt.item()) < 1e-13 * abs(L)
    for (dW, db), (W, b) in zip(g, tp):
        np.testing.assert_allclose(dW, W.grad.numpy(), rtol=1e-11, atol=1e-14)
        np.testing.assert_allclose(db, b.grad.numpy(), rtol=1e-11, atol=1e-14)


def test_grads_match_central_differences(case):
    params, X, Yl, Jl = case
    w = 1.3
    _, g = MO.grads(params, X, Yl, Jl, w)
    rng = np.random.default_rng(4)
    h = 1e-6
    for _ in range(20):
        l = int(rng.integers(len(params)))
        W, b = params[l]
        i, j = int(rng.integers(W.shape[0])), int(rng.integers(W.shape[1]))
        Wp, Wm = W.copy(), W.copy()
        Wp[i, j] += h
        Wm[i, j] -= h
        pp = list(params)
        pp[l] = (Wp, b)
        Lp = MO.loss(pp, X, Yl, Jl, w)
        pp[l] = (Wm, b)
        Lm = MO.loss(pp, X, Yl, Jl, w)
        assert abs((Lp - Lm) / (2 * h) - g[l][0][i, j]) < 1e-7 * max(1.0, abs(g[l][0][i, j]))


def test_grad_magnitudes_bound_the_gradient_and_its_rounding():
    """The running-error magnitudes dominate the gradient (triangle
    inequality) and bound what rounding every activation and adjoint to a
    coarse grid (relative 2^-7) does to it, at a small multiple of 2^-7."""
    rng = np.random.default_rng(2)
    params = MO.init_params([3, 16, 16, 16, 4], 1)
    params = [(W, rng.normal(0, 0.1, b.shape)) for W, b in params]
    X = rng.uniform(-1, 1, (32, 3))
    Yl, Jl = rng.normal(0, 1, (32, 4)), rng.normal(0, 1, (32, 4, 3))
    L, g = MO.grads(params, X, Yl, Jl, 0.7)
    mag = MO.grad_magnitudes(params, X, Yl, Jl, 0.7)
    for (dW, db), (mW, mb) in zip(g, mag):
        assert np.all(mW >= np.abs(dW) * (1 - 1e-12)) and np.all(mb >= np.abs(db) * (1 - 1e-12))
    # perturb every weight by a relative 2^-7 (a stand-in for coarse rounding):
    # the gradient moves by far less than 16 x 2^-7 x the magnitude
    u = 2.0 ** -7
    pert = [(W * (1 + u * rng.choice([-1, 1], W.shape)), b) for W, b in params]
    _, g2 = MO.grads(pert, X, Yl, Jl, 0.7)
    for (dW, db), (eW, eb), (mW, mb) in zip(g, g2, mag):
        assert np.all(np.abs(eW - dW) <= 16 * u * mW) and np.all(np.abs(eb - db) <= 16 * u * mb)
