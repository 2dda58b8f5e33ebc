"""FP64 CPU oracle for the learned surrogate (test infrastructure only).

The surrogate is a multilayer perceptron x -> y (x: normalised model
parameters, y: standardised prices) with SiLU hidden activations and a
linear output.  Training uses a price + gradient ("differential") loss, so
the network's input Jacobian J = dy/dx is part of its output and the weight
gradient needs the derivative of J with respect to the weights (double
backpropagation).  This module computes, plainly with numpy:

  forward_tangent(params, X)            -> Y [B, m], J [B, m, n_in]
  loss(params, X, Yl, Jl, w, jw=None)   -> L = mean_{b,i} (Y - Yl)^2
                                               + w mean_{b,i,j} c_b (J - Jl)^2
      (c_b: per-sample weights of the Jacobian term, all 1 by default)
  grads(params, X, Yl, Jl, w)           -> (L, [(dW_l, db_l)])
  grad_magnitudes(params, X, Yl, Jl, w) -> [(|dW_l|, |db_l|)]: the same
      backward pass with every factor replaced by its absolute value (the
      running-error magnitudes of a rounding analysis: a gradient element
      computed with relative rounding u in each factor of each term differs
      from the exact one by at most about (roundings along a term) u times
      this magnitude)

params: list of (W [fan_in, fan_out], b [fan_out]).  SiLU s(z) = z sig(z),
s' = sig (1 + z (1 - sig)), s'' = sig (1 - sig) (2 + z (1 - 2 sig)).
"""
import numpy as np


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * _sig(z)


def dsilu(z):
    s = _sig(z)
    return s * (1.0 + z * (1.0 - s))


def d2silu(z):
    s = _sig(z)
    return s * (1.0 - s) * (2.0 + z * (1.0 - 2.0 * s))


def _forward(params, X):
    """Keeps every layer's input (H, T) and pre-activations (Z, U)."""
    B, n_in = X.shape
    H = np.asarray(X, dtype=np.float64)
    T = np.broadcast_to(np.eye(n_in), (B, n_in, n_in)).copy()   # T[b, t, :] = dH/dx_t
    cache = []
    L = len(params)
    for l, (W, b) in enumerate(params):
        Z = H @ W + b
        U = T @ W                                              # tangent pre-activations
        cache.append((H, T, Z, U))
        if l < L - 1:
            H = silu(Z)
            T = dsilu(Z)[:, None, :] * U
        else:
            H, T = Z, U
    return H, T, cache


def forward_tangent(params, X):
    Y, T, _ = _forward(params, X)
    return Y, np.transpose(T, (0, 2, 1))                       # J[b, i, j] = dY_i/dx_j


def _jw(jw, B):
    return np.ones(B) if jw is None else np.asarray(jw, dtype=np.float64)


def loss(params, X, Yl, Jl, w, jw=None):
    Y, J = forward_tangent(params, X)
    c = _jw(jw, len(X))[:, None, None]
    return float(np.mean((Y - Yl) ** 2) + w * np.mean(c * (J - Jl) ** 2))


def grads(params, X, Yl, Jl, w, jw=None):
    Y, T, cache = _forward(params, X)
    J = np.transpose(T, (0, 2, 1))
    B, m = Y.shape
    n_in = X.shape[1]
    c = _jw(jw, B)[:, None, None]
    L_val = float(np.mean((Y - Yl) ** 2) + w * np.mean(c * (J - Jl) ** 2))
    Hb = 2.0 * (Y - Yl) / (B * m)                              # adjoint of Y
    Tb = np.transpose(2.0 * w * c * (J - Jl) / (B * m * n_in), (0, 2, 1))   # adjoint of T (tangent layout)
    out = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, b = params[l]
        Hin, Tin, Z, U = cache[l]
        if l == len(params) - 1:
            Zb, Ub = Hb, Tb                                    # linear output layer
        else:
            d1, d2 = dsilu(Z), d2silu(Z)
            Zb = Hb * d1 + np.sum(Tb * U, axis=1) * d2
            Ub = Tb * d1[:, None, :]
        dW = Hin.T @ Zb + np.einsum("bti,btj->ij", Tin, Ub)
        db = Zb.sum(axis=0)
        out[l] = (dW, db)
        Hb = Zb @ W.T
        Tb = Ub @ W.T
    return L_val, out


def grad_magnitudes(params, X, Yl, Jl, w, jw=None):
    Y, T, cache = _forward(params, X)
    J = np.transpose(T, (0, 2, 1))
    B, m = Y.shape
    n_in = X.shape[1]
    c = _jw(jw, B)[:, None, None]
    Hb = np.abs(2.0 * (Y - Yl) / (B * m))
    Tb = np.abs(np.transpose(2.0 * w * c * (J - Jl) / (B * m * n_in), (0, 2, 1)))
    out = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, b = params[l]
        Hin, Tin, Z, U = cache[l]
        Hin, Tin, U, Wa = np.abs(Hin), np.abs(Tin), np.abs(U), np.abs(W)
        if l == len(params) - 1:
            Zb, Ub = Hb, Tb
        else:
            d1, d2 = np.abs(dsilu(Z)), np.abs(d2silu(Z))
            Zb = Hb * d1 + np.sum(Tb * U, axis=1) * d2
            Ub = Tb * d1[:, None, :]
        dW = Hin.T @ Zb + np.einsum("bti,btj->ij", Tin, Ub)
        db = Zb.sum(axis=0)
        out[l] = (dW, db)
        Hb = Zb @ Wa.T
        Tb = Ub @ Wa.T
    return out


def init_params(sizes, seed):
    """He-style uniform init (FP64), the same recipe the GPU side uses only
    as a starting point; tests pass explicit weights to both sides."""
    rng = np.random.default_rng(seed)
    ps = []
    for a, c in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / a)
        ps.append((rng.uniform(-lim, lim, (a, c)), np.zeros(c)))
    return ps
