"""Error metrics and conditioning of a GPU result against the FP64 oracle.

TEST INFRASTRUCTURE ONLY, like the rest of this package: used by the tests,
the smoke check and the benchmark's oracle leg.  Nothing here computes any
part of the method; it compares results and measures how well a Monte Carlo
sum is conditioned.

Tolerances of the parity bounds (relative):
  E y   max_i |dEy_i| / max(|Ey_i|, 1e-2)                          <= 1e-5 (FP32 state)
  grad  max_j |dg_j| / max(|g_j|, 1e-3 max_k |g_k|)  (per component) <= 1e-4 (FP32 state)
The per-component form also catches errors in small gradient components
(rho and v0 of Heston, most nodes of a grid model) that a bound relative to
the largest component would hide.

Conditioning gate: an FP32 result is held to the bound where no single path
carries more than SHARE_GATE of the column (the one-path share).  Paths
whose variance nears zero carry the largest contributions and also follow
their FP64 trajectories least closely (percent-level differences in the
pathwise derivative), so the share bounds how far one such path can move a
component: 2% of a percent is the 1e-4 bound.  Measured: Heston Jacobian
columns at 2^16 paths with shares 4.6% and 13% were off by 1.5e-3 and 2e-3,
those with shares up to 1.8% by at most 4.4e-5.
"""
from __future__ import annotations

import numpy as np

EY_TOL_FP32 = 1e-5
GRAD_TOL_FP32 = 1e-4
SHARE_GATE = 0.02   # above: one path carries more than 2% of a column


def ey_err(got, ref) -> float:
    got, ref = np.asarray(got, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-2)))


def grad_err_inf(got, ref) -> float:
    """max_j |dg_j| / max_j |g_j|."""
    got, ref = np.asarray(got, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref)) / max(float(np.max(np.abs(ref))), 1e-300))


def grad_err(got, ref, floor: float = 1e-3) -> float:
    """max_j |dg_j| / max(|g_j|, floor * max_k |g_k|): per-component relative
    error, each component measured against itself unless it is below `floor`
    of the largest."""
    got, ref = np.asarray(got, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    scale = np.maximum(np.abs(ref), floor * max(float(np.max(np.abs(ref))), 1e-300))
    return float(np.max(np.abs(got - ref) / scale))


def one_path_share(per_path) -> np.ndarray:
    """Conditioning of a sum over paths, per column: the largest absolute
    contribution of a single path over the absolute value of the column's
    total.  Near 0 for a well-averaged Monte Carlo sum; near or above 1 when
    a handful of paths decide it (then last-bit differences between two
    correct implementations along those paths decide the result too)."""
    a = np.asarray(per_path, dtype=np.float64)
    a = a.reshape(a.shape[0], -1)
    tot = np.abs(a.sum(axis=0))
    return np.abs(a).max(axis=0) / np.maximum(tot, 1e-300)


def gradient_shares(O, pb, theta, C, Ey=None) -> np.ndarray:
    """One-path share of every component of the gradient of G at theta:
    the oracle's per-path reverse sweeps seeded with E y - C."""
    if Ey is None:
        Ey = O.forward(pb, theta)
    _, gp = O.vjp(pb, theta, np.asarray(Ey) - np.asarray(C), per_path=True)
    return one_path_share(gp)


def jacobian_shares(dy_paths) -> np.ndarray:
    """One-path share of every entry of the Jacobian of E y ([P, m, M] per-path
    derivatives from the oracle's tangent mode), as an [m, M] array."""
    d = np.asarray(dy_paths)
    return one_path_share(d.reshape(d.shape[0], -1)).reshape(d.shape[1:])
