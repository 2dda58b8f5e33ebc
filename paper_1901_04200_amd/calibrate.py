"""Calibration by gradient descent on G (the use the paper's title names).

One step: theta' = Proj_box(theta - alpha D grad G), with D = diag of the
squared box widths (so every coordinate moves on the scale of its box), and
Armijo backtracking on G: accept when G(theta') <= G(theta) + c grad.(theta' - theta).
The objective is any callable pair (value, value_and_grad); the Monte Carlo
one below evaluates G and grad G with the library's two-pass gradient.
Optional constraint: Feller's condition 2 kappa theta_bar >= xi^2 for Heston,
enforced by lowering xi.
"""
from __future__ import annotations

import dataclasses
import json
import math
from typing import Callable, List, Optional, Tuple

import numpy as np


@dataclasses.dataclass
class StepLog:
    it: int
    G: float
    grad_norm: float
    alpha: float
    accepted: bool
    n_evals: int
    source: str = "mc"
    note: str = ""


@dataclasses.dataclass
class Result:
    theta: np.ndarray
    G: float
    history: List[StepLog]
    status: str


def project(theta, lo, hi, feller: bool = False):
    th = np.minimum(np.maximum(np.asarray(theta, dtype=np.float64), lo), hi)
    if feller:
        xi_max = math.sqrt(max(2.0 * th[0] * th[1], 0.0))
        th[2] = min(th[2], max(xi_max, lo[2]))
    return th


def calibrate(value_and_grad: Callable[[np.ndarray], Tuple[float, np.ndarray]],
              value: Callable[[np.ndarray], float], theta0, lo, hi, *, max_iter: int = 50,
              alpha0: float = 1.0, c_armijo: float = 1e-4, shrink: float = 0.5, max_backtracks: int = 20,
              g_tol: float = 0.0, rel_tol: float = 1e-12, feller: bool = False,
              log: Optional[List[StepLog]] = None, jsonl_path: Optional[str] = None) -> Result:
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    D = (hi - lo) ** 2
    theta = project(theta0, lo, hi, feller)
    hist = log if log is not None else []
    G, g = value_and_grad(theta)
    alpha = alpha0 / max(float(np.max(np.abs(D * g))), 1e-300) * float(np.min(hi - lo)) * 0.1
    status = "max_iter"
    fh = open(jsonl_path, "a") if jsonl_path else None
    try:
        for it in range(max_iter):
            if not (np.isfinite(G) and np.all(np.isfinite(g))):
                status = "non_finite"
                break
            if G <= g_tol:
                status = "converged"
                break
            a = alpha
            accepted = False
            evals = 0
            for _ in range(max_backtracks):
                cand = project(theta - a * D * g, lo, hi, feller)
                step = cand - theta
                if not np.any(step):
                    break
                Gc = value(cand)
                evals += 1
                if np.isfinite(Gc) and Gc <= G + c_armijo * float(g @ step):
                    accepted = True
                    break
                a *= shrink
            rec = StepLog(it, float(G), float(np.linalg.norm(g)), a, accepted, evals)
            hist.append(rec)
            if fh:
                fh.write(json.dumps(dataclasses.asdict(rec)) + "\n")
            if not accepted:
                status = "line_search_failed"
                break
            G_old = G
            theta = cand
            G, g = value_and_grad(theta)
            alpha = a / shrink          # try a larger step next time
            if abs(G_old - G) <= rel_tol * max(G_old, 1e-300):
                status = "stalled"
                break
    finally:
        if fh:
            fh.close()
    return Result(theta=theta, G=float(G), history=hist, status=status)


class MonteCarloObjective:
    """G and grad G of one problem through the library (device-resident
    targets; theta crosses to the device per call)."""

    def __init__(self, mc, targets):
        import torch
        self.mc = mc
        self.C = torch.as_tensor(np.asarray(targets, dtype=np.float64), device=mc.device)
        self.n_grad = 0
        self.n_value = 0

    def value_and_grad(self, theta):
        Ey, G, g = self.mc.gradient(theta, self.C)
        self.n_grad += 1
        return float(G.item()), g.cpu().numpy()

    def value(self, theta):
        import torch
        Ey = self.mc.forward(theta)
        self.n_value += 1
        return float(0.5 * torch.sum((Ey - self.C) ** 2).item())
