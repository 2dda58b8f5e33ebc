"""Calibration by gradient descent on G (the use the paper's title names).

The driver needs only G and grad G, which the library's two-pass gradient
(steps 1-3 of the paper's gradient algorithm, eq. 0711C) delivers together.
It works in box-scaled coordinates u = (theta - lo) / (hi - lo) in [0, 1]^M,
where every parameter moves on the scale of its box.

method="lbfgs" (default): projected limited-memory BFGS.  The direction is
the two-loop recursion -H g over the last `memory` accepted steps, with the
coordinates that sit on a bound and are pushed outward by the gradient held
fixed; the trial point is the projection of u + a d onto the box, accepted by
the Armijo rule on the projected step, halving a otherwise.  A direction
that is not one of descent resets the memory to the scaled gradient.
method="gd": projected gradient steps with Armijo backtracking (the plain
descent of the paper's setting, kept for comparison).

Trial points are judged by `value_and_grad` (one two-pass gradient: its G for
the Armijo test, its gradient for the next direction), since an L-BFGS trial
point is nearly always accepted; `value` (a forward pass) is used only by
the plain descent's backtracking.

Optional constraint: Feller's condition 2 kappa theta_bar >= xi^2 for
Heston, enforced by lowering xi in the projection.
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
    n_grad: int = 0
    n_value: int = 0
    iterates: List[np.ndarray] = dataclasses.field(default_factory=list)


def project(theta, lo, hi, feller: bool = False):
    th = np.minimum(np.maximum(np.asarray(theta, dtype=np.float64), lo), hi)
    if feller:
        xi_max = math.sqrt(max(2.0 * th[0] * th[1], 0.0))
        th[2] = min(th[2], max(xi_max, lo[2]))
    return th


def projected_gradient_norm(u, gu) -> float:
    """|P(u - g) - u|_inf in box-scaled coordinates (0 at a stationary point
    of the box-constrained problem)."""
    return float(np.max(np.abs(np.clip(u - gu, 0.0, 1.0) - u)))


class LbfgsMemory:
    """The last `size` curvature pairs (s, y) and the two-loop recursion."""

    def __init__(self, size: int):
        self.size = size
        self.s: List[np.ndarray] = []
        self.y: List[np.ndarray] = []

    def clear(self):
        self.s.clear()
        self.y.clear()

    def push(self, s, y) -> bool:
        sy = float(s @ y)
        if not (sy > 1e-12 * float(np.linalg.norm(s)) * float(np.linalg.norm(y))):
            return False              # no positive curvature along s: skip the pair
        self.s.append(s.copy())
        self.y.append(y.copy())
        if len(self.s) > self.size:
            self.s.pop(0)
            self.y.pop(0)
        return True

    def apply(self, g, free):
        """-H g on the free coordinates (fixed ones held at 0)."""
        q = np.where(free, g, 0.0)
        alphas = []
        for s, y in zip(reversed(self.s), reversed(self.y)):
            sf, yf = np.where(free, s, 0.0), np.where(free, y, 0.0)
            sy = float(sf @ yf)
            if sy <= 0.0:
                continue
            a = float(sf @ q) / sy
            q = q - a * yf
            alphas.append((a, sf, yf, sy))
        if self.s:
            s, y = np.where(free, self.s[-1], 0.0), np.where(free, self.y[-1], 0.0)
            yy = float(y @ y)
            gamma = float(s @ y) / yy if yy > 0.0 and float(s @ y) > 0.0 else 1.0
        else:
            gamma = 1.0
        r = gamma * q
        for a, sf, yf, sy in reversed(alphas):
            b = float(yf @ r) / sy
            r = r + (a - b) * sf
        return -np.where(free, r, 0.0)


def calibrate(value_and_grad: Callable[[np.ndarray], Tuple[float, np.ndarray]],
              value: Optional[Callable[[np.ndarray], float]], theta0, lo, hi, *, method: str = "lbfgs",
              max_iter: int = 100, memory: int = 8, alpha0: float = 1.0, c_armijo: float = 1e-4,
              shrink: float = 0.5, max_backtracks: int = 20, g_tol: float = 0.0, pg_tol: float = 1e-12,
              rel_tol: float = 1e-12, feller: bool = False, log: Optional[List[StepLog]] = None,
              jsonl_path: Optional[str] = None) -> Result:
    """Minimise G over the box [lo, hi] from theta0.  Stops when G <= g_tol
    ("converged"), the projected gradient is below pg_tol ("stationary"), G
    changed by at most rel_tol relatively over an accepted step ("stalled"),
    no trial point passed the Armijo test ("line_search_failed"), a value
    was not finite ("non_finite"), or after max_iter iterations."""
    if method not in ("lbfgs", "gd"):
        raise ValueError(f"unknown method {method!r}")
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    w = hi - lo
    to_u = lambda th: (th - lo) / w
    to_th = lambda u: lo + w * u
    proj_u = lambda u: to_u(project(to_th(u), lo, hi, feller))

    hist = log if log is not None else []
    counts = {"grad": 0, "value": 0}

    def vg(u):
        counts["grad"] += 1
        G, g = value_and_grad(to_th(u))
        return float(G), np.asarray(g, dtype=np.float64) * w    # gradient in u

    def v(u):
        counts["value"] += 1
        return float(value(to_th(u)))

    u = proj_u(to_u(np.asarray(theta0, dtype=np.float64)))
    G, g = vg(u)
    iterates = [to_th(u)]
    mem = LbfgsMemory(memory)
    gd_alpha = alpha0 * 0.1 / max(float(np.max(np.abs(g))), 1e-300)
    status = "max_iter"
    fh = open(jsonl_path, "a") if jsonl_path else None
    try:
        for it in range(max_iter):
            if not (math.isfinite(G) and np.all(np.isfinite(g))):
                status = "non_finite"
                break
            if G <= g_tol:
                status = "converged"
                break
            if projected_gradient_norm(u, g) <= pg_tol:
                status = "stationary"
                break
            # coordinates held on their bound
            free = ~(((u <= 0.0) & (g > 0.0)) | ((u >= 1.0) & (g < 0.0)))
            if method == "lbfgs":
                d = mem.apply(g, free)
                if not float(g @ d) < 0.0:
                    mem.clear()
                    d = -np.where(free, g, 0.0)
                a = 1.0 if mem.s else min(1.0, 0.1 / max(float(np.max(np.abs(d))), 1e-300))
            else:
                d = -g
                a = gd_alpha
            accepted, evals = False, 0
            Gc = gc = None
            for _ in range(max_backtracks):
                cand = proj_u(u + a * d)
                step = cand - u
                if not np.any(step):
                    break
                if method == "lbfgs":
                    Gc, gc = vg(cand)
                else:
                    Gc = v(cand)
                evals += 1
                if math.isfinite(Gc) and Gc <= G + c_armijo * float(g @ step):
                    accepted = True
                    break
                a *= shrink
            rec = StepLog(it, float(G), float(np.linalg.norm(g / w)), a, accepted, evals)
            hist.append(rec)
            if fh:
                fh.write(json.dumps(dataclasses.asdict(rec)) + "\n")
            if not accepted:
                if method == "lbfgs" and mem.s:
                    mem.clear()        # retry from the scaled gradient before giving up
                    continue
                status = "line_search_failed"
                break
            G_old = G
            if method == "gd":
                Gc, gc = vg(cand)
                gd_alpha = a / shrink   # try a larger step next time
            mem.push(cand - u, gc - g)
            u, G, g = cand, Gc, gc
            iterates.append(to_th(u))
            if abs(G_old - G) <= rel_tol * max(G_old, 1e-300):
                status = "stalled"
                break
    finally:
        if fh:
            fh.close()
    return Result(theta=to_th(u), G=float(G), history=hist, status=status, n_grad=counts["grad"],
                  n_value=counts["value"], iterates=iterates)


class MonteCarloObjective:
    """G and grad G of one problem through the library: theta goes up
    through a pinned buffer, E y, G and grad come back in one copy, one
    synchronisation per call; the targets stay on the device."""

    def __init__(self, mc, targets):
        import torch
        self.torch = torch
        self.mc = mc
        self.C = torch.as_tensor(np.asarray(targets, dtype=np.float64), device=mc.device)
        m, M = mc.m, mc.M
        self.m = m
        self.th_host = torch.empty(M, dtype=torch.float64, pin_memory=True)
        self.th_dev = torch.empty(M, dtype=torch.float64, device=mc.device)
        self.out_dev = torch.empty(m + 1 + M, dtype=torch.float64, device=mc.device)   # E y, G, grad
        self.out_host = torch.empty(m + 1 + M, dtype=torch.float64, pin_memory=True)
        self.n_grad = 0
        self.n_value = 0

    def _run(self, theta, gradient):
        from . import capi
        t, m = self.torch, self.m
        self.th_host.copy_(t.from_numpy(np.asarray(theta, dtype=np.float64)))
        self.th_dev.copy_(self.th_host, non_blocking=True)
        o = self.out_dev
        if gradient:
            capi.calibrate_gradient(self.mc.ctx, self.th_dev, self.C, o[:m], o[m:m + 1], o[m + 1:])
        else:
            capi.calibrate_forward(self.mc.ctx, self.th_dev, o[:m])
        self.out_host.copy_(o, non_blocking=True)
        t.cuda.current_stream().synchronize()
        return self.out_host.numpy().copy()

    def value_and_grad(self, theta):
        out = self._run(theta, True)
        self.n_grad += 1
        return float(out[self.m]), out[self.m + 1:]

    def value(self, theta):
        out = self._run(theta, False)
        self.n_value += 1
        r = out[:self.m] - self.C.cpu().numpy()
        return 0.5 * float(r @ r)

    def prices_value_and_grad(self, theta):
        """(E y, G, grad) in one call (the trust-region iteration's judge)."""
        out = self._run(theta, True)
        self.n_grad += 1
        return out[:self.m], float(out[self.m]), out[self.m + 1:]
