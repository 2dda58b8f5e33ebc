"""Seeded synthetic inputs for the calibration workloads.

This module only draws and lays out inputs: parameter vectors, instrument
tables (maturity step, strike), grids, noise.  It contains none of the
method's arithmetic (no Euler step, no payoff, no derivative), so that both
the GPU library's callers and the CPU oracle's tests can take their inputs
from it.  Every draw uses ``numpy.random.default_rng(seed)``.

The paper's own experiment (a Heston stochastic-local-volatility calibration
with European calls, sizes unstated) has no data to ship; the problems below
stand in for it with the shapes of that experiment.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

MODEL_BS = 0
MODEL_HESTON = 1
MODEL_LV = 2
MODEL_SLV = 3
MODEL_BS_S = 4   # Black-Scholes with the Euler scheme applied to S itself

MODEL_NAMES = {MODEL_BS: "bs", MODEL_HESTON: "heston", MODEL_LV: "lv", MODEL_SLV: "slv", MODEL_BS_S: "bs_s"}

# Heston parameter box: kappa, theta_bar, xi, rho, v0
HESTON_LO = np.array([0.5, 0.01, 0.1, -0.9, 0.01])
HESTON_HI = np.array([5.0, 0.10, 1.0, 0.0, 0.10])
HESTON_NAMES = ("kappa", "theta_bar", "xi", "rho", "v0")


@dataclasses.dataclass
class Problem:
    """One calibration problem: model, discretisation, instruments, paths."""
    model: int
    n_params: int
    n_steps: int
    n_paths: int
    t_max: float
    instr_step: np.ndarray      # int32 [m], maturity step in 1..N
    instr_strike: np.ndarray    # float64 [m]
    s0: float = 100.0
    rate: float = 0.02
    seed: int = 1
    inst: int = 0
    t_nodes: Optional[np.ndarray] = None   # LV grid, time nodes (years)
    k_nodes: Optional[np.ndarray] = None   # LV grid, strike nodes
    sqrt_eps: float = 0.0                  # Heston: 0 = plain full truncation

    @property
    def n_instr(self) -> int:
        return int(len(self.instr_step))

    def with_(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------
# Black-Scholes: sigma = 0.20, targets at sigma = 0.25
# --------------------------------------------------------------------------
def bs_call(s0, k, r, t, sigma):
    """Closed-form Black-Scholes call, used only to set targets and pins."""
    from scipy.stats import norm
    k = np.asarray(k, dtype=np.float64)
    sd = sigma * math.sqrt(t)
    d1 = (math.log(s0) - np.log(k) + (r + 0.5 * sigma * sigma) * t) / sd
    d2 = d1 - sd
    return s0 * norm.cdf(d1) - k * math.exp(-r * t) * norm.cdf(d2)


def bs_vega(s0, k, r, t, sigma):
    from scipy.stats import norm
    k = np.asarray(k, dtype=np.float64)
    sd = sigma * math.sqrt(t)
    d1 = (math.log(s0) - np.log(k) + (r + 0.5 * sigma * sigma) * t) / sd
    return s0 * norm.pdf(d1) * math.sqrt(t)


def bs_problem(n_paths: int = 1 << 14, n_steps: int = 16, seed: int = 1, euler_on_s: bool = False):
    """Black-Scholes GBM, one parameter sigma, four calls K=80..110 at T=1;
    euler_on_s: the Euler scheme on S as the SDE is written (model 4)
    instead of on log S."""
    strikes = np.array([80.0, 90.0, 100.0, 110.0])
    pb = Problem(model=MODEL_BS_S if euler_on_s else MODEL_BS, n_params=1, n_steps=n_steps, n_paths=n_paths,
                 t_max=1.0,
                 instr_step=np.full(4, n_steps, dtype=np.int32), instr_strike=strikes,
                 s0=100.0, rate=0.02, seed=seed)
    theta = np.array([0.20])
    targets = bs_call(100.0, strikes, 0.02, 1.0, 0.25)
    return pb, theta, targets


# --------------------------------------------------------------------------
# Heston: 8 strikes x 5 maturities, 128 steps per year, N = 256 over 2 years
# --------------------------------------------------------------------------
def heston_draws(rng_seed: int, n: int) -> np.ndarray:
    rng = np.random.default_rng(rng_seed)
    return HESTON_LO + (HESTON_HI - HESTON_LO) * rng.random((n, 5))


def heston_instruments(n_strikes: int = 8, maturities=(0.25, 0.6875, 1.125, 1.5625, 2.0),
                       steps_per_year: int = 128):
    """Maturity-major instrument table (maturity step, strike)."""
    strikes = np.linspace(70.0, 130.0, n_strikes)
    steps = [int(round(t * steps_per_year)) for t in maturities]
    instr_step = np.repeat(np.array(steps, dtype=np.int32), n_strikes)
    instr_strike = np.tile(strikes, len(steps))
    return instr_step, instr_strike


def heston_problem(n_paths: int = 1 << 20, seed: int = 1, n_steps: int = 256, t_max: float = 2.0,
                   n_strikes: int = 8, n_maturities: int = 5):
    """Heston full-truncation problem; theta0 = first draw of rng(2),
    theta_target = second draw.  Returns (problem, theta0, theta_target, eps)
    where eps ~ N(0,1) from rng(3) sets the 0.1 % target noise."""
    mats = np.linspace(0.25, t_max, n_maturities)
    step_per_year = n_steps / t_max
    instr_step, instr_strike = heston_instruments(n_strikes, mats, step_per_year)
    pb = Problem(model=MODEL_HESTON, n_params=5, n_steps=n_steps, n_paths=n_paths, t_max=t_max,
                 instr_step=instr_step, instr_strike=instr_strike, s0=100.0, rate=0.02, seed=seed)
    draws = heston_draws(2, 2)
    eps = np.random.default_rng(3).standard_normal(len(instr_step))
    return pb, draws[0].copy(), draws[1].copy(), eps


def noisy_targets(prices: np.ndarray, eps: np.ndarray, rel: float = 1e-3) -> np.ndarray:
    """Targets = model prices at the target draw times (1 + rel * eps)."""
    return np.asarray(prices, dtype=np.float64) * (1.0 + rel * np.asarray(eps))


# --------------------------------------------------------------------------
# Local volatility: 10 maturities x 20 strikes, bilinear grid, M = 200
# --------------------------------------------------------------------------
def lv_surface(rng, t_nodes, k_nodes, s0: float = 100.0) -> np.ndarray:
    """A smooth random local-volatility surface on the nodes, inside
    [0.1, 0.5]: level + skew m + smile m^2 + term T with m = K/S0 - 1 and
    coefficients drawn uniformly (level 0.15..0.35, skew -0.3..0, smile
    0..0.5, term -0.05..0.05).  Flattened time-major [a * nK + k]."""
    level = rng.uniform(0.15, 0.35)
    skew = rng.uniform(-0.3, 0.0)
    smile = rng.uniform(0.0, 0.5)
    term = rng.uniform(-0.05, 0.05)
    T, K = np.meshgrid(np.asarray(t_nodes), np.asarray(k_nodes), indexing="ij")
    m = K / s0 - 1.0
    return np.clip(level + skew * m + smile * m * m + term * T, 0.1, 0.5).ravel()


def lv_problem(n_paths: int = 1 << 22, seed: int = 1, n_steps: int = 256, t_max: float = 2.0,
               n_t: int = 10, n_k: int = 20, surface: str = "smooth"):
    """Local volatility on a 10 x 20 grid.  surface="smooth": node values from
    lv_surface (draws 1 and 2 of rng(4) for theta0 and theta_target);
    surface="iid": every node value U(0.1, 0.5) independently (the first and
    second n_t n_k draws of rng(4))."""
    t_nodes = 0.2 * np.arange(1, n_t + 1) * (t_max / (0.2 * n_t))
    k_nodes = 55.0 + 5.0 * np.arange(n_k) * (19.0 / max(n_k - 1, 1))
    spy = n_steps / t_max
    steps = np.array([int(round(t * spy)) for t in t_nodes], dtype=np.int32)
    instr_step = np.repeat(steps, n_k)
    instr_strike = np.tile(k_nodes, n_t)
    pb = Problem(model=MODEL_LV, n_params=n_t * n_k, n_steps=n_steps, n_paths=n_paths, t_max=t_max,
                 instr_step=instr_step, instr_strike=instr_strike, s0=100.0, rate=0.02, seed=seed,
                 t_nodes=t_nodes, k_nodes=k_nodes)
    rng = np.random.default_rng(4)
    if surface == "iid":
        grid0 = rng.uniform(0.1, 0.5, n_t * n_k)
        grid_target = rng.uniform(0.1, 0.5, n_t * n_k)
    elif surface == "smooth":
        grid0 = lv_surface(rng, t_nodes, k_nodes)
        grid_target = lv_surface(rng, t_nodes, k_nodes)
    else:
        raise ValueError(f"unknown surface {surface!r}")
    eps = np.random.default_rng(5).standard_normal(len(instr_step))
    fd_coords = np.sort(np.random.default_rng(5).choice(n_t * n_k, size=min(10, n_t * n_k), replace=False))
    return pb, grid0, grid_target, eps, fd_coords


# --------------------------------------------------------------------------
# Heston stochastic local volatility (the paper's own test model)
# --------------------------------------------------------------------------
def leverage_surface(rng, t_nodes, k_nodes, s0: float = 100.0) -> np.ndarray:
    """A smooth random leverage surface around 1, inside [0.5, 1.5]:
    level U(0.8, 1.2) + skew U(-0.5, 0) m + smile U(0, 1) m^2 + term
    U(-0.1, 0.1) T with m = K/S0 - 1.  Flattened time-major [a * nK + k]."""
    level = rng.uniform(0.8, 1.2)
    skew = rng.uniform(-0.5, 0.0)
    smile = rng.uniform(0.0, 1.0)
    term = rng.uniform(-0.1, 0.1)
    T, K = np.meshgrid(np.asarray(t_nodes), np.asarray(k_nodes), indexing="ij")
    m = K / s0 - 1.0
    return np.clip(level + skew * m + smile * m * m + term * T, 0.5, 1.5).ravel()


def slv_problem(n_paths: int = 1 << 20, seed: int = 1, n_steps: int = 256, t_max: float = 2.0,
                n_t: int = 10, n_k: int = 20):
    """Heston SLV: leverage rows at the maturities 0.2..2.0 (row a governs
    the time up to maturity a), spot nodes 55..150, calls at every node
    (m = n_t n_k), Heston parameters from the Feller part of the box
    (draws of rng(21)), leverage surfaces from rng(22); targets priced at
    the second draw.  theta = (kappa, theta_bar, xi, rho, v0, L[a][k])."""
    t_nodes = 0.2 * np.arange(1, n_t + 1) * (t_max / (0.2 * n_t))
    k_nodes = 55.0 + 5.0 * np.arange(n_k) * (19.0 / max(n_k - 1, 1))
    spy = n_steps / t_max
    steps = np.array([int(round(t * spy)) for t in t_nodes], dtype=np.int32)
    pb = Problem(model=MODEL_SLV, n_params=5 + n_t * n_k, n_steps=n_steps, n_paths=n_paths, t_max=t_max,
                 instr_step=np.repeat(steps, n_k), instr_strike=np.tile(k_nodes, n_t), s0=100.0, rate=0.02,
                 seed=seed, t_nodes=t_nodes, k_nodes=k_nodes)
    hd = heston_feller_draws(21, 2)
    rng = np.random.default_rng(22)
    th0 = np.concatenate([hd[0], leverage_surface(rng, t_nodes, k_nodes)])
    tht = np.concatenate([hd[1], leverage_surface(rng, t_nodes, k_nodes)])
    eps = np.random.default_rng(23).standard_normal(pb.n_instr)
    fd_coords = np.sort(np.random.default_rng(24).choice(pb.n_params, size=min(10, pb.n_params), replace=False))
    return pb, th0, tht, eps, fd_coords


# --------------------------------------------------------------------------
# Surrogate training set: uniform draws in the Heston box
# --------------------------------------------------------------------------
def surrogate_draws(n: int, rng_seed: int = 6) -> np.ndarray:
    return heston_feller_draws(rng_seed, n)


def heston_feller_draws(rng_seed: int, n: int) -> np.ndarray:
    """Uniform draws on the part of the Heston box where Feller's condition
    2 kappa theta_bar >= xi^2 holds (rejection from uniform box draws, in
    the generator's order)."""
    rng = np.random.default_rng(rng_seed)
    out = []
    while len(out) < n:
        d = HESTON_LO + (HESTON_HI - HESTON_LO) * rng.random((max(4 * n, 64), 5))
        d = d[2.0 * d[:, 0] * d[:, 1] >= d[:, 2] ** 2]
        out.extend(d[: n - len(out)])
    return np.array(out)


# --------------------------------------------------------------------------
# Batched instances of uneven size
# --------------------------------------------------------------------------
def batched_instances(n_inst: int = 256, rng_seed: int = 7):
    """Heston instances with m ~ U{8..120}, P in {2^14, 2^16, 2^18},
    N in {64, 128, 256} over T_max = 2, maturities at 0.2..1.0 of T_max,
    strikes linspace(70, 130, ceil(m/5)) row-major truncated to m."""
    rng = np.random.default_rng(rng_seed)
    out = []
    for b in range(n_inst):
        m = int(rng.integers(8, 121))
        P = int(rng.choice([1 << 14, 1 << 16, 1 << 18]))
        N = int(rng.choice([64, 128, 256]))
        nk = int(math.ceil(m / 5))
        strikes = np.linspace(70.0, 130.0, nk)
        steps = [int(round(f * N)) for f in (0.2, 0.4, 0.6, 0.8, 1.0)]
        st = np.repeat(np.array(steps, dtype=np.int32), nk)[:m]
        kk = np.tile(strikes, 5)[:m]
        theta = HESTON_LO + (HESTON_HI - HESTON_LO) * rng.random(5)
        theta_t = HESTON_LO + (HESTON_HI - HESTON_LO) * rng.random(5)
        eps = rng.standard_normal(m)
        pb = Problem(model=MODEL_HESTON, n_params=5, n_steps=N, n_paths=P, t_max=2.0,
                     instr_step=st, instr_strike=kk, seed=1, inst=b)
        out.append((pb, theta, theta_t, eps))
    return out
