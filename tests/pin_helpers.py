"""Closed forms and independent derivative machinery used only to pin the oracle.

Nothing here is the method: these are textbook prices (Black-Scholes,
Heston's characteristic-function price) and a small generic reverse-mode AD
with an expectation operator, written from the algorithm in the paper's
appendix (expected backward automatic differentiation, after Fries).
"""
import math

import numpy as np
from scipy import integrate


# --------------------------------------------------------------------------
# Heston (1993) call by Fourier inversion, in the numerically stable form of
# Albrecher, Mayer, Schoutens and Tistaert (2007).
# --------------------------------------------------------------------------
def _heston_cf(u, T, s0, r, kappa, thb, xi, rho, v0):
    iu = 1j * u
    b = kappa - rho * xi * iu
    d = np.sqrt(b * b + xi * xi * (iu + u * u))
    g = (b - d) / (b + d)
    e = np.exp(-d * T)
    C = kappa * thb / (xi * xi) * ((b - d) * T - 2.0 * np.log((1.0 - g * e) / (1.0 - g)))
    D = (b - d) / (xi * xi) * (1.0 - e) / (1.0 - g * e)
    return np.exp(iu * (math.log(s0) + r * T) + C + D * v0)


def heston_call(s0, K, r, T, kappa, thb, xi, rho, v0):
    lnK = math.log(K)
    fwd = s0 * math.exp(r * T)

    def p_int(u, j):
        if j == 1:
            val = _heston_cf(u - 1j, T, s0, r, kappa, thb, xi, rho, v0) / fwd
        else:
            val = _heston_cf(u, T, s0, r, kappa, thb, xi, rho, v0)
        return (np.exp(-1j * u * lnK) * val / (1j * u)).real

    P1 = 0.5 + integrate.quad(p_int, 1e-10, 200.0, args=(1,), limit=400)[0] / math.pi
    P2 = 0.5 + integrate.quad(p_int, 1e-10, 200.0, args=(2,), limit=400)[0] / math.pi
    return s0 * P1 - K * math.exp(-r * T) * P2


# --------------------------------------------------------------------------
# Expected backward AD over an operator list (paper, appendix): random
# variables are vectors over paths; the adjoint of an expectation node adds
# E(adjoint) to its argument, every other node adds adjoint * partial.
# --------------------------------------------------------------------------
class Tape:
    def __init__(self, n_paths):
        self.n = n_paths
        self.vals = []      # value of each node (scalar broadcast or vector)
        self.args = []      # list of (arg index, partial) pairs
        self.is_E = []

    def _push(self, val, args, is_E=False):
        self.vals.append(np.broadcast_to(np.asarray(val, dtype=np.float64), (self.n,)).copy())
        self.args.append(args)
        self.is_E.append(is_E)
        return len(self.vals) - 1

    def const(self, v):
        return self._push(v, [])

    def var(self, v):
        return self._push(v, [])

    def add(self, a, b):
        return self._push(self.vals[a] + self.vals[b], [(a, 1.0), (b, 1.0)])

    def sub(self, a, b):
        return self._push(self.vals[a] - self.vals[b], [(a, 1.0), (b, -1.0)])

    def mul(self, a, b):
        return self._push(self.vals[a] * self.vals[b], [(a, self.vals[b]), (b, self.vals[a])])

    def scale(self, a, c):
        return self._push(c * self.vals[a], [(a, c)])

    def shift(self, a, c):
        return self._push(self.vals[a] + c, [(a, 1.0)])

    def exp(self, a):
        e = np.exp(self.vals[a])
        return self._push(e, [(a, e)])

    def sqrt(self, a):
        s = np.sqrt(self.vals[a])
        d = np.where(s > 0, 0.5 / np.where(s > 0, s, 1.0), 0.0)
        return self._push(s, [(a, d)])

    def relu(self, a):
        v = self.vals[a]
        return self._push(np.maximum(v, 0.0), [(a, (v > 0).astype(np.float64))])

    def expect(self, a):
        return self._push(np.full(self.n, self.vals[a].mean()), [(a, None)], is_E=True)

    def grad(self, out, wrt):
        adj = [np.zeros(self.n) for _ in self.vals]
        adj[out] = np.ones(self.n)
        for k in range(len(self.vals) - 1, -1, -1):
            for (j, d) in self.args[k]:
                if self.is_E[k]:
                    adj[j] = adj[j] + adj[k].mean()
                else:
                    adj[j] = adj[j] + adj[k] * d
        return [adj[w].mean() for w in wrt]
