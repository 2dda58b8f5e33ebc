"""ctypes shim over the FP64 CPU oracle (oracle/mcaad_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, by the smoke check and by the
CPU-baseline leg of the benchmark.  The GPU library never imports it.

Problems are passed duck-typed: any object with the attributes model,
n_params, n_steps, n_paths, t_max, instr_step, instr_strike, s0, rate, seed,
inst, t_nodes, k_nodes.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")


class _Problem(C.Structure):
    _fields_ = [
        ("model", C.c_int32), ("n_params", C.c_int32), ("n_instr", C.c_int32), ("n_steps", C.c_int32),
        ("n_paths", C.c_int64), ("seed", C.c_uint64), ("inst", C.c_uint32), ("pad_", C.c_uint32),
        ("s0", C.c_double), ("rate", C.c_double), ("t_max", C.c_double),
        ("instr_step", C.POINTER(C.c_int32)), ("instr_strike", C.POINTER(C.c_double)),
        ("n_t_nodes", C.c_int32), ("n_k_nodes", C.c_int32),
        ("t_nodes", C.POINTER(C.c_double)), ("k_nodes", C.POINTER(C.c_double)),
        ("sqrt_eps", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # noqa: F401  (package-relative when imported as oracle.oracle)
            _b.build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        pp = C.POINTER(_Problem)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_philox4x32_10.restype = None
        L.orc_philox_many.argtypes = [C.POINTER(C.c_uint32), C.c_int64, C.POINTER(C.c_uint32),
                                      C.POINTER(C.c_uint32)]
        L.orc_philox_many.restype = None
        L.orc_normals.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int32, dp]
        L.orc_normals.restype = None
        L.orc_forward.argtypes = [pp, dp, dp, dp]
        L.orc_vjp.argtypes = [pp, dp, dp, dp, dp]
        L.orc_gradient.argtypes = [pp, dp, dp, dp, dp, dp]
        L.orc_jacobian.argtypes = [pp, dp, dp, dp, dp, dp]
        L.orc_forward_cstep.argtypes = [pp, dp, C.c_int, C.c_double, dp, dp]
        for f in ("orc_forward", "orc_vjp", "orc_gradient", "orc_jacobian", "orc_forward_cstep"):
            getattr(L, f).restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_get_threads.argtypes = []
        L.orc_get_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


class _Packed:
    """Keeps the numpy buffers referenced by the C struct alive."""

    def __init__(self, pb):
        self.step = np.ascontiguousarray(pb.instr_step, dtype=np.int32)
        self.strike = np.ascontiguousarray(pb.instr_strike, dtype=np.float64)
        self.tn = None if pb.t_nodes is None else np.ascontiguousarray(pb.t_nodes, dtype=np.float64)
        self.kn = None if pb.k_nodes is None else np.ascontiguousarray(pb.k_nodes, dtype=np.float64)
        s = _Problem()
        s.model = int(pb.model)
        s.n_params = int(pb.n_params)
        s.n_instr = int(len(self.step))
        s.n_steps = int(pb.n_steps)
        s.n_paths = int(pb.n_paths)
        s.seed = int(pb.seed)
        s.inst = int(pb.inst)
        s.s0 = float(pb.s0)
        s.rate = float(pb.rate)
        s.t_max = float(pb.t_max)
        s.instr_step = self.step.ctypes.data_as(C.POINTER(C.c_int32))
        s.instr_strike = _dp(self.strike)
        s.n_t_nodes = 0 if self.tn is None else len(self.tn)
        s.n_k_nodes = 0 if self.kn is None else len(self.kn)
        s.t_nodes = _dp(self.tn)
        s.k_nodes = _dp(self.kn)
        s.sqrt_eps = float(getattr(pb, "sqrt_eps", 0.0))
        self.s = s

    @property
    def ref(self):
        return C.byref(self.s)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def philox(ctr, key):
    """Philox4x32-10 of one counter (4 x u32) and key (2 x u32)."""
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(o[i]) for i in range(4)]


def philox_many(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x32-10 of n counters ([n, 4] u32) under one key: [n, 4] u32."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    out = np.empty_like(c)
    u32p = C.POINTER(C.c_uint32)
    lib().orc_philox_many(c.ctypes.data_as(u32p), c.shape[0], k, out.ctypes.data_as(u32p))
    return out


def normals(seed: int, inst: int, path: int, q0: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    lib().orc_normals(int(seed), int(inst), int(path), int(q0), int(n), _dp(out))
    return out


def forward(pb, theta, per_path: bool = False):
    """Ey[m] (and optionally the P x m per-path payoffs)."""
    pk = _Packed(pb)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    m = pk.s.n_instr
    Ey = np.empty(m)
    yp = np.empty((pb.n_paths, m)) if per_path else None
    _check(lib().orc_forward(pk.ref, _dp(th), _dp(Ey), _dp(yp)), "forward")
    return (Ey, yp) if per_path else Ey


def vjp(pb, theta, lam, per_path: bool = False):
    """grad[j] = sum_i lam_i dEy_i/dtheta_j by the reverse sweep."""
    pk = _Packed(pb)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    la = np.ascontiguousarray(lam, dtype=np.float64)
    g = np.empty(pb.n_params)
    gp = np.empty((pb.n_paths, pb.n_params)) if per_path else None
    _check(lib().orc_vjp(pk.ref, _dp(th), _dp(la), _dp(g), _dp(gp)), "vjp")
    return (g, gp) if per_path else g


def gradient(pb, theta, targets):
    """(Ey, G, grad) by the paper's two-pass algorithm."""
    pk = _Packed(pb)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    Cc = np.ascontiguousarray(targets, dtype=np.float64)
    Ey = np.empty(pk.s.n_instr)
    G = np.empty(1)
    g = np.empty(pb.n_params)
    _check(lib().orc_gradient(pk.ref, _dp(th), _dp(Cc), _dp(Ey), _dp(G), _dp(g)), "gradient")
    return Ey, float(G[0]), g


def jacobian(pb, theta, per_path: bool = False):
    """(Ey, J[m, M]) by forward tangent mode; per-path arrays optional."""
    pk = _Packed(pb)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    m, M = pk.s.n_instr, pb.n_params
    Ey = np.empty(m)
    J = np.empty((m, M))
    yp = np.empty((pb.n_paths, m)) if per_path else None
    dyp = np.empty((pb.n_paths, m, M)) if per_path else None
    _check(lib().orc_jacobian(pk.ref, _dp(th), _dp(Ey), _dp(J), _dp(yp), _dp(dyp)), "jacobian")
    return (Ey, J, yp, dyp) if per_path else (Ey, J)


def forward_cstep(pb, theta, j: int, hc: float = 1e-30):
    """Complex-step forward: returns (Re Ey, Im Ey) at theta + i*hc*e_j."""
    pk = _Packed(pb)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    m = pk.s.n_instr
    re = np.empty(m)
    im = np.empty(m)
    _check(lib().orc_forward_cstep(pk.ref, _dp(th), int(j), float(hc), _dp(re), _dp(im)), "forward_cstep")
    return re, im
