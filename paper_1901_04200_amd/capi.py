"""Python binding of the C ABI in include/mcaad.h (argument marshalling only).

Every function here has the name of the C entry point it calls.  Device
arrays are torch tensors on the current HIP device (FP64, contiguous); the
stream is torch's current stream unless one is given.  Every step of the
path runs in the HIP kernels of libmcaad.so: if the library is missing this
module raises, it never falls back to host code.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libmcaad.so")

CAL_BS, CAL_HESTON, CAL_LV, CAL_SLV = 0, 1, 2, 3
CAL_FP32, CAL_FP64 = 0, 1
CAL_CKPT_AUTO, CAL_CKPT_RERUN, CAL_CKPT_STORE = 0, 1, 2
CAL_OK, CAL_EINVAL, CAL_ENOMEM, CAL_EHIP, CAL_EUNSUPPORTED = 0, -1, -2, -3, -4
CAL_FLAG_THETA, CAL_FLAG_NONFINITE, CAL_FLAG_CKPT = 1, 2, 4

EXPORTED = (
    "cal_validate", "cal_create", "cal_destroy", "calibrate_forward", "calibrate_vjp",
    "calibrate_forward_store", "calibrate_vjp_stored", "calibrate_gradient", "calibrate_jacobian", "calibrate_jacobian_batch", "cal_status", "cal_last_error",
    "cal_timing_enable", "cal_timing_read", "cal_geometry", "cal_philox", "cal_normals",
    "calibrate_gradient_static",
)


class cal_problem(C.Structure):
    _fields_ = [
        ("model", C.c_int32), ("precision", C.c_int32), ("n_params", C.c_int32), ("n_instr", C.c_int32),
        ("n_steps", C.c_int32), ("ckpt_every", C.c_int32), ("n_paths", C.c_int64), ("seed", C.c_uint64),
        ("inst", C.c_uint32), ("ckpt_mode", C.c_int32), ("max_batch", C.c_int32), ("paths_per_lane", C.c_int32),
        ("s0", C.c_double), ("rate", C.c_double), ("t_max", C.c_double), ("sqrt_eps", C.c_double),
        ("instr_step", C.POINTER(C.c_int32)), ("instr_strike", C.POINTER(C.c_double)),
        ("n_t_nodes", C.c_int32), ("n_k_nodes", C.c_int32),
        ("t_nodes", C.POINTER(C.c_double)), ("k_nodes", C.POINTER(C.c_double)),
    ]


class CalError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mcaad error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libmcaad.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, dp, i32, i64 = C.c_void_p, C.c_void_p, C.c_int32, C.c_int64
        pp = C.POINTER(cal_problem)
        sig = {
            "cal_validate": ([pp, C.c_char_p, i32], C.c_int),
            "cal_create": ([pp, C.POINTER(vp)], C.c_int),
            "cal_destroy": ([vp], C.c_int),
            "calibrate_forward": ([vp, dp, dp, vp], C.c_int),
            "calibrate_vjp": ([vp, dp, dp, dp, vp], C.c_int),
            "calibrate_forward_store": ([vp, dp, dp, vp], C.c_int),
            "calibrate_vjp_stored": ([vp, dp, dp, dp, vp], C.c_int),
            "calibrate_gradient": ([vp, dp, dp, dp, dp, dp, vp], C.c_int),
            "calibrate_jacobian": ([vp, dp, dp, dp, vp], C.c_int),
            "calibrate_jacobian_batch": ([vp, dp, i32, C.c_uint32, dp, dp, vp], C.c_int),
            "cal_status": ([vp, vp], C.c_int),
            "cal_last_error": ([vp], C.c_char_p),
            "cal_timing_enable": ([vp, i32], C.c_int),
            "cal_timing_read": ([vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_int64)], C.c_int),
            "cal_geometry": ([vp, C.POINTER(i32), C.POINTER(i64), C.POINTER(i32), C.POINTER(i32)], C.c_int),
            "cal_philox": ([vp, C.c_uint32, C.c_uint32, i64, vp, vp], C.c_int),
            "cal_normals": ([i32, C.c_uint64, C.c_uint32, C.c_uint32, i64, C.c_uint32, i32, vp, vp], C.c_int),
            "calibrate_gradient_static": ([pp, dp, dp, dp, dp, dp, dp, vp], C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(rc, ctx=None):
    if rc < 0:
        msg = lib().cal_last_error(ctx).decode()
        raise CalError(rc, msg)
    return rc


class Packed:
    """A cal_problem plus the host arrays it points at."""

    def __init__(self, pb, precision=CAL_FP32, ckpt_every=0, ckpt_mode=CAL_CKPT_AUTO, max_batch=0, paths_per_lane=0):
        import numpy as np
        self.step = np.ascontiguousarray(pb.instr_step, dtype=np.int32)
        self.strike = np.ascontiguousarray(pb.instr_strike, dtype=np.float64)
        self.tn = None if getattr(pb, "t_nodes", None) is None else np.ascontiguousarray(pb.t_nodes, dtype=np.float64)
        self.kn = None if getattr(pb, "k_nodes", None) is None else np.ascontiguousarray(pb.k_nodes, dtype=np.float64)
        s = cal_problem()
        s.model = int(pb.model)
        s.precision = int(precision)
        s.n_params = int(pb.n_params)
        s.n_instr = int(len(self.step))
        s.n_steps = int(pb.n_steps)
        s.ckpt_every = int(ckpt_every)
        s.n_paths = int(pb.n_paths)
        s.seed = int(pb.seed)
        s.inst = int(pb.inst)
        s.ckpt_mode = int(ckpt_mode)
        s.max_batch = int(max_batch)
        s.paths_per_lane = int(paths_per_lane)
        s.s0 = float(pb.s0)
        s.rate = float(pb.rate)
        s.t_max = float(pb.t_max)
        s.sqrt_eps = float(getattr(pb, "sqrt_eps", 0.0))
        s.instr_step = self.step.ctypes.data_as(C.POINTER(C.c_int32))
        s.instr_strike = self.strike.ctypes.data_as(C.POINTER(C.c_double))
        s.n_t_nodes = 0 if self.tn is None else len(self.tn)
        s.n_k_nodes = 0 if self.kn is None else len(self.kn)
        s.t_nodes = None if self.tn is None else self.tn.ctypes.data_as(C.POINTER(C.c_double))
        s.k_nodes = None if self.kn is None else self.kn.ctypes.data_as(C.POINTER(C.c_double))
        self.s = s


def cal_validate(pb, precision=CAL_FP32, ckpt_every=0, ckpt_mode=CAL_CKPT_AUTO, paths_per_lane=0):
    """(code, message) of the host-side problem check."""
    pk = Packed(pb, precision, ckpt_every, ckpt_mode, 0, paths_per_lane)
    buf = C.create_string_buffer(256)
    rc = lib().cal_validate(C.byref(pk.s), buf, 256)
    return rc, buf.value.decode()


def cal_create(pb, precision=CAL_FP32, ckpt_every=0, ckpt_mode=CAL_CKPT_AUTO, max_batch=0, paths_per_lane=0):
    pk = Packed(pb, precision, ckpt_every, ckpt_mode, max_batch, paths_per_lane)
    h = C.c_void_p()
    _check(lib().cal_create(C.byref(pk.s), C.byref(h)))
    return h


def cal_destroy(ctx):
    return _check(lib().cal_destroy(ctx))


def calibrate_forward(ctx, theta, Ey, stream=None):
    return _check(lib().calibrate_forward(ctx, _ptr(theta), _ptr(Ey), _stream(stream)), ctx)


def calibrate_vjp(ctx, theta, lam, grad, stream=None):
    return _check(lib().calibrate_vjp(ctx, _ptr(theta), _ptr(lam), _ptr(grad), _stream(stream)), ctx)


def calibrate_forward_store(ctx, theta, Ey, stream=None):
    return _check(lib().calibrate_forward_store(ctx, _ptr(theta), _ptr(Ey), _stream(stream)), ctx)


def calibrate_vjp_stored(ctx, theta, lam, grad, stream=None):
    return _check(lib().calibrate_vjp_stored(ctx, _ptr(theta), _ptr(lam), _ptr(grad), _stream(stream)), ctx)


def calibrate_gradient(ctx, theta, C_, Ey, G, grad, stream=None):
    return _check(lib().calibrate_gradient(ctx, _ptr(theta), _ptr(C_), _ptr(Ey), _ptr(G), _ptr(grad),
                                           _stream(stream)), ctx)


def calibrate_gradient_static(pb, theta, C_, Ey, G, grad, status, precision=CAL_FP32, ckpt_every=0,
                              ckpt_mode=CAL_CKPT_AUTO, paths_per_lane=0, stream=None):
    """calibrate_gradient without a context (buffers in the library's static
    device array); status: int32 device tensor [1], set to the call's flags."""
    pk = Packed(pb, precision, ckpt_every, ckpt_mode, 0, paths_per_lane)
    return _check(lib().calibrate_gradient_static(C.byref(pk.s), _ptr(theta), _ptr(C_), _ptr(Ey), _ptr(G),
                                                  _ptr(grad), _ptr(status), _stream(stream)))


def calibrate_jacobian(ctx, theta, Ey, J, stream=None):
    return _check(lib().calibrate_jacobian(ctx, _ptr(theta), _ptr(Ey), _ptr(J), _stream(stream)), ctx)


def calibrate_jacobian_batch(ctx, theta, n_inst, inst0, Ey, J, stream=None):
    return _check(lib().calibrate_jacobian_batch(ctx, _ptr(theta), int(n_inst), int(inst0), _ptr(Ey), _ptr(J),
                                                 _stream(stream)), ctx)


def cal_status(ctx, stream=None):
    return _check(lib().cal_status(ctx, _stream(stream)), ctx)


def cal_last_error(ctx=None):
    return lib().cal_last_error(ctx).decode()


def cal_timing_enable(ctx, on=True):
    return _check(lib().cal_timing_enable(ctx, int(bool(on))), ctx)


def cal_timing_read(ctx, which):
    ms = C.c_double()
    n = C.c_int64()
    _check(lib().cal_timing_read(ctx, int(which), C.byref(ms), C.byref(n)), ctx)
    return ms.value, n.value


def cal_geometry(ctx):
    t, k, mode = C.c_int32(), C.c_int32(), C.c_int32()
    b = C.c_int64()
    _check(lib().cal_geometry(ctx, C.byref(t), C.byref(b), C.byref(k), C.byref(mode)), ctx)
    return {"threads": t.value, "blocks": b.value, "ckpt_every": k.value, "ckpt_mode": mode.value}


def cal_philox(ctr, key0, key1, out, stream=None):
    return _check(lib().cal_philox(_ptr(ctr), int(key0), int(key1), int(ctr.numel() // 4), _ptr(out),
                                   _stream(stream)))


def cal_normals(precision, seed, inst, path0, n_paths, q0, nq, out, stream=None):
    return _check(lib().cal_normals(int(precision), int(seed), int(inst), int(path0), int(n_paths), int(q0),
                                    int(nq), _ptr(out), _stream(stream)))
