"""Batched calibration instances: binding of the calb_* entry points of
include/mcaad.h, graph capture/replay, and an autotuner that times the
captured step for each checkpoint spacing and persistent-grid size.
(Argument marshalling and timing only; the step runs in the HIP kernels.)"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np

from . import capi

EXPORTED = ("calb_create", "calb_destroy", "calb_offsets", "calb_configure", "calb_geometry",
            "calibrate_gradient_batch", "calb_capture", "calb_replay", "calb_status", "calb_last_error")

_done = False


def lib():
    global _done
    L = capi.lib()
    if not _done:
        vp, i32 = C.c_void_p, C.c_int32
        sig = {
            "calb_create": ([vp, i32, C.POINTER(vp)], C.c_int),
            "calb_destroy": ([vp], C.c_int),
            "calb_offsets": ([vp, C.POINTER(C.c_int64)], C.c_int),
            "calb_configure": ([vp, i32, i32, i32], C.c_int),
            "calb_geometry": ([vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)], C.c_int),
            "calibrate_gradient_batch": ([vp, vp, vp, vp, vp, vp, vp], C.c_int),
            "calb_capture": ([vp, vp, vp, vp, vp, vp, vp], C.c_int),
            "calb_replay": ([vp, vp], C.c_int),
            "calb_status": ([vp, vp], C.c_int),
            "calb_last_error": ([vp], C.c_char_p),
        }
        for n, (a, r) in sig.items():
            f = getattr(L, n)
            f.argtypes = a
            f.restype = r
        _done = True
    return L


def _p(t):
    return C.c_void_p(t.data_ptr())


class BatchCalibration:
    """All instances' theta [n, M], targets (concatenated) and outputs live
    on the device; gradient() runs one step eagerly, capture()/replay() run
    it as a HIP graph."""

    def __init__(self, problems, precision: str = "fp32", ckpt_every: int = 0):
        import torch
        self.torch = torch
        self.packs = [capi.Packed(pb, capi.CAL_FP64 if precision == "fp64" else capi.CAL_FP32, ckpt_every,
                                  capi.CAL_CKPT_STORE) for pb in problems]
        arr = (capi.cal_problem * len(problems))(*[p.s for p in self.packs])
        self.ctx = C.c_void_p()
        rc = lib().calb_create(arr, len(problems), C.byref(self.ctx))
        if rc != 0:
            raise capi.CalError(rc, lib().calb_last_error(None).decode())
        self.n = len(problems)
        self.M = int(problems[0].n_params)
        off = (C.c_int64 * (self.n + 1))()
        lib().calb_offsets(self.ctx, off)
        self.offsets = np.array(list(off), dtype=np.int64)
        dev = torch.device("cuda", torch.cuda.current_device())
        self.dev = dev
        self.Ey = torch.empty(int(self.offsets[-1]), dtype=torch.float64, device=dev)
        self.G = torch.empty(self.n, dtype=torch.float64, device=dev)
        self.grad = torch.empty(self.n, self.M, dtype=torch.float64, device=dev)
        self.capture_stream = torch.cuda.Stream()
        self._bound = None

    def _check(self, rc):
        if rc < 0:
            raise capi.CalError(rc, lib().calb_last_error(self.ctx).decode())
        return rc

    def configure(self, ckpt_every: int, workgroups_per_cu: int = 0, paths_per_lane: int = 1):
        self._check(lib().calb_configure(self.ctx, int(ckpt_every), int(workgroups_per_cu), int(paths_per_lane)))
        self._bound = None

    def geometry(self):
        k, g, n, ppl = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        lib().calb_geometry(self.ctx, C.byref(k), C.byref(g), C.byref(n), C.byref(ppl))
        return {"ckpt_every": k.value, "grid": g.value, "n_items": n.value, "paths_per_lane": ppl.value}

    def split(self, flat):
        return [flat[self.offsets[i]:self.offsets[i + 1]] for i in range(self.n)]

    def gradient(self, theta, C_flat, stream=None):
        th, Ct = theta.contiguous(), C_flat.contiguous()
        st = C.c_void_p(int(stream) if stream is not None else self.torch.cuda.current_stream().cuda_stream)
        self._check(lib().calibrate_gradient_batch(self.ctx, _p(th), _p(Ct), _p(self.Ey), _p(self.G),
                                                   _p(self.grad), st))
        return self.Ey, self.G, self.grad

    def capture(self, theta, C_flat):
        """Capture one step bound to these (device-resident) arrays."""
        self._keep = (theta.contiguous(), C_flat.contiguous())
        th, Ct = self._keep
        self.torch.cuda.synchronize()
        st = C.c_void_p(self.capture_stream.cuda_stream)
        self._check(lib().calb_capture(self.ctx, _p(th), _p(Ct), _p(self.Ey), _p(self.G), _p(self.grad), st))
        self._bound = True

    def replay(self, stream=None):
        st = C.c_void_p(int(stream) if stream is not None else self.torch.cuda.current_stream().cuda_stream)
        self._check(lib().calb_replay(self.ctx, st))
        return self.Ey, self.G, self.grad

    def status(self):
        return self._check(lib().calb_status(self.ctx, C.c_void_p(self.torch.cuda.current_stream().cuda_stream)))

    def autotune(self, theta, C_flat, ks=(8, 16, 32), wpcs=(0, 1, 2, 4), ppls=(1, 2), reps: int = 5):
        """Time the captured step for every (checkpoint spacing, persistent
        workgroups per CU, paths per lane), then the three fastest again in
        reverse order (so that the first-timed candidates, which meet a GPU
        whose clock has not settled, are not penalised), and keep the fastest.
        Returns (choice, table)."""
        def timed(cfg):
            self.configure(*cfg)
            self.capture(theta, C_flat)
            self.replay()
            self.torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                self.replay()
            self.torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps

        best_t = {}
        for k in ks:
            for w in wpcs:
                for ppl in ppls:
                    best_t[(k, w, ppl)] = timed((k, w, ppl))
        for cfg in sorted(best_t, key=best_t.get)[:3][::-1]:
            best_t[cfg] = min(best_t[cfg], timed(cfg))
        table = list(best_t.items())
        best = min(table, key=lambda r: r[1])[0]
        self.configure(*best)
        self.capture(theta, C_flat)
        return best, table

    def close(self):
        if self.ctx:
            lib().calb_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
