"""Torch-facing handle on one calibration problem (device memory and streams
only; the computation is the C ABI's)."""
from __future__ import annotations

import torch

from . import capi

_PREC = {"fp32": capi.CAL_FP32, "fp64": capi.CAL_FP64}
_MODE = {"auto": capi.CAL_CKPT_AUTO, "rerun": capi.CAL_CKPT_RERUN, "store": capi.CAL_CKPT_STORE}


class MonteCarloCalibration:
    """calibrate_forward / calibrate_vjp / calibrate_gradient / calibrate_jacobian
    on one problem.  theta, targets and lambda are FP64 tensors of the
    current device (host arrays are copied there)."""

    def __init__(self, problem, precision: str = "fp32", ckpt_every: int = 0, ckpt_mode: str = "auto",
                 max_batch: int = 0, paths_per_lane: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("the Monte Carlo calibration path needs a HIP device")
        self.problem = problem
        self.precision = precision
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.ctx = capi.cal_create(problem, _PREC[precision], ckpt_every, _MODE[ckpt_mode], max_batch,
                                   paths_per_lane)
        self.m = int(len(problem.instr_step))
        self.M = int(problem.n_params)
        # counts the calls whose sweep wrote the context's checkpoint buffer
        # (forward_store, vjp, gradient); vjp_stored reads what the last wrote
        self.ckpt_writes = 0

    def _dev(self, a, n):
        t = torch.as_tensor(a, dtype=torch.float64, device=self.device).contiguous()
        if t.numel() != n:
            raise ValueError(f"expected {n} values, got {t.numel()}")
        return t

    def forward(self, theta):
        th = self._dev(theta, self.M)
        Ey = torch.empty(self.m, dtype=torch.float64, device=self.device)
        capi.calibrate_forward(self.ctx, th, Ey)
        return Ey

    def forward_store(self, theta):
        """forward() that also keeps the checkpoints for vjp_stored."""
        th = self._dev(theta, self.M)
        Ey = torch.empty(self.m, dtype=torch.float64, device=self.device)
        capi.calibrate_forward_store(self.ctx, th, Ey)
        self.ckpt_writes += 1
        return Ey

    def vjp(self, theta, lam):
        th = self._dev(theta, self.M)
        la = self._dev(lam, self.m)
        g = torch.empty(self.M, dtype=torch.float64, device=self.device)
        capi.calibrate_vjp(self.ctx, th, la, g)
        self.ckpt_writes += 1
        return g

    def vjp_stored(self, theta, lam):
        """vjp() from the checkpoints the last checkpoint-writing call left
        (same theta required; the device flags CAL_FLAG_CKPT otherwise)."""
        th = self._dev(theta, self.M)
        la = self._dev(lam, self.m)
        g = torch.empty(self.M, dtype=torch.float64, device=self.device)
        capi.calibrate_vjp_stored(self.ctx, th, la, g)
        return g

    def gradient(self, theta, targets):
        th = self._dev(theta, self.M)
        C = self._dev(targets, self.m)
        Ey = torch.empty(self.m, dtype=torch.float64, device=self.device)
        G = torch.empty(1, dtype=torch.float64, device=self.device)
        g = torch.empty(self.M, dtype=torch.float64, device=self.device)
        capi.calibrate_gradient(self.ctx, th, C, Ey, G, g)
        self.ckpt_writes += 1
        return Ey, G, g

    def jacobian(self, theta):
        th = self._dev(theta, self.M)
        Ey = torch.empty(self.m, dtype=torch.float64, device=self.device)
        J = torch.empty(self.m, self.M, dtype=torch.float64, device=self.device)
        capi.calibrate_jacobian(self.ctx, th, Ey, J)
        return Ey, J

    def status(self) -> int:
        return capi.cal_status(self.ctx)

    def geometry(self) -> dict:
        return capi.cal_geometry(self.ctx)

    def close(self):
        if self.ctx is not None:
            capi.cal_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pick_config(problem, theta, targets, precision: str = "fp32", ks=(8, 16, 32), ppls=(1,), reps: int = 5):
    """Time `reps` gradient calls (after one warm-up) for every checkpoint
    spacing in `ks` and paths per lane in `ppls`; return (fastest (k, ppl),
    [((k, ppl), seconds per call)]).  The spacing trades pass 1's checkpoint
    stores and pass 2's register footprint (occupancy) against each other;
    more paths per lane mean fewer workgroups and fewer partial sums; which
    wins depends on the model, the sizes and the device."""
    table = []
    for k in ks:
        for ppl in ppls:
            mc = MonteCarloCalibration(problem, precision=precision, ckpt_every=k, ckpt_mode="store",
                                       paths_per_lane=ppl)
            th = mc._dev(theta, mc.M)
            C = mc._dev(targets, mc.m)
            Ey = torch.empty(mc.m, dtype=torch.float64, device=mc.device)
            G = torch.empty(1, dtype=torch.float64, device=mc.device)
            g = torch.empty(mc.M, dtype=torch.float64, device=mc.device)
            capi.calibrate_gradient(mc.ctx, th, C, Ey, G, g)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                capi.calibrate_gradient(mc.ctx, th, C, Ey, G, g)
            e1.record()
            torch.cuda.synchronize()
            table.append(((k, ppl), e0.elapsed_time(e1) * 1e-3 / reps))
            mc.close()
    return min(table, key=lambda r: r[1])[0], table
