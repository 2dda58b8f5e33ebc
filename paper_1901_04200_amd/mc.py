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


def pick_config(problem, theta, targets, precision: str = "fp32", ks=(8, 16, 32), ppls=(1,), reps: int = 10):
    """Time `reps` gradient calls (after two warm-up calls) for every checkpoint
    spacing in `ks` and paths per lane in `ppls`, in two rounds (the candidates
    in order, then in reverse, so that none is favoured by when it ran: clock
    and caches settle over the first calls); keep each candidate's faster round
    and return (fastest (k, ppl), [((k, ppl), seconds per call)]).  The spacing
    trades pass 1's checkpoint stores and pass 2's register footprint
    (occupancy) against each other; more paths per lane mean fewer workgroups
    and fewer partial sums; which wins depends on the model, the sizes and the
    device."""
    cands = []
    for k in ks:
        for ppl in ppls:
            mc = MonteCarloCalibration(problem, precision=precision, ckpt_every=k, ckpt_mode="store",
                                       paths_per_lane=ppl)
            args = (mc._dev(theta, mc.M), mc._dev(targets, mc.m),
                    torch.empty(mc.m, dtype=torch.float64, device=mc.device),
                    torch.empty(1, dtype=torch.float64, device=mc.device),
                    torch.empty(mc.M, dtype=torch.float64, device=mc.device))
            cands.append(((k, ppl), mc, args))
    best = {}
    try:
        for order in (cands, cands[::-1]):
            for key, mc, args in order:
                for _ in range(2):
                    capi.calibrate_gradient(mc.ctx, *args)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    capi.calibrate_gradient(mc.ctx, *args)
                e1.record()
                torch.cuda.synchronize()
                t = e0.elapsed_time(e1) * 1e-3 / reps
                best[key] = min(best.get(key, t), t)
    finally:
        for _, mc, _ in cands:
            mc.close()
    table = [(key, best[key]) for key, _, _ in cands]
    return min(table, key=lambda r: r[1])[0], table
