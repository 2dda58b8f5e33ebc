"""The learned surrogate: binding of include/mcaad_surrogate.h, its training on
labels the Monte Carlo path generates, and the surrogate-assisted
calibration step with the Monte Carlo gradient as judge and fallback.

Argument marshalling only: the network's forward pass, tangents, loss,
double backpropagation and Adam run in the HIP kernels of libmcaad.so.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
import time
from typing import List, Optional

import numpy as np

from . import capi

EXPORTED = ("mlp_create", "mlp_destroy", "mlp_num_params", "mlp_set_params", "mlp_get_params",
            "mlp_set_scaling", "mlp_forward", "mlp_loss_grad", "mlp_adam_step", "mlp_calibration_gradient",
            "mlp_last_error")

_sig_done = False


def lib():
    global _sig_done
    L = capi.lib()
    if not _sig_done:
        vp, i32 = C.c_void_p, C.c_int32
        sig = {
            "mlp_create": ([i32, i32, i32, i32, C.POINTER(vp)], C.c_int),
            "mlp_destroy": ([vp], C.c_int),
            "mlp_num_params": ([vp], C.c_int64),
            "mlp_set_params": ([vp, vp, vp], C.c_int),
            "mlp_get_params": ([vp, vp, vp], C.c_int),
            "mlp_set_scaling": ([vp, vp, vp, vp, vp, vp], C.c_int),
            "mlp_forward": ([vp, vp, i32, vp, vp, vp], C.c_int),
            "mlp_loss_grad": ([vp, vp, vp, vp, i32, C.c_float, vp, vp, vp], C.c_int),
            "mlp_adam_step": ([vp, vp, C.c_float, C.c_float, C.c_float, C.c_float, i32, vp], C.c_int),
            "mlp_calibration_gradient": ([vp, vp, i32, vp, vp, vp, vp, vp, vp], C.c_int),
            "mlp_last_error": ([vp], C.c_char_p),
        }
        for name, (a, r) in sig.items():
            f = getattr(L, name)
            f.argtypes = a
            f.restype = r
        _sig_done = True
    return L


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class MLP:
    """n_in -> H -> H -> H -> n_out with SiLU, on the device."""

    def __init__(self, n_in: int = 5, n_hidden: int = 256, n_out: int = 40, max_batch: int = 4096):
        import torch
        self.torch = torch
        self.n_in, self.H, self.n_out = n_in, n_hidden, n_out
        self.max_batch = max_batch
        self.ctx = C.c_void_p()
        rc = lib().mlp_create(n_in, n_hidden, n_out, max_batch, C.byref(self.ctx))
        if rc != 0:
            raise capi.CalError(rc, lib().mlp_last_error(None).decode())
        self.n_params = int(lib().mlp_num_params(self.ctx))
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.step_count = 0

    def _check(self, rc):
        if rc != 0:
            raise capi.CalError(rc, lib().mlp_last_error(self.ctx).decode())

    def layout(self):
        H, a, o = self.H, self.n_in, self.n_out
        shapes = [(a, H), (H,), (H, H), (H,), (H, H), (H,), (H, o), (o,)]
        out, off = [], 0
        for s in shapes:
            n = int(np.prod(s))
            out.append((off, s))
            off += n
        return out

    def pack(self, params) -> np.ndarray:
        flat = []
        for (W, b) in params:
            flat += [np.asarray(W, np.float32).ravel(), np.asarray(b, np.float32).ravel()]
        v = np.concatenate(flat)
        assert v.size == self.n_params
        return v

    def unpack(self, v):
        v = np.asarray(v)
        L = self.layout()
        return [(v[L[2 * l][0]:L[2 * l][0] + np.prod(L[2 * l][1])].reshape(L[2 * l][1]),
                 v[L[2 * l + 1][0]:L[2 * l + 1][0] + np.prod(L[2 * l + 1][1])]) for l in range(4)]

    def init_params(self, seed: int = 0):
        """He-uniform weights, zero biases (host draw, uploaded)."""
        rng = np.random.default_rng(seed)
        sizes = [self.n_in, self.H, self.H, self.H, self.n_out]
        ps = []
        for a, c in zip(sizes[:-1], sizes[1:]):
            lim = math.sqrt(6.0 / a)
            ps.append((rng.uniform(-lim, lim, (a, c)), np.zeros(c)))
        self.set_params(self.pack(ps))

    def set_params(self, v):
        t = self.torch.as_tensor(np.asarray(v, np.float32), device=self.dev).contiguous()
        self._check(lib().mlp_set_params(self.ctx, _ptr(t), _stream()))
        self.torch.cuda.synchronize()
        self.step_count = 0

    def get_params(self) -> np.ndarray:
        t = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self.dev)
        self._check(lib().mlp_get_params(self.ctx, _ptr(t), _stream()))
        return t.cpu().numpy()

    def set_scaling(self, in_shift, in_scale, out_shift, out_scale):
        ts = [self.torch.as_tensor(np.asarray(a, np.float32), device=self.dev).contiguous()
              for a in (in_shift, in_scale, out_shift, out_scale)]
        self._check(lib().mlp_set_scaling(self.ctx, *[_ptr(t) for t in ts], _stream()))
        self.torch.cuda.synchronize()

    def forward(self, theta):
        """theta [B, n_in] (device FP32) -> Y [B, n_out], J [B, n_out, n_in]."""
        th = theta.contiguous()
        B = th.shape[0]
        Y = self.torch.empty(B, self.n_out, dtype=self.torch.float32, device=self.dev)
        J = self.torch.empty(B, self.n_out, self.n_in, dtype=self.torch.float32, device=self.dev)
        self._check(lib().mlp_forward(self.ctx, _ptr(th), B, _ptr(Y), _ptr(J), _stream()))
        return Y, J

    def calibration_buffers(self, B: int):
        """Output tensors (Y, J, G, grad) for calibration_gradient(..., out=)
        on batches of B parameter vectors, for loops that evaluate again and
        again without allocating."""
        t, dev = self.torch, self.dev
        return (t.empty(B, self.n_out, dtype=t.float32, device=dev),
                t.empty(B, self.n_out, self.n_in, dtype=t.float32, device=dev),
                t.empty(B, dtype=t.float64, device=dev), t.empty(B, self.n_in, dtype=t.float64, device=dev))

    def calibration_gradient(self, theta, C, out=None):
        """theta [B, n_in] FP32, C [n_out] FP64 (device) -> G [B], grad [B, n_in]
        (FP64); out: tensors from calibration_buffers(B), written and returned
        instead of new ones."""
        th = theta.contiguous()
        B = th.shape[0]
        Y, J, G, g = out if out is not None else self.calibration_buffers(B)
        t = self.torch
        want = ((Y, (B, self.n_out), t.float32), (J, (B, self.n_out, self.n_in), t.float32), (G, (B,), t.float64),
                (g, (B, self.n_in), t.float64))
        for x, shape, dt in want:
            if tuple(x.shape) != shape or x.dtype != dt or not x.is_contiguous() or x.device != th.device:
                raise ValueError("output buffers must be those of calibration_buffers(B) for this batch")
        self._check(lib().mlp_calibration_gradient(self.ctx, _ptr(th), B, _ptr(C.contiguous()), _ptr(Y), _ptr(J),
                                                   _ptr(G), _ptr(g), _stream()))
        return G, g

    def loss_grad(self, theta, Ylab, Jlab, w: float, grad=None, loss=None):
        B = theta.shape[0]
        if grad is None:
            grad = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self.dev)
        if loss is None:
            loss = self.torch.empty(1, dtype=self.torch.float64, device=self.dev)
        self._check(lib().mlp_loss_grad(self.ctx, _ptr(theta), _ptr(Ylab), _ptr(Jlab), B, float(w), _ptr(loss),
                                        _ptr(grad), _stream()))
        return loss, grad

    def adam_step(self, grad, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        self._check(lib().mlp_adam_step(self.ctx, _ptr(grad), float(lr), float(beta1), float(beta2), float(eps),
                                        self.step_count, _stream()))

    def close(self):
        if self.ctx:
            lib().mlp_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# training labels from the Monte Carlo path (prices and tangent-mode Jacobian)
# ---------------------------------------------------------------------------
def generate_labels(problem, thetas: np.ndarray, n_paths: int, seed: int, inst0: int = 0,
                    chunk: int = 256, precision: str = "fp32"):
    """E y and dE y/dtheta for every row of thetas, each draw priced with its
    own paths (Philox key = seed, counter word 2 = inst0 + row)."""
    import torch
    pb = problem.with_(n_paths=n_paths, seed=seed)
    n = len(thetas)
    chunk = min(chunk, n)
    prec = capi.CAL_FP64 if precision == "fp64" else capi.CAL_FP32
    ctx = capi.cal_create(pb, prec, max_batch=chunk)
    m, M = pb.n_instr, pb.n_params
    Ey = torch.empty(n, m, dtype=torch.float64, device="cuda")
    J = torch.empty(n, m, M, dtype=torch.float64, device="cuda")
    th = torch.as_tensor(np.asarray(thetas, np.float64), device="cuda").contiguous()
    try:
        for s in range(0, n, chunk):
            k = min(chunk, n - s)
            capi.calibrate_jacobian_batch(ctx, th[s:s + k], k, inst0 + s, Ey[s:s + k], J[s:s + k])
        flags = capi.cal_status(ctx)
    finally:
        capi.cal_destroy(ctx)
    if flags:
        raise RuntimeError(f"label generation raised device status {flags}")
    return Ey, J


@dataclasses.dataclass
class TrainLog:
    epoch: int
    loss: float
    seconds: float


def fit(net: MLP, theta, Y, J, *, epochs: int, batch: int = 4096, lr: float = 1e-3, w: float = 1.0,
        lr_final: Optional[float] = None, seed: int = 0, log_every: int = 1) -> List[TrainLog]:
    """Adam on the differential loss over (theta, Y, J) device tensors (FP32).
    The learning rate decays geometrically to lr_final over the epochs."""
    import torch
    n = theta.shape[0]
    steps_per_epoch = n // batch
    assert steps_per_epoch >= 1, "need at least one full batch"
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    grad = torch.empty(net.n_params, dtype=torch.float32, device=net.dev)
    loss = torch.empty(1, dtype=torch.float64, device=net.dev)
    hist = []
    t0 = time.perf_counter()
    lr_f = lr if lr_final is None else lr_final
    for ep in range(epochs):
        lr_e = lr * (lr_f / lr) ** (ep / max(epochs - 1, 1))
        perm = torch.randperm(n, generator=g).to(net.dev)
        logged = (ep % log_every == 0) or ep == epochs - 1
        tot = torch.zeros(1, dtype=torch.float64, device=net.dev)   # summed on the device: no sync per step
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            net.loss_grad(theta[idx].contiguous(), Y[idx].contiguous(), J[idx].contiguous(), w, grad, loss)
            net.adam_step(grad, lr_e)
            if logged:
                tot += loss
        if logged:
            hist.append(TrainLog(ep, float(tot.item()) / steps_per_epoch, time.perf_counter() - t0))
    torch.cuda.synchronize()
    return hist


def standard_scaling(lo, hi, Y: np.ndarray):
    """Inputs mapped to [-1, 1]; outputs standardised per instrument."""
    lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
    mu = Y.mean(axis=0)
    sd = Y.std(axis=0) + 1e-6
    return (lo + hi) / 2, 2.0 / (hi - lo), mu, sd


# ---------------------------------------------------------------------------
# surrogate-assisted calibration step
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class StepRecord:
    it: int
    G_mc: float
    accepted_surrogate: bool
    grad_rel_err: float
    seconds_surrogate: float
    seconds_mc: float
    mc_calls: int = 1


def surrogate_calibration(net: MLP, mc, targets, theta0, lo, hi, *, iters: int = 20, alpha: float = 0.5,
                          feller: bool = True, max_backtracks: int = 12, g_stop: float = 0.0):
    """Each iteration proposes a step from the surrogate's gradient
    (projected, Armijo on the surrogate's G), then judges it with the Monte
    Carlo gradient at the proposal: accepted if the Monte Carlo G decreases,
    otherwise a Monte Carlo gradient step (with backtracking on the Monte
    Carlo G) is taken instead.  Every iteration logs the surrogate gradient's
    relative error against the Monte Carlo gradient and its Monte Carlo
    calls; the loop ends after `iters` iterations or once the Monte Carlo G
    is at most g_stop."""
    import torch
    from .calibrate import project
    lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
    D = (hi - lo) ** 2
    C = torch.as_tensor(np.asarray(targets, np.float64), device=mc.device)
    th = project(theta0, lo, hi, feller)
    recs = []

    def sur(th_):
        t = torch.as_tensor(np.asarray(th_, np.float32)[None, :], device=net.dev)
        G, g = net.calibration_gradient(t, C)
        return float(G.item()), g[0].cpu().numpy()

    Ey, G_mc, g_mc = mc.gradient(th, C)
    G_mc, g_mc = float(G_mc.item()), g_mc.cpu().numpy()
    for it in range(iters):
        if G_mc <= g_stop:
            break
        t0 = time.perf_counter()
        Gs, gs = sur(th)
        a = alpha
        cand = th
        for _ in range(max_backtracks):
            cand = project(th - a * D * gs, lo, hi, feller)
            if sur(cand)[0] <= Gs + 1e-4 * float(gs @ (cand - th)):
                break
            a *= 0.5
        ts = time.perf_counter() - t0
        t1 = time.perf_counter()
        Ey_c, G_c, g_c = mc.gradient(cand, C)
        G_c = float(G_c.item())
        tm = time.perf_counter() - t1
        err = float(np.linalg.norm(gs - g_mc) / max(np.linalg.norm(g_mc), 1e-300))
        accepted = G_c < G_mc
        calls = 1
        if accepted:
            th, G_mc, g_mc = cand, G_c, g_c.cpu().numpy()
        else:
            # fall back to a Monte Carlo gradient step
            a = alpha
            for _ in range(max_backtracks):
                cand = project(th - a * D * g_mc / max(np.max(np.abs(D * g_mc)), 1e-300) * 0.05, lo, hi, feller)
                Ey_c, G_c, g_c = mc.gradient(cand, C)
                calls += 1
                if float(G_c.item()) < G_mc:
                    th, G_mc, g_mc = cand, float(G_c.item()), g_c.cpu().numpy()
                    break
                a *= 0.5
        recs.append(StepRecord(it, G_mc, accepted, err, ts, tm, calls))
    return th, recs
