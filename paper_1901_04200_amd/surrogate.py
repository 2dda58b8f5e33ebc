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
            "mlp_set_scaling", "mlp_forward", "mlp_loss_grad", "mlp_adam_step", "mlp_adam_step_dev",
            "mlp_calibration_gradient", "mlp_last_error")

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
            "mlp_loss_grad": ([vp, vp, vp, vp, vp, vp, i32, C.c_float, vp, vp, vp], C.c_int),
            "mlp_adam_step": ([vp, vp, C.c_float, C.c_float, C.c_float, C.c_float, i32, vp], C.c_int),
            "mlp_adam_step_dev": ([vp, vp, vp, C.c_float, C.c_float, C.c_float, vp, vp], C.c_int),
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

    def loss_grad(self, theta, Ylab, Jlab, w: float, grad=None, loss=None, jw=None, idx=None):
        """Differential loss and its gradient; jw: per-sample weights of the
        Jacobian term (None: all 1); idx [B] (int32, device): the batch's rows
        of theta, Ylab, Jlab and jw (None: the first B rows in order)."""
        B = theta.shape[0] if idx is None else idx.shape[0]
        if grad is None:
            grad = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self.dev)
        if loss is None:
            loss = self.torch.empty(1, dtype=self.torch.float64, device=self.dev)
        self._check(lib().mlp_loss_grad(self.ctx, _ptr(theta), _ptr(Ylab), _ptr(Jlab),
                                        None if jw is None else _ptr(jw), None if idx is None else _ptr(idx), B,
                                        float(w), _ptr(loss),
                                        _ptr(grad), _stream()))
        return loss, grad

    def adam_step(self, grad, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        self._check(lib().mlp_adam_step(self.ctx, _ptr(grad), float(lr), float(beta1), float(beta2), float(eps),
                                        self.step_count, _stream()))

    def adam_step_dev(self, grad, lr_dev, t_dev, beta1=0.9, beta2=0.999, eps=1e-8):
        """Adam with the learning rate lr_dev[0] and step count t_dev[0] read on
        the device (t_dev incremented there)."""
        self._check(lib().mlp_adam_step_dev(self.ctx, _ptr(grad), _ptr(lr_dev), float(beta1), float(beta2), float(eps),
                                            _ptr(t_dev), _stream()))

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
        lr_final: Optional[float] = None, seed: int = 0, log_every: int = 1, jw=None,
        graph: bool = True) -> List[TrainLog]:
    """Adam on the differential loss over (theta, Y, J) device tensors (FP32),
    jw: per-sample weights of the Jacobian term (device FP32, or None).
    The learning rate decays geometrically to lr_final over the epochs.

    The data stay where they are: each epoch's permutation (drawn on the
    host) goes to a device buffer, and every step's kernels read their batch
    through its slice of it; the learning rate and the Adam step count live
    on the device too.  An epoch therefore launches the same work every time:
    with graph=True the second epoch is captured in a HIP graph and replayed
    for every later one (no host launches per step), the first runs eagerly.
    The results do not depend on graph."""
    import torch
    n = theta.shape[0]
    steps_per_epoch = n // batch
    assert steps_per_epoch >= 1, "need at least one full batch"
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    dev = net.dev
    grad = torch.empty(net.n_params, dtype=torch.float32, device=dev)
    perm_dev = torch.empty(n, dtype=torch.int32, device=dev)
    lr_host = torch.empty(1, dtype=torch.float32, pin_memory=True)
    lr_dev = torch.empty(1, dtype=torch.float32, device=dev)
    t_dev = torch.full((1,), net.step_count + 1, dtype=torch.int32, device=dev)
    losses = torch.zeros(steps_per_epoch, dtype=torch.float64, device=dev)   # one slot per step: no sync
    theta, Y, J = theta.contiguous(), Y.contiguous(), J.contiguous()
    jw = None if jw is None else jw.contiguous()

    def epoch():
        for s in range(steps_per_epoch):
            net.loss_grad(theta, Y, J, w, grad, losses[s:s + 1], jw=jw, idx=perm_dev[s * batch:(s + 1) * batch])
            net.adam_step_dev(grad, lr_dev, t_dev)

    hist = []
    t0 = time.perf_counter()
    lr_f = lr if lr_final is None else lr_final
    cg = None
    for ep in range(epochs):
        lr_e = lr * (lr_f / lr) ** (ep / max(epochs - 1, 1))
        perm_dev.copy_(torch.randperm(n, generator=g).to(torch.int32))
        lr_host[0] = lr_e
        lr_dev.copy_(lr_host, non_blocking=True)
        if graph and ep >= 1:
            if cg is None:
                torch.cuda.synchronize()
                cg = torch.cuda.CUDAGraph()
                with torch.cuda.graph(cg):
                    epoch()
            cg.replay()
        else:
            epoch()
        if (ep % log_every == 0) or ep == epochs - 1:
            hist.append(TrainLog(ep, float(losses.sum().item()) / steps_per_epoch, time.perf_counter() - t0))
    torch.cuda.synchronize()
    net.step_count += epochs * steps_per_epoch
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
    radius: float = 0.0
    ratio: float = 0.0
    inner_launches: int = 0


class DeviceSurrogate:
    """The trained network as the calibration step's model: at a batch of
    parameter vectors (all trial points of one step in one launch) its
    prices Y, Jacobians J and, given targets, G = 1/2 |Y - C|^2 and
    J^T (Y - C).  Buffers and their addresses are fixed once; the outputs sit
    side by side in one device buffer, so one copy and one synchronisation
    bring them back; the targets are uploaded only when they change."""

    def __init__(self, net: MLP, max_points: int = 32):
        import torch
        self.net, self.torch = net, torch
        self.max_points = B = max_points
        n, o = net.n_in, net.n_out
        self.n, self.o = n, o
        dev = net.dev
        self.th_host = torch.zeros(B, n, dtype=torch.float32, pin_memory=True)
        self.th_dev = torch.zeros(B, n, dtype=torch.float32, device=dev)
        self.C_host = torch.zeros(o, dtype=torch.float64, pin_memory=True)
        self.C_dev = torch.zeros(o, dtype=torch.float64, device=dev)
        self.C_now = None
        # one buffer: G [B], grad [B, n] (FP64), then Y [B, o], J [B, o, n] (FP32)
        self.nG, self.nY, self.nJ = 8 * B * (1 + n), 4 * B * o, 4 * B * o * n
        tot = self.nG + self.nY + self.nJ
        self.raw = torch.empty(tot, dtype=torch.uint8, device=dev)
        self.raw_host = torch.empty(tot, dtype=torch.uint8, pin_memory=True)
        self.raw_np = self.raw_host.numpy()
        self.th_np, self.C_np = self.th_host.numpy(), self.C_host.numpy()
        vp = C.c_void_p
        base = self.raw.data_ptr()
        self.p_G, self.p_Y, self.p_J = base, base + self.nG, base + self.nG + self.nY
        self.p_th, self.p_C = vp(self.th_dev.data_ptr()), vp(self.C_dev.data_ptr())
        self.launches = 0

    def evaluate(self, thetas, C_):
        """(Y [B, o], J [B, o, n], G [B], grad [B, n]) as host arrays at the
        rows of thetas, with targets C_ (FP64 [o])."""
        t = self.torch
        B, n, o = len(thetas), self.n, self.o
        if B > self.max_points:
            raise ValueError(f"at most {self.max_points} points per launch")
        self.th_np[:B] = thetas
        self.th_dev.copy_(self.th_host, non_blocking=True)
        if self.C_now is None or not np.array_equal(C_, self.C_now):
            self.C_now = np.array(C_, dtype=np.float64)
            self.C_np[:] = self.C_now
            self.C_dev.copy_(self.C_host, non_blocking=True)
        vp = C.c_void_p
        self.net._check(lib().mlp_calibration_gradient(
            self.net.ctx, self.p_th, B, self.p_C, vp(self.p_Y), vp(self.p_J), vp(self.p_G), vp(self.p_G + 8 * B),
            vp(t.cuda.current_stream().cuda_stream)))
        self.launches += 1
        self.raw_host.copy_(self.raw, non_blocking=True)
        t.cuda.current_stream().synchronize()
        r = self.raw_np
        Gg = r[:self.nG].view(np.float64)
        Y = r[self.nG:self.nG + self.nY].view(np.float32)[:B * o].reshape(B, o).astype(np.float64)
        J = r[self.nG + self.nY:].view(np.float32)[:B * o * n].reshape(B, o, n).astype(np.float64)
        return Y, J, Gg[:B].copy(), Gg[B:B * (1 + n)].reshape(B, n).copy()


def _lm_candidates(u0, gm, Ju, lo_u, hi_u, feasible):
    """Trial points from u0 for a least-squares model with gradient gm and
    Jacobian Ju (both in box-scaled coordinates): Levenberg-Marquardt steps
    -(Ju^T Ju + mu I)^-1 gm for a ladder of mu (from pure Gauss-Newton to
    nearly gradient steps) at full and half length, and two projected
    gradient steps, all projected onto the feasible set; [B, M]."""
    M = len(u0)
    H = Ju.T @ Ju
    scale = max(float(np.trace(H)) / M, 1e-300)
    mus = scale * np.array([1e-8, 1e-4, 1e-3, 1e-2, 1e-1, 1.0, 10.0])
    A = H[None, :, :] + mus[:, None, None] * np.eye(M)[None, :, :]
    steps = -np.linalg.solve(A, np.broadcast_to(gm, (len(mus), M))[:, :, None])[:, :, 0]
    gstep = -gm / max(float(np.max(np.abs(gm))), 1e-300) * float(np.max(hi_u - lo_u))
    pts = np.concatenate([u0 + steps, u0 + 0.5 * steps, (u0 + gstep)[None, :], (u0 + 0.25 * gstep)[None, :]])
    return feasible(pts, lo_u, hi_u)


def trust_region_calibration(mc_value_grad, sur_eval, targets, theta0, lo, hi, *, iters: int = 50,
                             g_stop: float = 0.0, feller: bool = True, radius0: float = 0.5, model_steps: int = 2,
                             eta: float = 0.05):
    """Surrogate-assisted calibration: a trust-region iteration whose model
    is the surrogate made exact to first order at the current point, and
    whose judge is the Monte Carlo gradient.

    At theta_k the Monte Carlo path gives E y_k, G_k and g_k (one two-pass
    gradient).  The surrogate's prices y_s are shifted so that they equal
    E y_k at theta_k (the surrogate's functional with targets
    C' = C - E y_k + y_s(theta_k)), and a linear term c (theta - theta_k) with
    c = g_k - J_s(theta_k)^T (E y_k - C) makes its gradient there g_k:
        m(theta) = G_s(theta; C') + c (theta - theta_k),  m(theta_k) = G_k.
    m is minimised over the box intersected with |u - u_k|_inf <= radius
    (u: box-scaled coordinates) by `model_steps` batched Gauss-Newton steps
    on the surrogate alone: from the current point, Levenberg-Marquardt steps
    for a ladder of damping values with the surrogate's Jacobian, all
    evaluated in one launch, the best kept.  The Monte Carlo gradient at the
    result theta_c decides: accepted when G(theta_c) < G_k (then its
    gradient is the next iteration's), the radius grows when the actual
    decrease is at least 3/4 of the predicted one at a step on the boundary
    and shrinks to a quarter of the step when the ratio is below eta.  After
    two rejections in a row the next trial point is a projected L-BFGS step
    on the Monte Carlo gradients themselves (the curvature pairs every Monte
    Carlo call leaves), inside the radius.  Every iteration costs one Monte
    Carlo gradient; the surrogate supplies the curvature, the Monte Carlo
    gradient the first-order term, the verdict and the fallback.

    mc_value_grad(theta) -> (E y, G, grad); sur_eval(thetas [B, M], C) ->
    (Y [B, m], J [B, m, M], G [B], grad [B, M]).  Returns
    (theta, [StepRecord])."""
    from .calibrate import LbfgsMemory
    lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
    w = hi - lo
    C = np.asarray(targets, np.float64)

    def feasible(u, lo_u, hi_u):
        """Points [B, M] clipped to [lo_u, hi_u], then (Heston) xi lowered
        onto Feller's condition 2 kappa theta_bar >= xi^2."""
        u = np.clip(u, lo_u, hi_u)
        if feller:
            th = lo + w * u
            xi_max = np.maximum(np.sqrt(np.maximum(2.0 * th[:, 0] * th[:, 1], 0.0)), lo[2])
            th[:, 2] = np.minimum(th[:, 2], xi_max)
            u = (th - lo) / w
        return u

    u = feasible(((np.asarray(theta0, np.float64) - lo) / w)[None, :], 0.0, 1.0)[0]
    th = lo + w * u
    Ey, G, g = mc_value_grad(th)
    radius = radius0
    mc_mem = LbfgsMemory(8)
    rejected = 0
    ys = Js = None          # the surrogate's prices and Jacobian at theta_k, when known
    recs: List[StepRecord] = []
    for it in range(iters):
        if G <= g_stop or radius < 1e-9:
            break
        t0 = time.perf_counter()
        lo_u, hi_u = np.maximum(0.0, u - radius), np.minimum(1.0, u + radius)
        gk_u = np.asarray(g) * w
        err, launches = float("nan"), 0
        if rejected >= 2:
            # fallback: projected L-BFGS step on the Monte Carlo gradients
            free = ~(((u <= 0.0) & (gk_u > 0.0)) | ((u >= 1.0) & (gk_u < 0.0)))
            d = mc_mem.apply(gk_u, free)
            if not float(gk_u @ d) < 0.0:
                d = -np.where(free, gk_u, 0.0)
            a = 1.0 if mc_mem.s else radius / max(float(np.max(np.abs(d))), 1e-300)
            u_c = feasible((u + a * d)[None, :], lo_u, hi_u)[0]
            m_c = G + float(gk_u @ (u_c - u))       # the linear model's value
            source = False
            ys_c = Js_c = None
        else:
            if ys is None:
                Y0, J0, _, _ = sur_eval(th[None, :], C)
                launches += 1
                ys, Js = Y0[0], J0[0]
            Cp = C - np.asarray(Ey) + ys
            c = np.asarray(g) - Js.T @ (np.asarray(Ey) - C)
            err = float(np.linalg.norm(Js.T @ (np.asarray(Ey) - C) - g) / max(np.linalg.norm(g), 1e-300))
            u_b, m_b, gm_b, J_b, y_b = u, G, gk_u, Js * w[None, :], ys
            for _ in range(model_steps):
                pts = _lm_candidates(u_b, gm_b, J_b, lo_u, hi_u, feasible)
                pts_th = lo + w * pts
                Yc, Jc, Gc, gc = sur_eval(pts_th, Cp)
                launches += 1
                mvals = Gc + (pts_th - th) @ c
                j = int(np.argmin(np.where(np.isfinite(mvals), mvals, np.inf)))
                if not mvals[j] < m_b:
                    break
                u_b, m_b, gm_b, J_b, y_b = pts[j], float(mvals[j]), (gc[j] + c) * w, Jc[j] * w[None, :], Yc[j]
            u_c, m_c = u_b, m_b
            ys_c, Js_c = y_b, J_b / w[None, :]
            source = True
        th_c = lo + w * u_c
        t_s = time.perf_counter() - t0
        pred = G - m_c
        step = float(np.max(np.abs(u_c - u)))
        if step == 0.0 or not pred > 0.0:
            radius *= 0.25
            rejected += 1
            recs.append(StepRecord(it, float(G), False, err, t_s, 0.0, 0, radius, 0.0, launches))
            continue
        t1 = time.perf_counter()
        Ey_c, G_c, g_c = mc_value_grad(th_c)
        t_mc = time.perf_counter() - t1
        ratio = (G - G_c) / pred
        accepted = bool(np.isfinite(G_c) and G_c < G)
        if np.all(np.isfinite(g_c)):
            mc_mem.push(u_c - u, np.asarray(g_c) * w - gk_u)
        if accepted:
            u, th, Ey, G, g = u_c, th_c, Ey_c, G_c, g_c
            ys, Js = ys_c, Js_c
            rejected = 0
        else:
            rejected += 1
        if ratio >= 0.75 and step >= 0.8 * radius:
            radius = min(2.0 * radius, 1.0)
        elif ratio < eta or not accepted:
            radius = 0.25 * step
        recs.append(StepRecord(it, float(G), accepted and source, err, t_s, t_mc, 1, radius, float(ratio), launches))
    return th, recs


def surrogate_calibration(net: MLP, mc, targets, theta0, lo, hi, *, iters: int = 50, feller: bool = True,
                          g_stop: float = 0.0, **kw):
    """trust_region_calibration with the trained network on the device as
    the model and the library's two-pass Monte Carlo gradient as the judge.
    Returns (theta, [StepRecord])."""
    from .calibrate import MonteCarloObjective
    C_ = np.asarray(targets, np.float64)
    sur = DeviceSurrogate(net, max_points=16)
    obj = MonteCarloObjective(mc, C_)
    return trust_region_calibration(obj.prices_value_and_grad, sur.evaluate, C_, theta0, lo, hi, iters=iters,
                                    g_stop=g_stop, feller=feller, **kw)
