"""GPU parity of the surrogate kernels against the FP64 MLP oracle, and of
its training labels against the FP64 Monte Carlo oracle.

Tolerance (derived from the arithmetic): the oracle is given the device's
bf16-rounded weights, so the remaining difference is the bf16 rounding of
activations and adjoints where they enter the products (relative u = 2^-9
per rounding, a few roundings deep) plus FP32 accumulation: outputs within
2e-2 of their largest magnitude; every weight-gradient element within
16 u times its running-error magnitude (the oracle's backward pass with
every factor taken in absolute value: a term whose factors carry relative
errors e1, e2, ... is off by at most (e1 + e2 + ...) times its magnitude;
16 covers the roundings along the deepest term, three forward and three
backward products with their activations, with room).  Labels (FP32 Monte Carlo) follow the Monte Carlo
bounds: 1e-5 on prices, 1e-4 on the Jacobian.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mlp_oracle as MO
from oracle import parity as PY
from paper_1901_04200_amd import surrogate as S
from paper_1901_04200_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def bf16(x):
    u = np.asarray(x, np.float32).copy().view(np.uint32)
    u = (u + np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))) & np.uint32(0xFFFF0000)
    return u.view(np.float32).astype(np.float64)


def rand_params(sizes, seed):
    rng = np.random.default_rng(seed)
    ps = []
    for a, c in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / a)
        ps.append((rng.uniform(-lim, lim, (a, c)).astype(np.float32), rng.normal(0, 0.1, c).astype(np.float32)))
    return ps


def device_view(params):
    """The weights the device multiplies with: bf16 copies of W (first layer
    and biases stay FP32)."""
    out = []
    for l, (Wt, b) in enumerate(params):
        out.append((Wt.astype(np.float64) if l == 0 else bf16(Wt), b.astype(np.float64)))
    return out


@pytest.mark.parametrize("H,nout,B", [(128, 7, 128), (128, 7, 5), (256, 40, 4096)])
def test_forward_and_jacobian(H, nout, B):
    say(f"mlp forward H={H} n_out={nout} B={B}")
    net = S.MLP(5, H, nout, max_batch=max(B, 128))
    params = rand_params([5, H, H, H, nout], 1)
    net.set_params(net.pack(params))
    X = np.random.default_rng(2).uniform(-1, 1, (B, 5)).astype(np.float32)
    Y, J = net.forward(torch.as_tensor(X, device="cuda"))
    Y, J = Y.cpu().numpy(), J.cpu().numpy()
    Yo, Jo = MO.forward_tangent(device_view(params), X.astype(np.float64))
    ey = np.max(np.abs(Y - Yo)) / np.max(np.abs(Yo))
    ej = np.max(np.abs(J - Jo)) / np.max(np.abs(Jo))
    say(f"  rel err Y {ey:.2e} J {ej:.2e}")
    assert ey < 2e-2 and ej < 2e-2
    net.close()


@pytest.mark.parametrize("nin,H,nout,B", [(5, 1024, 40, 3), (8, 128, 7, 2), (9, 128, 7, 2), (1, 128, 3, 64)])
def test_forward_shapes_against_oracle(nin, H, nout, B):
    """Both evaluation paths (one launch per call for small batches with
    n_in <= 8, the GEMM path otherwise) against the oracle."""
    say(f"mlp forward n_in={nin} H={H} n_out={nout} B={B}")
    net = S.MLP(nin, H, nout, max_batch=128)
    params = rand_params([nin, H, H, H, nout], 11)
    net.set_params(net.pack(params))
    X = np.random.default_rng(12).uniform(-1, 1, (B, nin)).astype(np.float32)
    Y, J = net.forward(torch.as_tensor(X, device="cuda"))
    Yo, Jo = MO.forward_tangent(device_view(params), X.astype(np.float64))
    ey = np.max(np.abs(Y.cpu().numpy() - Yo)) / np.max(np.abs(Yo))
    ej = np.max(np.abs(J.cpu().numpy() - Jo)) / np.max(np.abs(Jo))
    say(f"  rel err Y {ey:.2e} J {ej:.2e}")
    assert ey < 2e-2 and ej < 2e-2
    net.close()


@pytest.mark.parametrize("H,nout", [(128, 7), (256, 40)])
def test_small_batches_match_the_gemm_path(H, nout):
    """A sample evaluated in a batch of 1 or 64 (one launch) and in a batch of
    200 (GEMMs): the same MFMA products on the same bf16 operands, summed over
    k in the same order, and the same elementwise arithmetic, so the outputs,
    the functional and its gradient are bitwise the same."""
    net = S.MLP(5, H, nout, max_batch=256)
    net.set_params(net.pack(rand_params([5, H, H, H, nout], 13)))
    X = torch.as_tensor(np.random.default_rng(14).uniform(-1, 1, (200, 5)), dtype=torch.float32, device="cuda")
    C = torch.linspace(-1.0, 1.0, nout, dtype=torch.float64, device="cuda")
    Yb, Jb = net.forward(X)
    Gb, gb = net.calibration_gradient(X, C)
    Yb, Jb, Gb, gb = (t.cpu().numpy() for t in (Yb, Jb, Gb, gb))
    for B in (1, 64):
        Ys, Js = net.forward(X[:B])
        Gs, gs = net.calibration_gradient(X[:B], C)
        Ys, Js, Gs, gs = (t.cpu().numpy() for t in (Ys, Js, Gs, gs))
        ey = np.max(np.abs(Ys - Yb[:B])) / np.max(np.abs(Yb[:B]))
        ej = np.max(np.abs(Js - Jb[:B])) / np.max(np.abs(Jb[:B]))
        say(f"  H={H} B={B}: small vs GEMM path, rel diff Y {ey:.1e} J {ej:.1e}")
        for a, c in ((Ys, Yb[:B]), (Js, Jb[:B]), (Gs, Gb[:B]), (gs, gb[:B])):
            np.testing.assert_array_equal(a, c)
    net.close()


def test_scaling_maps_units():
    net = S.MLP(5, 128, 7, max_batch=128)
    params = rand_params([5, 128, 128, 128, 7], 3)
    net.set_params(net.pack(params))
    lo, hi = W.HESTON_LO, W.HESTON_HI
    shift, scale = (lo + hi) / 2, 2 / (hi - lo)
    oshift, oscale = np.linspace(1, 7, 7), np.linspace(0.5, 2, 7)
    net.set_scaling(shift, scale, oshift, oscale)
    th = W.heston_draws(9, 128).astype(np.float32)
    Y, J = net.forward(torch.as_tensor(th, device="cuda"))
    Yo, Jo = MO.forward_tangent(device_view(params), (th.astype(np.float64) - shift) * scale)
    Yo = Yo * oscale + oshift
    Jo = Jo * oscale[None, :, None] * scale[None, None, :]
    assert np.max(np.abs(Y.cpu().numpy() - Yo)) < 2e-2 * np.max(np.abs(Yo))
    assert np.max(np.abs(J.cpu().numpy() - Jo)) < 2e-2 * np.max(np.abs(Jo))
    net.close()


@pytest.mark.parametrize("nin,H,nout,B,weighted", [(5, 128, 7, 256, False), (5, 256, 40, 4096, False),
                                                  (5, 256, 40, 512, True), (1, 512, 64, 128, False),
                                                  (7, 256, 40, 256, True), (8, 128, 5, 128, False),
                                                  (16, 1024, 3, 128, False)])
def test_loss_and_double_backprop(nin, H, nout, B, weighted):
    """Widths 128 to 1024 (4 to 32 k-tiles per product, 1 to 48 split-K
    partials of the weight gradients), one to sixteen inputs (up to seven on
    the fused row-block kernels, above on the separate ones), the widest
    output tile (64 units), per-sample Jacobian-term weights (some zero, with
    non-finite labels there that must never be read as numbers)."""
    say(f"mlp loss/grad n_in={nin} H={H} n_out={nout} B={B} weighted={weighted}")
    net = S.MLP(nin, H, nout, max_batch=B)
    params = rand_params([nin, H, H, H, nout], 5)
    net.set_params(net.pack(params))
    rng = np.random.default_rng(6)
    X = rng.uniform(-1, 1, (B, nin)).astype(np.float32)
    Yl = rng.normal(0, 1, (B, nout)).astype(np.float32)
    Jl = rng.normal(0, 1, (B, nout, nin)).astype(np.float32)
    w = 0.8
    jw = (rng.integers(0, 3, B) * 0.5).astype(np.float32) if weighted else None
    Jdev = Jl.copy()
    if weighted:
        Jdev[jw == 0] = np.inf     # labels of zero-weight samples are never read
    loss, grad = net.loss_grad(*(torch.as_tensor(a, device="cuda") for a in (X, Yl, Jdev)), w,
                               jw=None if jw is None else torch.as_tensor(jw, device="cuda"))
    L, go = MO.grads(device_view(params), X.astype(np.float64), Yl.astype(np.float64), Jl.astype(np.float64), w,
                     jw=jw)
    say(f"  loss gpu {loss.item():.6g} oracle {L:.6g}")
    assert abs(loss.item() - L) < 2e-2 * L
    gg = net.unpack(grad.cpu().numpy())
    mag = MO.grad_magnitudes(device_view(params), X.astype(np.float64), Yl.astype(np.float64),
                             Jl.astype(np.float64), w, jw=jw)
    u = 2.0 ** -9
    for l in range(4):
        for k in range(2):
            a, b, mg = gg[l][k], go[l][k], mag[l][k]
            ratio = np.abs(a - b) / np.maximum(u * mg, 1e-30)
            e = np.linalg.norm(a - b) / np.linalg.norm(b)
            say(f"  layer {l + 1} {'W' if k == 0 else 'b'}: rel norm err {e:.2e}, largest |error| / (u magnitude) "
                f"{ratio.max():.2f}, median {np.median(ratio):.3f}")
            assert np.all(np.abs(a - b) <= 16 * u * mg + 1e-7 * np.max(np.abs(b))), (l, k)
    net.close()


def test_adam_step_matches_reference():
    net = S.MLP(5, 128, 7, max_batch=128)
    params = rand_params([5, 128, 128, 128, 7], 8)
    p0 = net.pack(params)
    net.set_params(p0)
    rng = np.random.default_rng(9)
    m = np.zeros_like(p0, dtype=np.float64)
    v = np.zeros_like(p0, dtype=np.float64)
    p = p0.astype(np.float64)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    for t in range(1, 4):
        g = rng.normal(0, 1, p0.size).astype(np.float32)
        net.adam_step(torch.as_tensor(g, device="cuda"), lr, b1, b2, eps)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g.astype(np.float64) ** 2
        p = p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    np.testing.assert_allclose(net.get_params(), p, rtol=1e-5, atol=1e-7)
    net.close()


def test_calibration_gradient_kernel():
    """G = 1/2 |y - C|^2 and J^T (y - C): exactly those of the network's own
    outputs, and within the bounds that the forward tolerance implies of the
    oracle's."""
    net = S.MLP(5, 128, 7, max_batch=128)
    net.set_params(net.pack(rand_params([5, 128, 128, 128, 7], 4)))
    th = torch.as_tensor(np.random.default_rng(5).uniform(-1, 1, (9, 5)), dtype=torch.float32, device="cuda")
    C = torch.linspace(-1.0, 1.0, 7, dtype=torch.float64, device="cuda")
    params = rand_params([5, 128, 128, 128, 7], 4)
    G, g = net.calibration_gradient(th, C)
    Y, J = net.forward(th)
    r = Y.double().cpu().numpy() - C.cpu().numpy()
    np.testing.assert_allclose(G.cpu().numpy(), 0.5 * np.sum(r * r, axis=1), rtol=1e-12)
    np.testing.assert_allclose(g.cpu().numpy(), np.einsum("bij,bi->bj", J.double().cpu().numpy(), r), rtol=1e-10,
                               atol=1e-12)
    # against the oracle: with every output within ey of the oracle's and every
    # Jacobian entry within ej (the forward tolerance, 2e-2 of the largest
    # magnitude), G_b = 1/2 |r_b|^2 is off by at most sum_i (|r_i| ey + ey^2 / 2)
    # and g_bj = sum_i J_bij r_bi by at most sum_i (ej |r_i| + |J_ij| ey + ej ey)
    Yo, Jo = MO.forward_tangent(device_view(params), th.double().cpu().numpy())
    ro = Yo - C.cpu().numpy()
    ey, ej = 2e-2 * np.max(np.abs(Yo)), 2e-2 * np.max(np.abs(Jo))
    Go, go = 0.5 * np.sum(ro * ro, axis=1), np.einsum("bij,bi->bj", Jo, ro)
    G_tol = np.sum(np.abs(ro) * ey + 0.5 * ey * ey, axis=1)
    g_tol = np.einsum("bij,bi->bj", np.abs(Jo), np.full_like(ro, ey)) + ej * np.sum(np.abs(ro) + ey, axis=1)[:, None]
    dG, dg = np.abs(G.cpu().numpy() - Go), np.abs(g.cpu().numpy() - go)
    say(f"  calibration gradient vs oracle: G {np.max(dG / G_tol):.2f}, g {np.max(dg / g_tol):.2f} of the bounds")
    assert np.all(dG <= G_tol) and np.all(dg <= g_tol)
    # into preallocated buffers: the same values, twice in a row
    bufs = net.calibration_buffers(9)
    for _ in range(2):
        G2, g2 = net.calibration_gradient(th, C, out=bufs)
        assert G2.data_ptr() == bufs[2].data_ptr() and g2.data_ptr() == bufs[3].data_ptr()
        assert torch.equal(G2, G) and torch.equal(g2, g)
    with pytest.raises(ValueError):
        net.calibration_gradient(th, C, out=net.calibration_buffers(8))
    Y8, J8, G8, g8 = net.calibration_buffers(9)
    with pytest.raises(ValueError):
        net.calibration_gradient(th, C, out=(Y8, J8, G8.float(), g8))
    net.close()


def test_labels_match_oracle_jacobian(orc):
    """calibrate_jacobian_batch on 8 draws at 2^16 paths (own Philox
    instance each) against the oracle's tangent mode with the same streams;
    the FP32 Jacobian is asserted on the draws where no path carries more
    than 2% of any Jacobian entry, the rest stated."""
    pb, _, _, _ = W.heston_problem(n_paths=1 << 16)
    draws = W.heston_feller_draws(6, 8)
    Ey, J = S.generate_labels(pb, draws, n_paths=1 << 16, seed=4, inst0=100, chunk=8)
    Ey, J = Ey.cpu().numpy(), J.cpu().numpy()
    Ey64, J64 = S.generate_labels(pb, draws, n_paths=1 << 16, seed=4, inst0=100, chunk=8, precision="fp64")
    Ey64, J64 = Ey64.cpu().numpy(), J64.cpu().numpy()
    n_checked = 0
    for i, th in enumerate(draws):
        sub = pb.with_(seed=4, inst=100 + i)
        Eo, Jo, _, dyp = orc.jacobian(sub, th, per_path=True)
        # conditioning: the largest share of one path in any Jacobian column
        col = dyp.sum(axis=1)
        share = float(np.max(np.abs(col).max(0) / np.abs(col.sum(0))))
        ey = np.max(np.abs(Ey[i] - Eo) / np.maximum(np.abs(Eo), 1e-2))
        ej = np.max(np.abs(J[i] - Jo)) / np.max(np.abs(Jo))
        ej64 = np.max(np.abs(J64[i] - Jo)) / np.max(np.abs(Jo))
        say(f"  draw {i}: one-path share {share:.3f}; fp32 Ey {ey:.2e} J {ej:.2e}; fp64 J {ej64:.2e}")
        assert np.max(np.abs(Ey64[i] - Eo) / np.maximum(np.abs(Eo), 1e-2)) <= 1e-12
        assert ej64 <= 1e-9
        assert ey <= 1e-5
        if share <= PY.SHARE_GATE:
            assert ej <= 1e-4
            n_checked += 1
    assert n_checked >= 4


def test_training_reduces_loss():
    """A short fit on Monte Carlo labels lowers the differential loss."""
    pb, _, _, _ = W.heston_problem(n_paths=1 << 12)
    draws = W.heston_feller_draws(12, 1024)
    Ey, J = S.generate_labels(pb, draws, n_paths=1 << 12, seed=4, chunk=256)
    net = S.MLP(5, 256, 40, max_batch=512)
    net.init_params(0)
    sh, sc, mu, sd = S.standard_scaling(W.HESTON_LO, W.HESTON_HI, Ey.cpu().numpy())
    net.set_scaling(sh, sc, mu, sd)
    th = torch.as_tensor(draws, dtype=torch.float32, device="cuda")
    hist = S.fit(net, th, Ey.float(), J.float(), epochs=30, batch=512, lr=2e-3, w=0.1)
    say(f"  loss {hist[0].loss:.4g} -> {hist[-1].loss:.4g}")
    assert hist[-1].loss < 0.1 * hist[0].loss
    net.close()


def test_surrogate_assisted_calibration():
    """The surrogate-assisted iteration only accepts Monte Carlo improvements
    (G never rises), makes at most one Monte Carlo call per iteration, and
    stops at g_stop."""
    from paper_1901_04200_amd.mc import MonteCarloCalibration
    pb, _, _, _ = W.heston_problem(n_paths=1 << 14)
    draws = W.heston_feller_draws(12, 1024)
    Ey, J = S.generate_labels(pb, draws, n_paths=1 << 12, seed=4, chunk=256)
    net = S.MLP(5, 256, 40, max_batch=512)
    net.init_params(0)
    sh, sc, mu, sd = S.standard_scaling(W.HESTON_LO, W.HESTON_HI, Ey.cpu().numpy())
    net.set_scaling(sh, sc, mu, sd)
    S.fit(net, torch.as_tensor(draws, dtype=torch.float32, device="cuda"), Ey.float(), J.float(), epochs=30,
          batch=512, lr=2e-3, w=0.1)
    th0, tht = W.heston_feller_draws(13, 2)
    mc = MonteCarloCalibration(pb)
    C = mc.forward(tht).cpu().numpy()
    G0 = float(mc.gradient(th0, C)[1].item())
    th, recs = S.surrogate_calibration(net, mc, C, th0, W.HESTON_LO, W.HESTON_HI, iters=12)
    Gs = [G0] + [r.G_mc for r in recs]
    say("  G:", " ".join(f"{g:.3g}" for g in Gs), "accepted", sum(r.accepted_surrogate for r in recs))
    assert all(b <= a for a, b in zip(Gs, Gs[1:]))
    assert Gs[-1] < G0
    assert all(r.mc_calls in (0, 1) for r in recs) and sum(r.mc_calls for r in recs) >= 1
    stop = 0.5 * (G0 + Gs[-1])
    _, recs2 = S.surrogate_calibration(net, mc, C, th0, W.HESTON_LO, W.HESTON_HI, iters=12, g_stop=stop)
    assert len(recs2) <= len(recs) and recs2[-1].G_mc <= stop
    mc.close()
    net.close()


def test_training_graph_matches_eager():
    """Training epochs replayed from a captured graph (batches through a
    device permutation buffer, learning rate and step count on the device)
    give the eager loop's parameters bit for bit, the losses too (each
    epoch's permutation and learning rate are copied in, and the loss read
    back, eagerly between the replays); another network's eager work after
    the loop does not disturb them."""
    rng = np.random.default_rng(21)
    n, nin, nout = 1024, 5, 40
    th = torch.as_tensor(rng.uniform(-1, 1, (n, nin)), dtype=torch.float32, device="cuda")
    Y = torch.as_tensor(rng.normal(0, 1, (n, nout)), dtype=torch.float32, device="cuda")
    J = torch.as_tensor(rng.normal(0, 1, (n, nout, nin)), dtype=torch.float32, device="cuda")
    jw = torch.as_tensor((rng.random(n) < 0.7).astype(np.float32), device="cuda")
    out = {}
    for graph in (False, True):
        net = S.MLP(nin, 256, nout, max_batch=256)
        net.init_params(3)
        other = S.MLP(nin, 128, 7, max_batch=128)
        other.init_params(4)
        hist = S.fit(net, th, Y, J, epochs=5, batch=256, lr=2e-3, lr_final=1e-3, w=0.5, jw=jw, graph=graph)
        other.forward(th[:128])
        out[graph] = (net.get_params(), [h.loss for h in hist])
        net.close()
        other.close()
    np.testing.assert_array_equal(out[True][0], out[False][0])
    assert out[True][1] == out[False][1]
