"""calibrate_gradient_static (the entry point that allocates nothing: its
buffers live in the library's static device array) against
calibrate_gradient on a context made from the same problem: the same E y,
G and gradient bit for bit, on consecutive calls of different sizes (the
second smaller, so stale contents of the array beyond its buffers cannot
matter), and a clear refusal of a problem too large for the array."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1901_04200_amd import capi
from paper_1901_04200_amd import workloads as W
from paper_1901_04200_amd.mc import MonteCarloCalibration

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    capi.lib()
    return torch.device("cuda", 0)


def both(pb, theta, C, precision, **kw):
    prec = capi.CAL_FP64 if precision == "fp64" else capi.CAL_FP32
    th = torch.as_tensor(np.asarray(theta, np.float64), device="cuda")
    Cd = torch.as_tensor(np.asarray(C, np.float64), device="cuda")
    m, M = pb.n_instr, pb.n_params
    out_s = [torch.full((n,), np.nan, dtype=torch.float64, device="cuda") for n in (m, 1, M)]
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    capi.calibrate_gradient_static(pb, th, Cd, *out_s, status, precision=prec, **kw)
    torch.cuda.synchronize()
    mc = MonteCarloCalibration(pb, precision=precision, ckpt_every=kw.get("ckpt_every", 0),
                               ckpt_mode={capi.CAL_CKPT_RERUN: "rerun"}.get(kw.get("ckpt_mode"), "auto"),
                               paths_per_lane=kw.get("paths_per_lane", 0))
    out_c = mc.gradient(theta, C)
    flags = mc.status()
    mc.close()
    return [t.cpu().numpy() for t in out_s], int(status.item()), [t.cpu().numpy() for t in out_c], flags


def test_static_matches_context_two_calls():
    # first call: the benchmark's workload (2^20 Heston paths x 256 steps, K = 16)
    pb, th0, tht, eps = W.heston_problem()
    th = W.heston_draws(2, 10)[9]
    C = np.linspace(2.0, 30.0, pb.n_instr)
    say("static vs context: heston fp32 2^20 x 256, K=16")
    s, st, c, flags = both(pb, th, C, "fp32", ckpt_every=16)
    assert st == 0 and flags == 0
    for a, b in zip(s, c):
        np.testing.assert_array_equal(a, b)
    # second call, smaller: Heston FP64 with a ragged path count, re-run mode, 2 paths per lane
    pb2, _, _, _ = W.heston_problem(n_paths=3 * 512 + 77, n_steps=72, t_max=0.5625)
    C2 = np.linspace(3.0, 9.0, pb2.n_instr)
    say("static vs context: heston fp64 1613 x 72, re-run mode, 2 paths per lane")
    s, st, c, flags = both(pb2, th, C2, "fp64", ckpt_mode=capi.CAL_CKPT_RERUN, paths_per_lane=2)
    assert st == 0 and flags == 0
    for a, b in zip(s, c):
        np.testing.assert_array_equal(a, b)
    # third, smaller again: Black-Scholes FP64, 4 instruments
    pb3, th3, C3 = W.bs_problem(n_paths=1000)
    say("static vs context: bs fp64 1000 x 16")
    s, st, c, flags = both(pb3, th3, C3, "fp64")
    assert st == 0 and flags == 0
    for a, b in zip(s, c):
        np.testing.assert_array_equal(a, b)


def test_static_reports_status_and_refuses_oversize():
    pb, _, _, _ = W.heston_problem(n_paths=4096, n_steps=64, t_max=0.5)
    th = np.array([1.0, 0.04, 0.5, -1.5, 0.04])       # rho outside (-1, 1)
    C = np.full(pb.n_instr, 5.0)
    say("static: theta outside the domain sets the status word")
    s, st, c, flags = both(pb, th, C, "fp32")
    assert st & capi.CAL_FLAG_THETA and flags & capi.CAL_FLAG_THETA
    big, _, _, _ = W.heston_problem(n_paths=1 << 22)
    m = big.n_instr
    bufs = [torch.empty(n, dtype=torch.float64, device="cuda") for n in (5, m, m, 1, 5)]
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    say("static: 2^22 Heston paths do not fit the static array")
    with pytest.raises(capi.CalError) as ei:
        capi.calibrate_gradient_static(big, *bufs, status, ckpt_every=16)
    assert ei.value.code == capi.CAL_EINVAL and "bytes of scratch" in str(ei.value)
    with pytest.raises(capi.CalError) as ei:
        capi.calibrate_gradient_static(W.lv_problem(n_paths=256)[0], *bufs[:2], bufs[1], bufs[3], bufs[4], status)
    assert ei.value.code == capi.CAL_EUNSUPPORTED
