"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/mcaad.h declares, and rejects bad problems before
any HIP call."""
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1901_04200_amd import capi
from paper_1901_04200_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcaad.h")


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(capi.LIB_PATH):
        pytest.fail("libmcaad.so is not built; run __graft_entry__.build()")
    return capi.lib()


def test_header_declarations_are_exported(L):
    from paper_1901_04200_amd import batch, surrogate
    names = _declared()
    assert set(names) == set(capi.EXPORTED) | set(surrogate.EXPORTED) | set(batch.EXPORTED), names
    out = subprocess.run(["nm", "-D", "--defined-only", capi.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(L, n)


def _ok(pb, **kw):
    return capi.cal_validate(pb, **kw)


def test_validate_accepts_the_workloads(L):
    pb, _, _ = W.bs_problem()
    assert _ok(pb, precision=capi.CAL_FP64)[0] == capi.CAL_OK
    pb2, _, _, _ = W.heston_problem()
    assert _ok(pb2)[0] == capi.CAL_OK
    assert _ok(pb2, ckpt_every=32, ckpt_mode=capi.CAL_CKPT_RERUN)[0] == capi.CAL_OK
    # the smoothed square root exists in the oracle only
    rc, msg = _ok(pb2.with_(sqrt_eps=1e-4))
    assert rc == capi.CAL_EUNSUPPORTED and "sqrt_eps" in msg
    # Black-Scholes with the Euler scheme on S: one parameter, like log-Euler
    pbs, _, _ = W.bs_problem(euler_on_s=True)
    assert _ok(pbs, precision=capi.CAL_FP64)[0] == capi.CAL_OK
    rc, msg = _ok(pbs.with_(n_params=2))
    assert rc == capi.CAL_EINVAL and "n_params" in msg


@pytest.mark.parametrize("change,expect", [
    (dict(n_paths=0), "n_paths"),
    (dict(n_paths=(1 << 32) + 1), "n_paths"),
    (dict(n_steps=0), "n_steps"),
    (dict(instr_step=np.array([0, 1, 2, 3], dtype=np.int32)), "instr_step"),
    (dict(instr_step=np.array([1, 2, 3, 17], dtype=np.int32)), "instr_step"),
    (dict(instr_strike=np.array([1.0, -1.0, 2.0, 3.0])), "strike"),
    (dict(instr_strike=np.array([1.0, np.nan, 2.0, 3.0])), "strike"),
    (dict(s0=0.0), "s0"),
    (dict(t_max=-1.0), "t_max"),
    (dict(n_params=2), "n_params"),
    (dict(model=7), "model"),
    (dict(sqrt_eps=-1e-3), "sqrt_eps"),
])
def test_validate_rejects_bad_problems(L, change, expect):
    pb, _, _ = W.bs_problem()
    rc, msg = _ok(pb.with_(**change))
    assert rc == capi.CAL_EINVAL
    assert expect in msg


def test_validate_rejects_bad_options(L):
    pb, _, _, _ = W.heston_problem()
    assert _ok(pb, ckpt_every=12)[0] == capi.CAL_EINVAL
    assert _ok(pb, ckpt_mode=5)[0] == capi.CAL_EINVAL
    assert _ok(pb, precision=3)[0] == capi.CAL_EINVAL
    assert _ok(pb.with_(instr_step=np.zeros(0, np.int32), instr_strike=np.zeros(0)))[0] == capi.CAL_EINVAL
    big = 2049
    assert _ok(pb.with_(instr_step=np.full(big, 1, np.int32), instr_strike=np.ones(big)))[0] == capi.CAL_EINVAL


def test_local_vol_validation(L):
    pb = W.lv_problem(n_paths=1024)[0]
    assert _ok(pb)[0] == capi.CAL_OK
    k = pb.k_nodes.copy()
    k[3] += 0.5
    rc, msg = _ok(pb.with_(k_nodes=k))
    assert rc == capi.CAL_EINVAL and "uniformly" in msg
    t = pb.t_nodes.copy()
    t[2] = t[1]
    assert _ok(pb.with_(t_nodes=t))[0] == capi.CAL_EINVAL
    assert _ok(pb.with_(n_params=199))[0] == capi.CAL_EINVAL
    assert _ok(pb.with_(sqrt_eps=1e-4))[0] == capi.CAL_EUNSUPPORTED


def test_paths_per_lane_validation(L):
    pb, _, _, _ = W.heston_problem()
    for ppl in (0, 1, 2, 4):
        assert capi.cal_validate(pb, paths_per_lane=ppl)[0] == capi.CAL_OK
    for ppl in (3, 8, -1):
        rc, msg = capi.cal_validate(pb, paths_per_lane=ppl)
        assert rc == capi.CAL_EINVAL and "paths_per_lane" in msg
    lv = W.lv_problem(n_paths=1024)[0]
    assert capi.cal_validate(lv, paths_per_lane=1)[0] == capi.CAL_OK
    assert capi.cal_validate(lv, paths_per_lane=2)[0] == capi.CAL_OK
    assert capi.cal_validate(lv, paths_per_lane=4)[0] == capi.CAL_EUNSUPPORTED
    slv = W.slv_problem(n_paths=1024)[0]
    assert capi.cal_validate(slv, paths_per_lane=4)[0] == capi.CAL_OK
    assert capi.cal_validate(slv.with_(n_params=204))[0] == capi.CAL_EINVAL
