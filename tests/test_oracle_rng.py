"""Pins for the oracle's random stream.

The paper only says that F consumes N independent random variables per path
(problem statement of F : R^{M+N} -> R^m).  The stream is Philox4x32-10
(Salmon et al., SC'11) with uniforms ((w >> 9) + 0.5) 2^-23 and Box-Muller
pairs.  Pins: the raw words against rocRAND's independent Philox engine, and
the normals against the standard normal law.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _counters(n, seed=12345):
    rng = np.random.default_rng(seed)
    cs = rng.integers(0, 2 ** 32, size=(n, 6), dtype=np.uint64)
    edge = []
    for v in (0, 1, 2 ** 31, 2 ** 32 - 1, 2 ** 32 - 2):
        edge.append([v, v, v, v, v, v])
        edge.append([v, 0, 0, 0, 0, 0])
        edge.append([0, v, 0, 0, v, 0])
        edge.append([0, 0, v, 0, 0, v])
        edge.append([0, 0, 0, v, 0, 0])
    edge += [[q, p, 0, 0, 1, 0] for q in range(4) for p in range(4)]
    return np.vstack([np.array(edge, dtype=np.uint64), cs])


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build rocRAND's host Philox")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_rocrand")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--cuda-host-only", "-I/opt/rocm/include",
                    os.path.join(HERE, "pins", "philox_rocrand.cpp"), "-o", exe], check=True)
    return exe


def test_philox_matches_rocrand(orc, rocrand_philox):
    cs = _counters(20000)
    inp = "\n".join(" ".join(str(int(v)) for v in row) for row in cs) + "\n"
    out = subprocess.run([rocrand_philox], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)
    assert ref.shape == (len(cs), 4)
    mine = np.array([orc.philox(row[:4], row[4:]) for row in cs], dtype=np.uint64)
    np.testing.assert_array_equal(mine, ref)


def test_philox_counter_and_key_sensitivity(orc):
    base = orc.philox([5, 6, 7, 8], [9, 10])
    for i in range(4):
        c = [5, 6, 7, 8]
        c[i] ^= 1
        assert orc.philox(c, [9, 10]) != base
    assert orc.philox([5, 6, 7, 8], [9, 11]) != base


def test_normals_law(orc):
    from scipy import stats
    z = np.concatenate([orc.normals(7, 0, p, 0, 4096) for p in range(4096)])  # 2^24 draws
    n = len(z)
    # the smallest uniform is 2^-24, so |z| <= sqrt(48 ln 2)
    assert np.abs(z).max() <= np.sqrt(48 * np.log(2)) + 1e-12
    se = 1.0 / np.sqrt(n)
    assert abs(z.mean()) < 4 * se
    assert abs(z.var() - 1.0) < 4 * np.sqrt(2.0 / n)
    kurt = np.mean(z ** 4)
    assert abs(kurt - 3.0) < 4 * np.sqrt(96.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # pairs from one Box-Muller draw and neighbouring pairs are uncorrelated
    zz = z.reshape(-1, 4)
    for a, b in ((0, 1), (2, 3), (1, 2), (0, 2)):
        assert abs(np.corrcoef(zz[:, a], zz[:, b])[0, 1]) < 4 / np.sqrt(len(zz))


def test_normals_layout(orc):
    """Normal q of a path comes from Philox call floor(q/4); slices agree."""
    full = orc.normals(3, 2, 11, 0, 64)
    for q0 in (0, 1, 3, 4, 17, 60):
        part = orc.normals(3, 2, 11, q0, 4)
        np.testing.assert_array_equal(part, full[q0:q0 + 4])
    # different paths / instances / seeds give different streams
    assert not np.array_equal(full, orc.normals(3, 2, 12, 0, 64))
    assert not np.array_equal(full, orc.normals(3, 3, 11, 0, 64))
    assert not np.array_equal(full, orc.normals(4, 2, 11, 0, 64))
