"""Pins of the oracle's random numbers: Philox4x32-10 against rocRAND's
independent implementation, our LN / SINCOS2PI against libm, and the
Box-Muller normals against the standard normal law (Eq. 2 asks for
zero-mean, unit-variance Gaussian z)."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_helper(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rr")
    subprocess.check_call([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950",
                           os.path.join(HERE, "helpers", "rocrand_philox.cpp"), "-o", exe],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return exe


def test_philox_matches_rocrand(orc, rocrand_helper):
    rng = np.random.default_rng(11)
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF,) * 6, (1, 2, 3, 4, 5, 6), (7, 0xFFFFFFFF, 16, 0, 3, 0)]
    cases += [tuple(int(v) for v in rng.integers(0, 2**32, size=6, dtype=np.uint64)) for _ in range(300)]
    # the counters the method uses: (walker, step, purpose, 0)
    cases += [(w, t, p, 0, 2, 0) for w in (0, 1, 999_999) for t in (0, 1, 4999) for p in (0, 1, 2, 16, 79)]
    inp = "\n".join(" ".join(str(v) for v in c) for c in cases) + "\n"
    out = subprocess.run([rocrand_helper], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for c, line in zip(cases, out):
        ref = [int(v) for v in line.split()]
        got = orc.philox(c[:4], c[4:]).tolist()
        assert got == ref, (c, got, ref)


def test_ln_against_libm(orc):
    rng = np.random.default_rng(1)
    us = np.concatenate([rng.uniform(size=20000), 2.0 ** -rng.uniform(0, 33, size=20000),
                         [0.5 / 2**32, 1.0 - 0.5 / 2**32, 0.5, 1.0, math.sqrt(0.5), 0.70710678118654746]])
    worst = 0.0
    for u in us:
        ref = math.log(u)
        got = orc.ln(u)
        if ref != 0:
            worst = max(worst, abs(got - ref) / (math.ulp(ref)))
        else:
            assert abs(got) < 1e-300
    assert worst <= 2.0, worst


def test_sincos2pi_against_libm(orc):
    rng = np.random.default_rng(2)
    us = np.concatenate([rng.uniform(size=20000), np.arange(64) / 64.0, [1 - 2**-53, 2**-40]])
    # reference in x87 extended precision, so that the rounding of 2 pi u
    # does not dominate the comparison
    two_pi = np.longdouble("6.28318530717958647692528676655900577")
    for u in us:
        s, c = orc.sincos2pi(u)
        x = two_pi * np.longdouble(u)
        assert abs(s - float(np.sin(x))) <= 2.5e-16
        assert abs(c - float(np.cos(x))) <= 2.5e-16
        assert abs(s * s + c * c - 1.0) <= 6.7e-16


def test_normals_are_standard_normal(orc):
    n = 2_000_000
    z = orc.normals(3, 0, 12345, n).ravel()
    N = z.size
    assert abs(z.mean()) < 4.0 / math.sqrt(N)
    assert abs(z.var() - 1.0) < 4.0 * math.sqrt(2.0 / N)
    assert np.max(np.abs(z)) <= math.sqrt(66 * math.log(2)) + 1e-12
    assert stats.kstest(z[:200000], "norm").pvalue > 1e-3
    # the three components of one draw are uncorrelated
    zz = z.reshape(-1, 3)
    c = np.corrcoef(zz.T)
    assert np.max(np.abs(c - np.eye(3))) < 4.0 / math.sqrt(zz.shape[0])


def test_normals_depend_on_every_counter_word(orc):
    key = np.array([5, 0], np.uint32)
    base = orc.philox([1, 2, 3, 0], key)
    for i in range(4):
        c = [1, 2, 3, 0]
        c[i] += 1
        assert not np.array_equal(orc.philox(c, key), base)
    assert not np.array_equal(orc.philox([1, 2, 3, 0], [5, 1]), base)
