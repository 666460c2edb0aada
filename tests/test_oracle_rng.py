"""Pins of the oracle's counter-based generator and sample transforms (CPU only)."""
import math
import os

import numpy as np
import pytest
from scipy import special, stats

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for r in rows:
        out = O.philox(r[0:4], r[4:6])
        assert [int(x) for x in out] == r[6:10]


def _py_philox(c, k):
    # independent transcription of the SC'11 round function, used on random inputs
    c, k = list(c), list(k)
    for _ in range(10):
        p0, p1 = 0xD2511F53 * c[0], 0xCD9E8D57 * c[2]
        c = [(p1 >> 32) ^ c[1] ^ k[0], p1 & 0xFFFFFFFF, (p0 >> 32) ^ c[3] ^ k[1], p0 & 0xFFFFFFFF]
        k = [(k[0] + 0x9E3779B9) & 0xFFFFFFFF, (k[1] + 0xBB67AE85) & 0xFFFFFFFF]
    return c


def test_philox_random_counters_match_second_implementation():
    rng = np.random.default_rng(11)
    for _ in range(2000):
        c = [int(x) for x in rng.integers(0, 2**32, 4, dtype=np.uint64)]
        k = [int(x) for x in rng.integers(0, 2**32, 2, dtype=np.uint64)]
        assert [int(x) for x in O.philox(c, k)] == _py_philox(c, k)


def test_u01_open_interval_and_exact():
    assert O.u01(0) == 2.0**-24
    assert O.u01(0xFFFFFFFF) == 1.0 - 2.0**-24
    for x in [1, 511, 512, 0x80000000, 0x7FFFFFFF, 0xDEADBEEF]:
        u = O.u01(x)
        assert u == ((x >> 9) + 0.5) * 2.0**-23  # exact: no rounding in binary32
        assert 0.0 < u < 1.0


def _ulp(x):
    return np.spacing(np.float32(abs(x)))


def test_ln_against_libm():
    rng = np.random.default_rng(5)
    xs = np.concatenate([
        ((np.arange(0, 2**23, 977) + 0.5) * 2.0**-23),          # the uniform grid
        rng.uniform(1e-7, 1.0, 4000), rng.uniform(1.0, 1e4, 2000),
        [2.0**-24, 1.0 - 2.0**-24, 0.5, 0.7071067, 0.70710677, 1.4142135, 1.4142136, 2.0, 1.0]])
    for x in xs.astype(np.float32):
        got = O.ln(float(x))
        ref = math.log(float(x))
        # within two units in the last place of the result (absolute 2^-25 near 1)
        assert abs(got - ref) <= max(2 * _ulp(ref), 2.0**-25), (x, got, ref)
    assert O.ln(1.0) == 0.0


def test_sincos_2pi_against_libm():
    us = np.concatenate([(np.arange(0, 2**23, 331) + 0.5) * 2.0**-23,
                         [0.0, 0.125, 0.25, 0.375, 0.5, 0.75, 0.999]]).astype(np.float32)
    for u in us:
        s, c = O.sincos_2pi(float(u))
        a = 2.0 * math.pi * float(u)
        assert abs(s - math.sin(a)) <= 3e-7 and abs(c - math.cos(a)) <= 3e-7, (u, s, c)
        assert abs(s * s + c * c - 1.0) < 1e-6
    assert O.sincos_2pi(0.0) == (0.0, 1.0)


@pytest.mark.parametrize("d", [1, 2, 3, 6, 12, 32])
def test_chi_mean_closed_form(d):
    ref = math.sqrt(2.0) * math.exp(special.gammaln((d + 1) / 2) - special.gammaln(d / 2))
    assert abs(O.chi_mean(d) - ref) < 1e-12 * ref
    assert abs(O.chi_mean(d) - stats.chi(d).mean()) < 1e-10


def test_chi_mean_special_values():
    assert abs(O.chi_mean(1) - math.sqrt(2 / math.pi)) < 1e-15
    assert abs(O.chi_mean(2) - math.sqrt(math.pi / 2)) < 1e-15
