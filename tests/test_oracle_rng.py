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


_ROCRAND_PROBE = r"""
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
// reads lines "c0 c1 c2 c3 k0 k1", prints Philox4x32-10(c, k) via rocRAND's engine
int main() {
  unsigned c[4], k[2];
  while (std::scanf("%u %u %u %u %u %u", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
    const unsigned long long seed = ((unsigned long long)k[1] << 32) | k[0];
    const unsigned long long subseq = ((unsigned long long)c[3] << 32) | c[2];
    const unsigned long long offset = 4ull * (((unsigned long long)c[1] << 32) | c[0]);
    rocrand_device::philox4x32_10_engine e(seed, subseq, offset);
    const uint4 r = e.next4();
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


def test_philox_matches_rocrand(tmp_path):
    # rocRAND's Philox4x32-10 as an independent implementation: its engine,
    # seeded with the key, subsequence (c2, c3) and offset 4 (c0, c1), yields
    # Philox(c, key) as its first four outputs (the upper counter words stay
    # below 2^30 so the 4x offset does not carry out of 64 bits)
    import shutil
    import subprocess
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc or rocRAND headers not available")
    src = tmp_path / "probe.cpp"
    exe = tmp_path / "probe"
    src.write_text(_ROCRAND_PROBE)
    subprocess.run([hipcc, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-O1",
                    "-o", str(exe), str(src)],
                   check=True, capture_output=True, timeout=300)
    rng = np.random.default_rng(7)
    cases = rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64)
    cases[:, 1] %= 2**30
    cases[:5, :4] = 0
    cases[5] = [0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF]
    inp = "\n".join(" ".join(str(int(v)) for v in row) for row in cases) + "\n"
    res = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True,
                         timeout=60)
    got = np.array([[int(x) for x in line.split()] for line in res.stdout.strip().splitlines()],
                   np.uint64)
    assert got.shape == (len(cases), 4)
    for row, g in zip(cases, got):
        want = O.philox(row[:4].astype(np.uint32), row[4:].astype(np.uint32))
        assert np.array_equal(want.astype(np.uint64), g), (row, want, g)
