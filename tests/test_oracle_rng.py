"""Pins for the oracle's random-number layer: Philox4x32-10, the 52-bit
uniform and the series logarithm behind the exponential waiting time
tau = -log(r1)/lambda of Appendix A."""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    return rows


def test_philox_published_known_answers(orc):
    rows = _kat_rows()
    assert len(rows) == 3
    for r in rows:
        ctr, key, want = r[0:4], r[4:6], r[6:10]
        assert list(orc.philox(key, ctr)) == want


_ROCRAND_PROBE = r"""
#include <cstdio>
#include <cstdlib>
#include <rocrand/rocrand_philox4x32_10.h>
// Raw Philox4x32-10 blocks from rocRAND's engine: key = seed, counter word
// pair (0,1) = offset/4 and pair (2,3) = subsequence.
int main(int argc, char** argv) {
  for (int a = 1; a + 4 < argc; a += 5) {
    unsigned long long seed = strtoull(argv[a], 0, 0);
    unsigned long long c01 = strtoull(argv[a + 1], 0, 0) | (strtoull(argv[a + 2], 0, 0) << 32);
    unsigned long long c23 = strtoull(argv[a + 3], 0, 0) | (strtoull(argv[a + 4], 0, 0) << 32);
    rocrand_device::philox4x32_10_engine eng(seed, c23, 0);
    eng.discard(c01 * 4ull);
    unsigned w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
    printf("%08x %08x %08x %08x\n", w0, w1, w2, w3);
  }
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available to build the rocRAND probe")
def test_philox_matches_rocrand(orc):
    """Independent implementation: rocRAND's philox4x32_10 engine (host side)."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    rng = np.random.default_rng(7)
    cases = []
    for _ in range(40):
        seed = int(rng.integers(0, 2**63))
        c0, c2, c3 = (int(x) for x in rng.integers(0, 2**32, 3))
        c1 = int(rng.integers(0, 2**29))  # keeps 4*(c0 + c1*2^32) inside 64 bits
        cases.append((seed, c0, c1, c2, c3))
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.cpp")
        exe = os.path.join(d, "probe")
        with open(src, "w") as f:
            f.write(_ROCRAND_PROBE)
        subprocess.run([hipcc, "-O1", "-x", "c++", src, "-o", exe,
                        "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"],
                       check=True, capture_output=True)
        args = [str(x) for c in cases for x in c]
        out = subprocess.run([exe] + args, check=True, capture_output=True, text=True).stdout
    got = [[int(x, 16) for x in line.split()] for line in out.strip().splitlines()]
    assert len(got) == len(cases)
    for (seed, c0, c1, c2, c3), want in zip(cases, got):
        key = [seed & 0xFFFFFFFF, seed >> 32]
        assert list(orc.philox(key, [c0, c1, c2, c3])) == want


def test_uniform_open_interval_and_resolution(orc):
    lo = orc.uniform(0, 0)
    hi = orc.uniform(0xFFFFFFFF, 0xFFFFFFFF)
    assert 0.0 < lo < 1e-15 and lo == 2.0 ** -53
    assert hi < 1.0 and 1.0 - hi == 2.0 ** -53
    # the low 12 bits of the second word never matter; bit 12 does
    assert orc.uniform(5, 0xFFF) == orc.uniform(5, 0)
    assert orc.uniform(5, 0x1000) - orc.uniform(5, 0) == 2.0 ** -52


def test_uniform_from_philox_is_uniform(orc):
    vals = []
    for i in range(4000):
        w = orc.philox([123, 0], [i, 7, 3, 0])
        vals += [orc.uniform(w[0], w[1]), orc.uniform(w[2], w[3])]
    vals = np.array(vals)
    assert stats.kstest(vals, "uniform").pvalue > 1e-4
    hist = np.histogram(vals, bins=20, range=(0, 1))[0]
    assert stats.chisquare(hist).pvalue > 1e-4


def _ulp_diff(a, b):
    ia = np.frombuffer(np.float64(a).tobytes(), np.int64)[0]
    ib = np.frombuffer(np.float64(b).tobytes(), np.int64)[0]
    return abs(int(ia) - int(ib))


def test_plog_special_values(orc):
    assert orc.plog(1.0) == 0.0
    assert orc.plog(0.5) == -math.log(2.0)
    assert orc.plog(0.25) == -2 * math.log(2.0)
    assert orc.plog(2.0 ** -53) == -53 * math.log(2.0)


def test_plog_against_libm_and_mpmath(orc):
    import mpmath
    mpmath.mp.prec = 120
    rng = np.random.default_rng(11)
    xs = np.concatenate([rng.random(20000), 1.0 - rng.random(2000) * 1e-6,
                         np.exp(-rng.random(2000) * 36), rng.random(2000) * 1e-12])
    xs = xs[(xs > 2.0 ** -53) & (xs <= 1.0)]
    worst = 0
    for x in xs:
        worst = max(worst, _ulp_diff(orc.plog(float(x)), math.log(float(x))))
    assert worst <= 2, worst
    # relative error against a 120-bit reference
    for x in xs[:500]:
        ref = mpmath.log(mpmath.mpf(float(x)))
        if ref != 0:
            assert abs((orc.plog(float(x)) - ref) / ref) < 4e-16


def test_exponential_variates_from_plog(orc):
    """-plog(U) of Philox uniforms is Exp(1): KS test and the first moments."""
    e = []
    for i in range(20000):
        w = orc.philox([99, 1], [i, 0, 0, 0])
        e.append(-orc.plog(orc.uniform(w[0], w[1])))
    e = np.array(e)
    assert stats.kstest(e, "expon").pvalue > 1e-4
    assert abs(e.mean() - 1.0) < 5 * 1 / math.sqrt(len(e))
