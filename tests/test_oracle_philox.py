"""Pin the oracle's Philox4x32-10 against a third-party implementation.

rocRAND ships a host-callable Philox4x32-10 engine (SC'11 generator).  Its
engine state after ``rocrand_init(seed, subsequence, offset)`` with offset a
multiple of 4 is key = (seed lo, seed hi), counter = (offset/4 lo, offset/4 hi,
subsequence lo, subsequence hi); ``rocrand()`` then returns the four words of
that block in order.  The probe below is compiled for the host only; it runs
no GPU code.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

PROBE = r"""
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
int main() {
  unsigned long long seed, sub, off;
  while (scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, sub, off, &st);
    unsigned a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
    printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
"""


def _cases():
    rng = np.random.default_rng(20170503)
    cases = [(0, 0, 0), (2**64 - 1, 2**64 - 1, 4 * (2**62 - 1)), (1, 0, 0), (0, 1, 0), (0, 0, 4)]
    for _ in range(200):
        seed = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        sub = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        off = 4 * int(rng.integers(0, 2**62))
        cases.append((seed, sub, off))
    return cases


@pytest.fixture(scope="module")
def rocrand_blocks(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("hipcc or rocRAND headers not available")
    d = tmp_path_factory.mktemp("rocrand")
    src, exe = d / "probe.cpp", d / "probe"
    src.write_text(PROBE)
    subprocess.run([hipcc, "-O1", str(src), "-o", str(exe)], check=True, capture_output=True)
    cases = _cases()
    inp = "".join("%d %d %d\n" % c for c in cases)
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout
    rows = [tuple(int(v) for v in line.split()) for line in out.strip().splitlines()]
    assert len(rows) == len(cases)
    return list(zip(cases, rows))


def test_philox_matches_rocrand(orc, rocrand_blocks):
    m32 = 0xFFFFFFFF
    for (seed, sub, off), expect in rocrand_blocks:
        n = off // 4
        key = (seed & m32, seed >> 32)
        ctr = (n & m32, n >> 32, sub & m32, sub >> 32)
        assert orc.philox(key, ctr) == expect, (seed, sub, off)


def test_philox_is_a_bijection_sample(orc):
    # distinct counters give distinct blocks (Philox is a keyed bijection)
    seen = set()
    for c in range(4096):
        seen.add(orc.philox((7, 9), (c, 0, 0, 0)))
    assert len(seen) == 4096


def test_philox_output_bits_balanced(orc):
    # each output bit is set about half the time over many counters
    ones = np.zeros(128)
    n = 4096
    for c in range(n):
        w = orc.philox((1, 0), (c, 3, 5, 7))
        for j, v in enumerate(w):
            ones[32 * j:32 * j + 32] += [(v >> b) & 1 for b in range(32)]
    frac = ones / n
    assert np.all(np.abs(frac - 0.5) < 5 * 0.5 / np.sqrt(n))
