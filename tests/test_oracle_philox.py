"""Pins of the oracle's counter-based generator (Philox4x32-10, Salmon et al.
SC'11) and of its uniform construction, against implementations that share
nothing with it: a pure-Python big-integer transcription of the published
round structure, and rocRAND's own Philox4x32-10 engine compiled for the host."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox_bigint(ctr, key, rounds=10):
    """Philox4x32 as described in Sec. 5 of the paper by Salmon et al.:
    per round, the two products M0*c0 and M1*c2 are split into hi/lo halves and
    the new block is (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key is
    advanced by the Weyl constants between rounds."""
    c = list(ctr)
    k0, k1 = key
    for r in range(rounds):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & MASK, p1 & MASK, ((p0 >> 32) ^ c[3] ^ k1) & MASK, p0 & MASK]
    return c


def _random_blocks(n, seed=1234, hi_limit=MASK):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        c = [int(v) for v in rng.integers(0, 2**32, size=4, dtype=np.uint64)]
        c[1] = c[1] % (hi_limit + 1)
        k = [int(v) for v in rng.integers(0, 2**32, size=2, dtype=np.uint64)]
        out.append((c, k))
    edge = [([0, 0, 0, 0], [0, 0]), ([MASK] * 4, [MASK, MASK]), ([1, 0, 0, 0], [0, 0]), ([0, 0, 0, 1], [1, 0])]
    return edge + out


def test_philox_matches_bigint_transcription(orc):
    for c, k in _random_blocks(2000):
        assert orc.philox4x32_10(c, k) == philox_bigint(c, k)


def _rocrand_runner():
    src = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
    rocrand_device::philox4x32_10_engine eng(seed, sub, off);
    uint4 r = eng.next4();
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""
    inc = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    cxx = shutil.which("g++")
    if not os.path.exists(inc) or cxx is None:
        return None
    d = tempfile.mkdtemp(prefix="philox_rocrand_")
    with open(os.path.join(d, "r.cpp"), "w") as f:
        f.write(src)
    exe = os.path.join(d, "r")
    r = subprocess.run([cxx, "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", os.path.join(d, "r.cpp"),
                        "-o", exe], capture_output=True, text=True)
    if r.returncode != 0:
        return None
    return exe


def test_philox_matches_rocrand_engine(orc):
    """rocRAND's engine seeded with (seed, subsequence, offset) runs the block
    counter (offset/4 lo, offset/4 hi, subsequence lo, subsequence hi) under
    key (seed lo, seed hi); its first four outputs are that block."""
    exe = _rocrand_runner()
    if exe is None:
        pytest.skip("rocRAND headers or a host C++ compiler are not available")
    blocks = _random_blocks(500, seed=99, hi_limit=(1 << 30) - 1)
    blocks = [b for b in blocks if b[0][1] < (1 << 30)]
    inp = "\n".join(" ".join(str(v) for v in c + k) for c, k in blocks) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for (c, k), line in zip(blocks, out):
        assert orc.philox4x32_10(c, k) == [int(v) for v in line.split()]


def test_uniform53_construction(orc):
    assert orc.uniform53(0, 0) == 0.0
    top = orc.uniform53(MASK, MASK)
    assert top < 1.0 and top == 1.0 - 2.0**-53
    # exact 53-bit integer scaled by 2^-53
    assert orc.uniform53(1 << 5, 0) == 2.0**-27
    assert orc.uniform53(0, 1 << 6) == 2.0**-53
    rng = np.random.default_rng(7)
    a = rng.integers(0, 2**32, size=20000, dtype=np.uint64)
    b = rng.integers(0, 2**32, size=20000, dtype=np.uint64)
    u = np.array([orc.uniform53(int(x), int(y)) for x, y in zip(a, b)])
    expect = ((a >> 5).astype(np.float64) * 2.0**26 + (b >> 6).astype(np.float64)) * 2.0**-53
    assert np.array_equal(u, expect)


def test_philox_uniform_moments(orc):
    """Uniforms drawn through the generator: mean 1/2, variance 1/12, and a
    chi-square over 64 bins."""
    n = 40000
    u = np.empty(n)
    for i in range(n):
        w = orc.philox4x32_10([i, 0, 3, 2], [0, 0])
        u[i] = orc.uniform53(w[0], w[1])
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 5 * np.sqrt(1 / 180 / n)
    h, _ = np.histogram(u, bins=64, range=(0, 1))
    e = n / 64
    chi2 = ((h - e) ** 2 / e).sum()
    # 63 dof: mean 63, sd ~11.2; 5 sigma bound
    assert chi2 < 63 + 5 * np.sqrt(2 * 63)
