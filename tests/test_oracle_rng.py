"""Pins of the oracle's random-number contract.

Philox4x32-10 is checked against (a) the Random123 known-answer vectors and
(b) PyTorch's independent header-only implementation (ATen PhiloxRNGEngine.h),
whose engine(seed, subsequence, offset) uses key = seed and counter =
(offset, subsequence), the layout the oracle uses with subsequence = history and
offset = block.  The uniform conversion is checked for range, resolution and the
word-pair selection of even and odd draws.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    for ctr, key, out in _kat():
        assert O.philox(ctr, key) == out


TORCH_PROG = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
    unsigned long long seed = strtoull(argv[1], 0, 10);
    unsigned long long sub = strtoull(argv[2], 0, 10);
    unsigned long long off = strtoull(argv[3], 0, 10);
    at::philox_engine e(seed, sub, off);
    for (int i = 0; i < 4; ++i) printf("%u ", e());
    printf("\n");
    return 0;
}
"""


@pytest.fixture(scope="module")
def torch_philox_exe():
    try:
        import torch
    except Exception:
        pytest.skip("torch not importable")
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if not os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")):
        pytest.skip("torch headers not shipped")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "p.cpp")
    exe = os.path.join(d, "p")
    with open(src, "w") as f:
        f.write(TORCH_PROG)
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-I", inc, src, "-o", exe], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("could not compile against torch headers: " + r.stderr[-500:])
    return exe


def test_philox_matches_torch_engine(torch_philox_exe):
    cases = [(4096, 0, 0), (4096, 1, 0), (4096, 0, 1), (4096, 123456789, 7), (2**63 + 12345, 2**40 + 3, 2**33 + 5),
             (0, 0, 0), (1, 2**64 - 1, 2**64 - 2)]
    for seed, sub, off in cases:
        out = subprocess.run([torch_philox_exe, str(seed), str(sub), str(off)], capture_output=True, text=True,
                             check=True).stdout.split()
        ref = [int(x) for x in out]
        ctr = [off & 0xFFFFFFFF, off >> 32, sub & 0xFFFFFFFF, sub >> 32]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        assert O.philox(ctr, key) == ref, (seed, sub, off)


def test_uniform_word_selection_and_range(torch_philox_exe):
    seed, h = 4096, 987654321
    for k in range(8):
        block = k >> 1
        out = subprocess.run([torch_philox_exe, str(seed), str(h), str(block)], capture_output=True, text=True,
                             check=True).stdout.split()
        w = [int(x) for x in out]
        a, b = (w[0], w[1]) if k % 2 == 0 else (w[2], w[3])
        expect = ((a >> 5) * 2.0 ** 26 + (b >> 6)) / 2.0 ** 53
        assert O.uniform(seed, h, k) == expect


def test_uniform_distribution():
    u = np.array([O.uniform(4096, h, k) for h in range(2000) for k in range(10)])
    assert u.min() >= 0.0 and u.max() < 1.0
    hist, _ = np.histogram(u, bins=20, range=(0, 1))
    exp = len(u) / 20
    chi2 = ((hist - exp) ** 2 / exp).sum()
    from scipy.stats import chi2 as C2
    assert C2.sf(chi2, 19) > 1e-3
    # resolution: 53-bit values are multiples of 2^-53
    assert np.all(np.floor(u * 2.0 ** 53) == u * 2.0 ** 53)
