"""Pins of the oracle's random-number layer: Philox and the 53-bit uniform.

Philox (Salmon et al., SC'11) is not in the paper; it is the counter-based
generator both sides draw from.  The oracle builds its 4x32 and 4x64
instances from one round macro; the 4x64 instance is checked bit-for-bit
against numpy's independent Philox4x64-10, which pins the round structure
(word permutation, xor placement, key schedule).  The 4x32 instance, the one
both sides draw from, is checked bit-for-bit against PyTorch's header-only
at::Philox4_32 engine (an independent implementation, compiled here with
g++) over 120 000+ counters and keys, including the all-ones counter and key:
that pins its multipliers 0xD2511F53 / 0xCD9E8D57 as well as the round
structure.  The Weyl constants are also derived from the golden ratio and
sqrt 3, and the output bytes are checked for uniformity.
"""
import math
import os
import shutil
import subprocess
from decimal import Decimal, getcontext

import numpy as np
import pytest

from oracle import binding as B


@pytest.mark.parametrize("seed", range(6))
def test_philox4x64_matches_numpy(seed):
    rng = np.random.default_rng(seed)
    for _ in range(20):
        ctr = [int(v) for v in rng.integers(0, 2**63, size=4, dtype=np.uint64)]
        key = [int(v) for v in rng.integers(0, 2**63, size=2, dtype=np.uint64)]
        # numpy's Philox increments the 256-bit counter before each block
        prev = list(ctr)
        prev[0] = (prev[0] - 1) % 2**64
        if ctr[0] == 0:
            prev[1] = (prev[1] - 1) % 2**64
        ref = np.random.Philox(counter=prev, key=key).random_raw(4)
        assert [int(v) for v in ref] == B.philox4x64(ctr, key)


def test_weyl_constants_are_golden_ratio_and_sqrt3():
    # Philox key schedule bumps: fractional parts of the golden ratio and sqrt(3)
    getcontext().prec = 60
    phi = (1 + Decimal(5).sqrt()) / 2
    s3 = Decimal(3).sqrt()
    assert int((phi - 1) * 2**32) == 0x9E3779B9
    assert int((s3 - 1) * 2**32) == 0xBB67AE85
    assert int((phi - 1) * 2**64) == 0x9E3779B97F4A7C15
    assert int((s3 - 1) * 2**64) == 0xBB67AE8584CAA73B


def test_philox4x32_is_a_bijection_sample_and_key_sensitive():
    outs = set()
    for c in range(2000):
        outs.add(tuple(B.philox4x32([c, 0, 0, 0], [1, 2])))
    assert len(outs) == 2000
    a = B.philox4x32([7, 8, 9, 10], [1, 2])
    b = B.philox4x32([7, 8, 9, 10], [1, 3])
    assert sum(bin(x ^ y).count("1") for x, y in zip(a, b)) > 40  # avalanche


def test_philox4x32_uniform_bytes_chi2():
    words = np.array([B.philox4x32([i, 3, 1, 0], [0, 0]) for i in range(4096)], dtype=np.uint32).ravel()
    by = words.view(np.uint8)
    counts = np.bincount(by, minlength=256)
    exp = by.size / 256
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    # 255 dof: mean 255, sd ~22.6; 5 sigma band
    assert 255 - 5 * 22.6 < chi2 < 255 + 5 * 22.6


def test_u53_range_and_resolution():
    assert B.u53(0, 0) == 0.0
    assert B.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0**-53
    assert B.u53(0, 1 << 6) == 2.0**-53  # lowest bit of the second word that counts
    assert B.u53(0, 63) == 0.0           # the low 6 bits of the second word are dropped
    assert B.u53(1 << 5, 0) == 2.0**-27
    assert B.u53(0x80000000, 0) == 0.5
    rng = np.random.default_rng(1)
    for a, b in rng.integers(0, 2**32, size=(200, 2)):
        u = B.u53(int(a), int(b))
        assert 0.0 <= u < 1.0
        assert math.ldexp(u, 53) == int(math.ldexp(u, 53))  # a multiple of 2^-53


def _torch_philox_driver(tmp_path):
    """Build the at::Philox4_32 driver with g++ against torch's headers."""
    torch = pytest.importorskip("torch")
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    hdr = os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")
    if not os.path.exists(hdr):
        pytest.skip("torch headers not installed")
    src = os.path.join(os.path.dirname(__file__), "golden", "philox_torch_driver.cpp")
    exe = str(tmp_path / "philox_torch")
    subprocess.run([gxx, "-O1", "-std=c++17", "-I", inc, src, "-o", exe], check=True, capture_output=True)
    return exe


def test_philox4x32_matches_torch_engine(tmp_path):
    exe = _torch_philox_driver(tmp_path)
    rng = np.random.default_rng(2024)
    ones = 0xFFFFFFFF
    rows = [(0, 0, 0, 0, 0, 0), (ones, ones, ones, ones, ones, ones), (ones, 0, ones, 0, 0, ones),
            (1, 2, 3, 4, 5, 6)]
    rows += [tuple(int(v) for v in r) for r in rng.integers(0, 2**32, size=(2000, 6), dtype=np.uint64)]
    # runs of consecutive counters in the layout the method uses (particle id,
    # step, stream, call) under several seeds, one wrapping past 2^32 - 1
    runs = [(0, 0, 1, 0, 0), (0x123456789ABCDEF, 7, 2, 0, 40_000), ((1 << 64) - 1, 0xFFFFFFFF, 4, 3, 2**32 - 20_000),
            (3, 100, 5, 1, 123_456_789)]
    fills = []
    for seed, c1, c2, c3, c0 in runs:
        n = 30_000
        fills.append(((seed, c0, c1, c2, c3), B.philox_fill(seed, c0, c1, c2, c3, n)))
        rows += [((c0 + i) & ones, c1, c2, c3, seed & ones, seed >> 32) for i in range(n)]
    assert len(rows) >= 120_000
    inp = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split()
    ref = np.array(out, dtype=np.uint64).astype(np.uint32).reshape(-1, 4)
    assert ref.shape[0] == len(rows)
    nrand = len(rows) - sum(f.shape[0] for _, f in fills)
    for r, want in zip(rows[:nrand], ref[:nrand]):
        assert B.philox4x32(list(r[:4]), list(r[4:])) == [int(w) for w in want], r
    # counter 0, key 0: 6627e8d5 e169c58d bc57ac4c 9b00dbd8
    assert [int(w) for w in ref[0]] == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    off = nrand
    for _, f in fills:
        assert np.array_equal(f, ref[off:off + f.shape[0]])
        off += f.shape[0]
