"""Pins of the oracle's Philox generator (Salmon et al., SC'11).

The oracle's 4x32 variant (the one every draw of the simulation uses) is
checked against the published known-answer vectors of Philox4x32-10
(tests/golden/philox4x32_10_kat.txt); its 4x64 variant, built from the same
round structure, against numpy's independent Philox-4x64-10; the Weyl
constants against their closed forms; the output against avalanche and
uniformity properties.
"""
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "philox4x32_10_kat.txt")


def philox4x32_kat():
    """(counter, key, output) rows of the published Philox4x32-10 vectors"""
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((tuple(w[0:4]), tuple(w[4:6]), tuple(w[6:10])))
    return rows


def test_philox4x32_known_answers():
    rows = philox4x32_kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert tuple(int(x) for x in oracle.philox4x32(ctr, key)) == want, (ctr, key)


@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (0, 0, 0, 0)),
    ((1, 2), (0, 0, 0, 0)),
    ((0xDEADBEEFCAFEF00D, 0x0123456789ABCDEF), (5, 7, 11, 13)),
    ((2**64 - 1, 2**64 - 1), (2**64 - 3, 2**64 - 1, 2**64 - 1, 2**64 - 1)),
])
def test_philox4x64_matches_numpy(key, ctr):
    # numpy increments its 256-bit counter before each block: the block for
    # counter c+1 is the first one it returns.
    bg = np.random.Philox(key=np.array(key, np.uint64), counter=np.array(ctr, np.uint64))
    got_np = bg.random_raw(8)
    c = list(ctr)
    for blk in range(2):
        # 256-bit little-endian increment
        for w in range(4):
            c[w] = (c[w] + 1) % 2**64
            if c[w] != 0:
                break
        mine = oracle.philox4x64(c, key)
        assert [int(x) for x in mine] == [int(x) for x in got_np[4 * blk:4 * blk + 4]]


def test_weyl_constants_closed_form():
    # the key schedule adds the golden-ratio and sqrt(3)-1 fractions; both
    # widths must use the same constants truncated to the word size
    getcontext().prec = 60
    phi_frac = (Decimal(5).sqrt() - 1) / 2
    s3_frac = Decimal(3).sqrt() - 1
    assert int(phi_frac * 2**32) == 0x9E3779B9
    assert int(s3_frac * 2**32) == 0xBB67AE85
    assert int(phi_frac * 2**64) == 0x9E3779B97F4A7C15
    assert int(s3_frac * 2**64) == 0xBB67AE8584CAA73B


def test_philox4x32_key_schedule_matters():
    # with zero multipliers' inputs the output is determined by the key
    # schedule alone: counter 0, key 0 must not map to 0, and distinct keys
    # give distinct outputs
    a = oracle.philox4x32((0, 0, 0, 0), (0, 0))
    b = oracle.philox4x32((0, 0, 0, 0), (1, 0))
    assert any(int(x) for x in a)
    assert list(a) != list(b)


def test_philox4x32_avalanche():
    rng = np.random.default_rng(0)
    flips = []
    for _ in range(200):
        ctr = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        key = rng.integers(0, 2**32, size=2, dtype=np.uint64)
        base = oracle.philox4x32(ctr, key)
        w = int(rng.integers(0, 4))
        bit = int(rng.integers(0, 32))
        c2 = ctr.copy()
        c2[w] ^= np.uint64(1 << bit)
        out = oracle.philox4x32(c2, key)
        diff = sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(base, out))
        flips.append(diff)
    # 128 output bits: each should flip with probability 1/2
    assert abs(np.mean(flips) - 64.0) < 2.0


def test_philox4x32_uniform_12way():
    # the neighbour choice floor(r * 12 / 2^32) must be uniform over 12
    n = 24000
    counts = np.zeros(12, int)
    for e in range(n // 4):
        out = oracle.philox4x32((e, 17, 0, 0), (1, 0))
        for r in out:
            counts[(int(r) * 12) >> 32] += 1
    expected = n / 12
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    # 11 degrees of freedom; p = 1e-4 critical value ~ 37.4
    assert chi2 < 37.4, counts


def test_stage_order_is_a_permutation_and_varies():
    seen = set()
    for e in range(64):
        o = oracle.stage_order(12345, e)
        assert sorted(o) == list(range(16))
        seen.add(tuple(o))
    assert len(seen) > 60
    # first stage uniform over the 16 colours (chi-square, 15 dof)
    firsts = np.zeros(16, int)
    for e in range(3200):
        firsts[oracle.stage_order(99, e)[0]] += 1
    chi2 = float(((firsts - 200.0) ** 2 / 200.0).sum())
    assert chi2 < 44.3  # p = 1e-4 critical value for 15 dof
