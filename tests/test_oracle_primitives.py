"""Pins of the oracle's building blocks against mathematics that fixes them.

Nothing here re-types the oracle's formulas: each check compares against an
independent definition (exact rational arithmetic, closed forms of the
geometric law, brute-force sorting, distribution tests).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2106_03058_amd import inputs


def _round_fraction(q: Fraction, prec: int, emin: int) -> float:
    """Round a rational to the nearest binary float with `prec` bits and
    smallest exponent emin (units 2^emin), ties to even -- by integer math."""
    if q == 0:
        return 0.0
    sign = -1.0 if q < 0 else 1.0
    q = abs(q)
    # exponent e with 2^e <= q < 2^(e+1)
    e = q.numerator.bit_length() - q.denominator.bit_length()
    if Fraction(2) ** e > q:
        e -= 1
    # spacing of representable values around q
    ulp_exp = max(e - (prec - 1), emin)
    scaled = q / Fraction(2) ** ulp_exp
    fl = scaled.numerator // scaled.denominator
    rem = scaled - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return sign * math.ldexp(float(fl), ulp_exp)


def _fp32_rne(q: Fraction) -> float:
    return _round_fraction(q, 24, -149)


def _fp64_rne(q: Fraction) -> float:
    return _round_fraction(q, 53, -1074)


@pytest.mark.parametrize("seed", range(6))
def test_exact_sum_fp32_matches_rational(orc, seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 200))
    mags = rng.uniform(-40, 10, size=k)
    vals = (rng.choice([-1.0, 1.0], size=k) * 2.0 ** mags).astype(np.float32).astype(np.float64)
    if seed % 2:  # force heavy cancellation
        vals = np.concatenate([vals, -vals[: k // 2], [1e-30, -3e-38]])
        vals = vals.astype(np.float32).astype(np.float64)
    exact = sum((Fraction(float(v)) for v in vals), Fraction(0))
    assert orc.exact_sum(vals, 32) == _fp32_rne(exact)


@pytest.mark.parametrize("seed", range(4))
def test_exact_sum_fp64_matches_rational(orc, seed):
    rng = np.random.default_rng(100 + seed)
    k = int(rng.integers(1, 300))
    vals = rng.choice([-1.0, 1.0], size=k) * 2.0 ** rng.uniform(-200, 60, size=k)
    exact = sum((Fraction(float(v)) for v in vals), Fraction(0))
    got = orc.exact_sum(vals, 64)
    assert got == _fp64_rne(exact)
    assert got == float(exact)  # CPython int/int division is correctly rounded


def test_exact_sum_ties_and_edges(orc):
    u = 2.0 ** -24
    # 1 + u/2... exact halfway cases go to the even neighbour
    assert orc.exact_sum([1.0, u], 32) == 1.0
    assert orc.exact_sum([1.0, 3 * u], 32) == 1.0 + 4 * u
    # just above halfway rounds up (sticky bit far below)
    assert orc.exact_sum([1.0, u, 2.0 ** -140], 32) == 1.0 + 2 * u
    # cancellation to an exact zero is +0
    z = orc.exact_sum([0.1, -0.1], 64)
    assert z == 0.0 and math.copysign(1.0, z) == 1.0
    # subnormal binary32 results are exact
    tiny = float(np.float32(1e-45))
    assert orc.exact_sum([tiny, tiny, tiny], 32) == float(np.float32(3 * tiny))
    # overflow past the binary32 range is +inf
    big = float(np.finfo(np.float32).max)
    assert orc.exact_sum([big, big], 32) == math.inf
    assert orc.exact_sum([], 32) == 0.0


def test_skip_half_is_exact(orc):
    # For p = 1/2 every 1 - (1-p)^K = 1 - 2^-K is exact (while the lifting
    # products stay within 53 bits), so K = floor(-log2(1-V)).
    for k in range(0, 37):
        lo = 1.0 - 2.0 ** -k
        assert orc.skip(0.5, lo) == k
        if k > 0:
            assert orc.skip(0.5, math.nextafter(lo, 0.0)) == k - 1
    assert orc.skip(0.5, 0.0) == 0


def test_skip_extremes(orc):
    for V in (0.0, 0.3, 0.999999):
        assert orc.skip(1.0, V) == 0  # every trial succeeds
    assert orc.skip(1e-12, 0.5) == 127  # no success inside the lifting range
    # small p: 1-(1-p)^K ~ K p, so the skip is about V/p
    assert abs(orc.skip(1e-3, 0.05) - 51) <= 1


@pytest.mark.parametrize("p", [0.02, 0.1, 0.35, 0.8])
def test_skip_follows_geometric_law(orc, p):
    rng = np.random.default_rng(7)
    N = 40000
    V = rng.random(N)
    K = np.array([orc.skip(p, float(v)) for v in V])
    # skips are capped at 127 (runs never exceed 64 positions): lump the tail
    kmax = min(int(np.ceil(np.log(1e-3) / np.log(1 - p))), 127)
    obs = np.bincount(np.minimum(K, kmax), minlength=kmax + 1)
    pk = p * (1 - p) ** np.arange(kmax)
    exp = np.append(pk, (1 - p) ** kmax) * N
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    from scipy.stats import chi2 as chi2d

    assert chi2 < chi2d.ppf(0.9999, kmax)


def test_philox_statistics(orc):
    key = np.array([0x1234ABCD, 0x0BADF00D], dtype=np.uint32)
    outs = np.array([orc.philox([i, 7, 3, 5], key) for i in range(4096)], dtype=np.uint32)
    bits = np.unpackbits(outs.view(np.uint8))
    assert abs(bits.mean() - 0.5) < 0.005
    # each byte value equally likely
    by = outs.view(np.uint8).ravel()
    obs = np.bincount(by, minlength=256)
    exp = by.size / 256
    from scipy.stats import chi2 as chi2d

    assert float(((obs - exp) ** 2 / exp).sum()) < chi2d.ppf(0.9999, 255)
    # avalanche: flipping one counter bit flips about half of the 128 output bits
    flips = []
    for i in range(256):
        ctr = np.array([i, 11, 22, 33], dtype=np.uint32)
        base = orc.philox(ctr, key)
        for word in range(4):
            c2 = ctr.copy()
            c2[word] ^= np.uint32(1 << (i % 32))
            diff = np.bitwise_xor(base, orc.philox(c2, key))
            flips.append(int(np.unpackbits(diff.view(np.uint8)).sum()))
    assert abs(np.mean(flips) - 64) < 2.0
    # different keys give different streams
    assert not np.array_equal(orc.philox([1, 2, 3, 4], key), orc.philox([1, 2, 3, 4], key + 1))


def _kat():
    import json
    import os

    with open(os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")) as f:
        return json.load(f)


def test_philox_known_answers(orc):
    """The published Philox4x32-10 vectors (tests/golden/philox4x32_10_kat.json):
    a wrong multiplier, Weyl increment, round count or word exchange changes
    every one of them."""
    for v in _kat()["vectors"]:
        ctr = np.array([int(h, 16) for h in v["ctr"]], dtype=np.uint32)
        key = np.array([int(h, 16) for h in v["key"]], dtype=np.uint32)
        out = [int(h, 16) for h in v["out"]]
        assert orc.philox(ctr, key).tolist() == out


def test_splitmix64_known_answer(orc):
    for v in _kat()["splitmix64"]["vectors"]:
        assert orc.splitmix64(int(v["in"], 16)) == int(v["out"], 16)


def test_splitmix_no_collisions(orc):
    hs = {orc.splitmix64(i) for i in range(20000)}
    assert len(hs) == 20000


def test_degree_sort_matches_brute_force(orc):
    g = inputs.chung_lu(3000, 12, 2.3, seed=5)
    sg = orc.degree_sort(g)
    deg = np.diff(g.row_ptr)
    assert np.array_equal(sg.deg, deg)
    for u in range(g.n):
        row = g.col[g.row_ptr[u]:g.row_ptr[u + 1]]
        ref = row[np.lexsort((row, deg[row]))]
        assert np.array_equal(sg.col[g.row_ptr[u]:g.row_ptr[u + 1]], ref)


def test_level_tables_closed_forms(orc):
    alpha, L = 0.2, 20
    w = inputs.weights_ppr(alpha, L)
    S, Y, rho, kappa = orc.level_tables(w)
    i = np.arange(L + 1)
    Yc = (1 - alpha) ** i - (1 - alpha) ** (L + 1)
    assert np.allclose(Y[:-1], Yc, rtol=1e-13, atol=0)
    assert Y[-1] == 0.0
    assert abs(S - (1 - (1 - alpha) ** (L + 1))) < 1e-15
    assert np.allclose(rho[:-1], Yc[1:] / Yc[:-1], rtol=1e-13)
    assert np.allclose(kappa, S * w / Yc, rtol=1e-13)
    assert rho[L] == 0.0
    # transition probability: all mass moves, only the last level is kept
    S, Y, rho, kappa = orc.level_tables(inputs.weights_tp(10))
    assert S == 1.0 and np.all(Y[:11] == 1.0)
    assert np.all(rho[:10] == 1.0) and np.all(kappa[:10] == 0.0) and kappa[10] == 1.0


def test_theta_is_l1_norm(orc):
    rng = np.random.default_rng(3)
    x = rng.standard_normal(10007).astype(np.float32).astype(np.float64)
    exact = math.fsum(abs(v) for v in x)
    th = orc.theta(x, 1e-7)
    assert abs(th - 1e-7 * exact) <= 1e-7 * exact * 1e-12
    xi = rng.integers(-1000, 1000, size=9000).astype(np.float64)  # exactly summable
    assert orc.theta(xi, 0.5) == 0.5 * float(np.abs(xi).sum())
    assert orc.theta(np.zeros(5), 1e-3) == 0.0
