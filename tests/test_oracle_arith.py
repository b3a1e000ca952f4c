"""Pins for the oracle's real and complex multi-component arithmetic.

Each oracle operation must equal the greedy round-to-nearest expansion of the EXACT
result, recomputed here with Python's exact rationals (``fractions.Fraction``) and
CPython's correctly rounded ``float(Fraction)``.  The comparison is bitwise.  This pins
the number format of the paper (Sec. 1: DD 106, TD 159, QD 212 bits): the relative error
of every result is below 2^-(53C) and the components are non-overlapping.
"""
from fractions import Fraction

import numpy as np
import pytest

CS = [2, 3, 4]


def greedy(x: Fraction, C: int):
    out = []
    for _ in range(C):
        if x == 0 or abs(x) < Fraction(2) ** -1022:
            out.append(0.0)
            x = Fraction(0)
            continue
        f = float(x)
        out.append(f)
        x -= Fraction(f)
    return out


def fr(v):
    return sum((Fraction(float(c)) for c in v), Fraction(0))


def rand_mp(rng, C, canonical=True):
    """Random value with random exponent gaps between components and random zeros."""
    e0 = int(rng.integers(-60, 60))
    comps = [float(np.ldexp(rng.uniform(0.5, 1.0) * rng.choice([-1, 1]), e0))]
    e = e0
    for _ in range(1, C):
        e -= int(rng.integers(53, 53 + (200 if rng.random() < 0.2 else 12)))
        v = 0.0 if rng.random() < 0.1 else float(np.ldexp(rng.uniform(-1.0, 1.0), e))
        comps.append(v)
    if canonical:
        return greedy(fr(comps), C)
    return comps


def cases(C, n, seed):
    rng = np.random.default_rng(seed)
    for t in range(n):
        a = rand_mp(rng, C, canonical=rng.random() < 0.8)
        kind = t % 5
        if kind == 0:   # heavy cancellation: b close to -a
            bb = [-x for x in a]
            pert = rand_mp(rng, C)
            k = int(rng.integers(0, C))
            bb[k] = float(bb[k] + np.ldexp(pert[0], -int(rng.integers(40, 200))))
            b = bb
        elif kind == 1:  # exact cancellation
            b = [-x for x in a]
        elif kind == 2:  # zero operand
            b = [0.0] * C
        else:
            b = rand_mp(rng, C, canonical=rng.random() < 0.8)
        yield a, b


def bits(v):
    return [float(x).hex() for x in v]


@pytest.mark.parametrize("C", CS)
def test_add_sub_exact_rounding(orc, C):
    for a, b in cases(C, 1500, 10 + C):
        got = orc.mp_add(a, b, C)
        ref = greedy(fr(a) + fr(b), C)
        assert bits(got) == bits(ref), (a, b)
        got = orc.mp_sub(a, b, C)
        ref = greedy(fr(a) - fr(b), C)
        assert bits(got) == bits(ref), (a, b)


@pytest.mark.parametrize("C", CS)
def test_mul_exact_rounding(orc, C):
    for a, b in cases(C, 1500, 20 + C):
        got = orc.mp_mul(a, b, C)
        ref = greedy(fr(a) * fr(b), C)
        assert bits(got) == bits(ref), (a, b)


@pytest.mark.parametrize("C", CS)
def test_div_exact_rounding(orc, C):
    rng = np.random.default_rng(30 + C)
    for t in range(1000):
        a = rand_mp(rng, C, canonical=rng.random() < 0.8)
        b = rand_mp(rng, C, canonical=rng.random() < 0.8)
        if t % 7 == 0:
            a = [0.0] * C
        got = orc.mp_div(a, b, C)
        ref = greedy(fr(a) / fr(b), C)
        assert bits(got) == bits(ref), (a, b)


@pytest.mark.parametrize("C", CS)
def test_round_of_many_terms(orc, C):
    rng = np.random.default_rng(40 + C)
    for _ in range(400):
        k = int(rng.integers(1, 12))
        v = [float(np.ldexp(rng.uniform(-1, 1), int(rng.integers(-300, 300)))) for _ in range(k)]
        got = orc.mp_round(v, C)
        assert bits(got) == bits(greedy(sum(map(Fraction, v), Fraction(0)), C))


@pytest.mark.parametrize("C", CS)
def test_relative_error_and_nonoverlap(orc, C):
    """Closed-form property of greedy RN: |x - sum(c)| <= 2^-(53C) |x| and
    |c_{k+1}| <= ulp(c_k)/2."""
    rng = np.random.default_rng(50 + C)
    for a, b in cases(C, 300, 50 + C):
        x = fr(a) * fr(b)
        got = orc.mp_mul(a, b, C)
        assert abs(x - fr(got)) <= abs(x) * Fraction(2) ** (-53 * C)
        for k in range(C - 1):
            if got[k] != 0.0:
                assert abs(got[k + 1]) <= np.spacing(abs(got[k])) / 2
            else:
                assert got[k + 1] == 0.0


def _zf(z):
    return fr(z[0]), fr(z[1])


@pytest.mark.parametrize("C", CS)
def test_complex_4m_product(orc, C):
    """Eq. (4m): each real product rounded, then the sub / add rounded."""
    rng = np.random.default_rng(60 + C)
    for _ in range(300):
        a = (rand_mp(rng, C), rand_mp(rng, C))
        b = (rand_mp(rng, C), rand_mp(rng, C))
        re, im = orc.z_mul4m(a, b, C)
        ar, ai = _zf(a)
        br, bi = _zf(b)
        t1 = fr(greedy(ar * br, C))
        t2 = fr(greedy(ai * bi, C))
        t3 = fr(greedy(ai * br, C))
        t4 = fr(greedy(ar * bi, C))
        assert bits(re) == bits(greedy(t1 - t2, C))
        assert bits(im) == bits(greedy(t3 + t4, C))


@pytest.mark.parametrize("C", CS)
def test_complex_reciprocal(orc, C):
    """1/b = conj(b)/|b|^2, |b|^2 rounded once; then each quotient rounded once."""
    rng = np.random.default_rng(70 + C)
    for _ in range(200):
        b = (rand_mp(rng, C), rand_mp(rng, C))
        re, im = orc.z_recip(b, C)
        br, bi = _zf(b)
        d = fr(greedy(br * br + bi * bi, C))
        assert bits(re) == bits(greedy(br / d, C))
        assert bits(im) == bits(greedy(-bi / d, C))
        # and the result is 1/b to about 2^-(53C) relative (closed form)
        zr, zi = fr(re), fr(im)
        prod_r = zr * br - zi * bi
        prod_i = zr * bi + zi * br
        tol = Fraction(2) ** (-53 * C + 3)
        assert abs(prod_r - 1) <= tol and abs(prod_i) <= tol


@pytest.mark.parametrize("C", CS)
def test_cabs1_compare_exact(orc, C):
    rng = np.random.default_rng(80 + C)
    for t in range(300):
        a = (rand_mp(rng, C), rand_mp(rng, C))
        if t % 4 == 0:      # exact tie with swapped / negated parts
            b = ([-x for x in a[1]], a[0])
        elif t % 4 == 1:    # near tie in the last component
            b = (list(a[0]), list(a[1]))
            b[1][C - 1] = float(np.nextafter(b[1][C - 1], np.inf))
        else:
            b = (rand_mp(rng, C), rand_mp(rng, C))
        ca = abs(fr(a[0])) + abs(fr(a[1]))
        cb = abs(fr(b[0])) + abs(fr(b[1]))
        want = (ca > cb) - (ca < cb)
        assert orc.z_cabs1_cmp(a, b, C) == want
