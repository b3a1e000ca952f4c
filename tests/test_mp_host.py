"""The library's multi-component arithmetic (csrc/mp.hpp is __host__ __device__), compiled
for the host and checked on the CPU against exact rational arithmetic.  This catches
accuracy bugs in the device arithmetic without a GPU; the GPU tests then check the
kernels themselves against the oracle.

Bounds (closed forms for the algorithms used, u_C = 2^-(53C)):
  * renorm: exact (the value is unchanged) and non-overlapping (|c_{k+1}| <= ulp(c_k));
  * mul, recip: relative error <= 8 u_C;
  * add: error <= 8 u_C (|a| + |b|);
  * a - l*u (4M, one rounding per part): error <= 16 u_C (|a| + |l||u|) per part;
  * dot products: error <= 4 (n + 2) u_C sum |a_i b_i|.
"""
import ctypes as ct
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SHIM = os.path.join(ROOT, "tests", "host", "mp_host_shim.cpp")
OUT = os.path.join(ROOT, "_build", "mph.so")


@pytest.fixture(scope="module")
def H():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    subprocess.check_call([hipcc, "-x", "hip", "--cuda-host-only", "-O2", "-ffp-contract=off",
                           "-fPIC", "-shared", "-o", OUT, SHIM,
                           "-Wno-unused-command-line-argument"])
    return ct.CDLL(OUT)


def arr(v):
    return (ct.c_double * len(v))(*[float(x) for x in v])


def fr(v):
    return sum((Fraction(float(x)) for x in v), Fraction(0))


def rand_mp(rng, C):
    e0 = int(rng.integers(-30, 30))
    v = [float(np.ldexp(rng.uniform(0.5, 1) * rng.choice([-1, 1]), e0))]
    for k in range(1, C):
        v.append(float(np.ldexp(rng.uniform(-0.5, 0.5), e0 - 53 * k - int(rng.integers(0, 3)))))
    return v


CS = [2, 3, 4]


@pytest.mark.parametrize("C", CS)
def test_renorm_exact_and_nonoverlapping(H, C):
    rng = np.random.default_rng(C)
    o = arr([0] * C)
    for t in range(3000):
        a = rng.uniform(-1, 1)
        if t % 3 == 0:   # levels cancelling each other
            lev = [a, -a * (1 + rng.uniform(-1, 1) * 2.0 ** -int(rng.integers(1, 60)))]
            lev += [rng.uniform(-1, 1) * 2.0 ** -(40 * k) for k in range(1, C - 1)]
        elif t % 3 == 1:  # overlapping levels of similar size
            lev = [rng.uniform(-1, 1) * 2.0 ** -int(rng.integers(0, 8)) for _ in range(C)]
        else:
            lev = rand_mp(rng, C)
        lev = lev[:C]
        H.mph_renorm(C, arr(lev), o)
        out = list(o)
        assert fr(out) == fr(lev)
        for k in range(C - 1):
            if out[k] == 0:
                assert out[k + 1] == 0
            else:
                assert abs(out[k + 1]) <= np.spacing(abs(out[k]))


@pytest.mark.parametrize("C", CS)
def test_mul_add_recip_accuracy(H, C):
    rng = np.random.default_rng(10 + C)
    u = Fraction(2) ** (-53 * C)
    o = arr([0] * C)
    for _ in range(1500):
        a, b = rand_mp(rng, C), rand_mp(rng, C)
        H.mph_mul(C, arr(a), arr(b), o)
        ex = fr(a) * fr(b)
        assert abs(fr(list(o)) - ex) <= 8 * u * abs(ex)
        H.mph_add(C, arr(a), arr(b), o)
        ex = fr(a) + fr(b)
        assert abs(fr(list(o)) - ex) <= 8 * u * (abs(fr(a)) + abs(fr(b)))
        H.mph_recip(C, arr(a), o)
        assert abs(fr(list(o)) * fr(a) - 1) <= 8 * u


@pytest.mark.parametrize("C", CS)
def test_complex_ops_accuracy(H, C):
    rng = np.random.default_rng(20 + C)
    u = Fraction(2) ** (-53 * C)
    o = arr([0] * (2 * C))
    for t in range(800):
        a = rand_mp(rng, C) + rand_mp(rng, C)
        l_ = rand_mp(rng, C) + rand_mp(rng, C)
        uu = rand_mp(rng, C) + rand_mp(rng, C)
        if t % 4 == 0:  # a close to l*u: cancellation in the update
            pr = fr(l_[:C]) * fr(uu[:C]) - fr(l_[C:]) * fr(uu[C:])
            a[:C] = [float(pr)] + [0.0] * (C - 1)
        ar, ai = fr(a[:C]), fr(a[C:])
        lr, li = fr(l_[:C]), fr(l_[C:])
        ur, ui = fr(uu[:C]), fr(uu[C:])
        H.mph_zfms(C, arr(a), arr(l_), arr(uu), o)
        got = list(o)
        mag = abs(ar) + abs(ai) + (abs(lr) + abs(li)) * (abs(ur) + abs(ui))
        assert abs(fr(got[:C]) - (ar - (lr * ur - li * ui))) <= 16 * u * mag
        assert abs(fr(got[C:]) - (ai - (lr * ui + li * ur))) <= 16 * u * mag
        H.mph_zmul(C, arr(l_), arr(uu), o)
        got = list(o)
        mag = (abs(lr) + abs(li)) * (abs(ur) + abs(ui))
        assert abs(fr(got[:C]) - (lr * ur - li * ui)) <= 16 * u * mag
        assert abs(fr(got[C:]) - (lr * ui + li * ur)) <= 16 * u * mag
        H.mph_zrecip(C, arr(uu), o)
        got = list(o)
        zr, zi = fr(got[:C]), fr(got[C:])
        assert abs(zr * ur - zi * ui - 1) <= 16 * u and abs(zr * ui + zi * ur) <= 16 * u


@pytest.mark.parametrize("C", CS)
def test_dot_accuracy(H, C):
    rng = np.random.default_rng(30 + C)
    u = Fraction(2) ** (-53 * C)
    for n in (1, 7, 64, 128):
        a = [rand_mp(rng, C) for _ in range(n)]
        b = [rand_mp(rng, C) for _ in range(n)]
        o = arr([0] * C)
        H.mph_dot(C, n, arr(sum(a, [])), arr(sum(b, [])), o)
        ex = sum((fr(x) * fr(y) for x, y in zip(a, b)), Fraction(0))
        S = sum((abs(fr(x) * fr(y)) for x, y in zip(a, b)), Fraction(0))
        assert abs(fr(list(o)) - ex) <= 4 * (n + 2) * u * S


@pytest.mark.parametrize("C", CS)
def test_tidy_is_exact(H, C):
    """Re-levelling leaves the value of an accumulator unchanged, bit for bit in sum."""
    rng = np.random.default_rng(40 + C)
    for _ in range(500):
        e = int(rng.integers(-20, 20))
        lv = [float(np.ldexp(rng.uniform(-1, 1), e - int(rng.integers(0, 40)) * k))
              for k in range(C)]
        o = arr([0] * C)
        H.mph_tidy(C, arr(lv), o)
        assert fr(list(o)) == fr(lv)


@pytest.mark.parametrize("C", CS)
def test_long_same_sign_dot_with_tidy(H, C):
    """A long sum of same-sign products (the paper's uniform [0, 1] matrix-product
    workload, n = 2048) stays within 4 (n + 2) u sum |a_i b_i| when the accumulator is
    re-levelled every 16 terms, as the long products of the library do."""
    rng = np.random.default_rng(50 + C)
    u = Fraction(2) ** (-53 * C)
    n = 2048

    def vec():
        out = []
        for _ in range(n):
            x = Fraction(float(rng.uniform(0, 1)))
            t = float(x)
            for k in range(1, C):
                t = t * 2.0 ** -53 * float(rng.uniform(-1, 1))
                x += Fraction(t)
            comps = []
            for k in range(C):
                f = float(x)
                comps.append(f)
                x -= Fraction(f)
            out.append(comps)
        return out

    a, b = vec(), vec()
    ex = sum((fr(x) * fr(y) for x, y in zip(a, b)), Fraction(0))
    o = arr([0] * C)
    H.mph_dot_tidy(C, n, 16, arr(sum(a, [])), arr(sum(b, [])), o)
    assert abs(fr(list(o)) - ex) <= 4 * (n + 2) * u * ex


@pytest.mark.parametrize("C", CS)
def test_complex_reciprocal_extreme_magnitudes(H, C):
    """1/b for pivots of magnitude 2^+-230 .. 2^+-800 (about 1e+-70 .. 1e+-240), where
    the unscaled Re b^2 + Im b^2 overflows, underflows or has subnormal lower
    components: the result is finite and equals, bit for bit, 2^-k times the reciprocal
    of the same value at moderate magnitude, so it is exactly as accurate as there."""
    rng = np.random.default_rng(90 + C)
    o1, o2 = arr([0] * (2 * C)), arr([0] * (2 * C))
    for k in (-800, -600, -400, -230, 230, 400, 600, 800):
        for t in range(40):
            b = rand_mp(rng, C) + rand_mp(rng, C)
            H.mph_zrecip(C, arr(b), o1)
            H.mph_zrecip(C, arr([float(np.ldexp(x, k)) for x in b]), o2)
            got = list(o2)
            assert all(np.isfinite(got)), (k, t, got)
            assert [float(np.ldexp(x, -k)) for x in list(o1)] == got, (k, t)


@pytest.mark.parametrize("C", CS)
def test_complex_reciprocal_scaling_is_exact(H, C):
    """At moderate magnitudes the power-of-two scaling changes no bit: 1/(2^k b) equals
    2^-k (1/b) exactly, componentwise."""
    rng = np.random.default_rng(95 + C)
    o1, o2 = arr([0] * (2 * C)), arr([0] * (2 * C))
    for t in range(200):
        b = rand_mp(rng, C) + rand_mp(rng, C)
        k = int(rng.integers(-40, 40))
        H.mph_zrecip(C, arr(b), o1)
        H.mph_zrecip(C, arr([float(np.ldexp(x, k)) for x in b]), o2)
        assert [float(np.ldexp(x, -k)) for x in list(o1)] == list(o2)
