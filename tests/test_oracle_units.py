"""Oracle building blocks pinned to things other than the oracle itself.

* Philox4x32-10: rocRAND's engine (a third-party library, run on the host).
* Uniforms: exact rational arithmetic.
* log / exp / sincos: glibc (Python's math module) within 2-3 ulp, and the
  Cody-Waite split constants against a 80-digit evaluation of ln 2 and pi/2.
* Geometry: hand-derived distances, ties and volume lookups.
* Layouts (paper Sec. 3-4): bijectivity / disjointness of every mapping and
  the AoSoA pattern the paper describes for N = 2 ("AABBCCAABBCC").
"""
import math
import os
import subprocess
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- Philox ----
@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    src = os.path.join(HERE, "pins", "rocrand_philox_ref.cpp")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    try:
        subprocess.check_call(["hipcc", "-O1", "-o", exe, src], cwd=str(tmp_path_factory.getbasetemp()),
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    except (OSError, subprocess.CalledProcessError):
        pytest.skip("hipcc/rocRAND headers unavailable")
    return exe


def test_philox_matches_rocrand(oracle_mod, rocrand_ref):
    rng = np.random.default_rng(11)
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF)]
    for _ in range(400):
        c = rng.integers(0, 2**32, 4, dtype=np.uint64)
        c[1] &= 0x3FFFFFFF  # the rocRAND offset is 4 * (c1:c0) in 64 bits
        k = rng.integers(0, 2**32, 2, dtype=np.uint64)
        cases.append(tuple(int(x) for x in (*c, *k)))
    # the counters the transport uses: (step, block, hi32(id), 0)
    for n in range(0, 40, 7):
        for j in range(5):
            cases.append((n, j, 0x80000000 | n, 0, 7, 0xDEADBEEF))
    inp = "\n".join(" ".join(str(x) for x in c) for c in cases) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for c, line in zip(cases, out):
        want = [int(x) for x in line.split()]
        got = oracle_mod.philox(c[:4], c[4:])
        assert list(got) == want, c


def test_philox_bit_balance(oracle_mod):
    """Each output bit is set about half the time over 4000 counters."""
    words = np.array([oracle_mod.philox([i, 0, 0, 0], [1, 0]) for i in range(1000)], dtype=np.uint64).ravel()
    bits = np.array([(words >> b) & 1 for b in range(32)])
    frac = bits.mean(axis=1)
    assert np.all(np.abs(frac - 0.5) < 5 * 0.5 / math.sqrt(len(words)))


# -------------------------------------------------------------- uniforms ----
def test_uniforms_exact(oracle_mod):
    rng = np.random.default_rng(5)
    rs = [0, 1, 2**31, 2**32 - 1, 511, 512] + [int(x) for x in rng.integers(0, 2**32, 2000)]
    for r in rs:
        d = oracle_mod.u01(r)
        assert Fraction(d) == (Fraction(r) + Fraction(1, 2)) / 2**32
        assert 0.0 < d < 1.0
        f = oracle_mod.u01f(r)
        assert Fraction(float(f)) == (Fraction(r >> 9) + Fraction(1, 2)) / 2**23
        assert 0.0 < f < 1.0
    assert oracle_mod.u01(0) == 2.0**-33 and oracle_mod.u01(2**32 - 1) == 1.0 - 2.0**-33
    assert float(oracle_mod.u01f(0)) == 2.0**-24 and float(oracle_mod.u01f(2**32 - 1)) == 1.0 - 2.0**-24


# ------------------------------------------------------------------ math ----
def ulp_err(got, want):
    return abs(got - want) / math.ulp(want) if want != 0 else abs(got)


def f32_ulp_err(got, want_exact):
    w = np.float32(want_exact)
    u = float(np.spacing(np.abs(w)))
    return abs(float(got) - want_exact) / u


def test_split_constants(oracle_mod):
    getcontext().prec = 80
    ln2 = Decimal(2).ln()
    # pi from Machin's formula
    def atan_inv(x):
        x = Decimal(x)
        s, t, n, sign = Decimal(0), 1 / x, 1, 1
        while t / n > Decimal(10) ** -78:
            s += sign * t / n
            t /= x * x
            n += 2
            sign = -sign
        return s
    pio2 = (16 * atan_inv(5) - 4 * atan_inv(239)) / 2
    d, f = oracle_mod.constants()
    ln2_hi, ln2_lo, pio2_hi, pio2_lo = (Fraction(float(x)) for x in d[:4])
    # HI parts: rounded to 42 (ln 2) and 33 (pi/2) significant bits; LO the nearest double of the rest
    assert ln2_hi.denominator <= 2**42 and abs(Fraction(ln2) - ln2_hi) < Fraction(1, 2**42)
    assert abs(Fraction(ln2) - ln2_hi - ln2_lo) < Fraction(1, 2**96)
    assert pio2_hi.denominator <= 2**32 and abs(Fraction(pio2) - pio2_hi) < Fraction(1, 2**32)
    assert abs(Fraction(pio2) - pio2_hi - pio2_lo) < Fraction(1, 2**85)
    lf_hi, lf_lo, pf_hi, pf_lo = (Fraction(float(x)) for x in f[:4])
    assert lf_hi.denominator <= 2**16 and abs(Fraction(ln2) - lf_hi - lf_lo) < Fraction(1, 2**40)
    assert pf_hi.denominator <= 2**15 and abs(Fraction(pio2) - pf_hi - pf_lo) < Fraction(1, 2**40)
    assert float(d[7]) == math.pi and float(f[7]) == float(np.float32(math.pi))


def test_log_vs_glibc(oracle_mod):
    rng = np.random.default_rng(1)
    xs = list(2.0 ** rng.uniform(-34, 17, 20000)) + [1.0, 2.0, 0.5, math.sqrt(0.5), math.sqrt(2.0), 1e5, 2.0**-33]
    xs += [oracle_mod.u01(int(r)) for r in rng.integers(0, 2**32, 5000)]
    # f = (m-1)/(m+1) carries two roundings, so near x = 1 the result can be 3 ulp off
    errs = np.array([ulp_err(oracle_mod.log(x), math.log(x)) for x in xs if x != 1.0])
    assert errs.max() <= 3.0 and np.mean(errs <= 1.0) > 0.99
    assert oracle_mod.log(1.0) == 0.0


def test_exp_vs_glibc(oracle_mod):
    rng = np.random.default_rng(2)
    xs = list(rng.uniform(-30, 12, 20000)) + [0.0, 1.0, -1.0, math.log(2), 11.5129]
    worst = max(ulp_err(oracle_mod.exp(x), math.exp(x)) for x in xs)
    assert worst <= 2.0
    assert oracle_mod.exp(0.0) == 1.0


def test_sincos_vs_glibc(oracle_mod):
    rng = np.random.default_rng(3)
    xs = list(rng.uniform(0, 2 * math.pi, 20000)) + [0.0, math.pi / 2, math.pi, 1.5 * math.pi, 2 * math.pi, 1e-9]
    # bound: 2 ulp of the result plus the reduction error q * |pi/2 - PIO2_HI - PIO2_LO| < 4 * 2^-85
    red = 4 * 2.0**-85
    for x in xs:
        s, c = oracle_mod.sincos(x)
        assert abs(s - math.sin(x)) <= 2 * math.ulp(math.sin(x)) + red
        assert abs(c - math.cos(x)) <= 2 * math.ulp(math.cos(x)) + red
    assert oracle_mod.sincos(0.0) == (0.0, 1.0)


def test_float_math_vs_glibc(oracle_mod):
    rng = np.random.default_rng(4)
    for r in rng.integers(0, 2**32, 4000):
        u = oracle_mod.u01f(int(r))
        assert f32_ulp_err(oracle_mod.logf(u), math.log(float(u))) <= 3.0  # as in binary64, near 1
    for x in rng.uniform(1.0, 1e5, 3000).astype(np.float32):
        assert f32_ulp_err(oracle_mod.logf(x), math.log(float(x))) <= 3.0
    for x in rng.uniform(0.0, 11.6, 4000).astype(np.float32):
        assert f32_ulp_err(oracle_mod.expf(x), math.exp(float(x))) <= 2.0
    for x in rng.uniform(0.0, 2 * math.pi, 4000).astype(np.float32):
        s, c = oracle_mod.sincosf(x)
        # absolute bound 2 ulp of 1 near the zeros of sin / cos
        assert abs(float(s) - math.sin(float(x))) <= 2 * float(np.spacing(np.float32(max(abs(math.sin(float(x))), 0.5))))
        assert abs(float(c) - math.cos(float(x))) <= 2 * float(np.spacing(np.float32(max(abs(math.cos(float(x))), 0.5))))
    s, c = oracle_mod.sincosf(0.0)
    assert float(s) == 0.0 and float(c) == 1.0


def test_twice_electron_mass_is_pair_threshold():
    assert 2.0 * 0.511 == 1.022
    assert np.float32(2.0) * np.float32(0.511) == np.float32(1.022)


# -------------------------------------------------------------- geometry ----
def test_locate(oracle_mod):
    assert oracle_mod.locate([0, 0, 0]) == (0, 0)
    assert oracle_mod.locate([0, 0, 2.2999]) == (0, 0)
    assert oracle_mod.locate([0, 0, 2.3]) == (0, 1)
    assert oracle_mod.locate([0, 0, 7.9999]) == (0, 1)
    assert oracle_mod.locate([0, 0, 8.0]) == (0, 2)
    assert oracle_mod.locate([200, -200, 399.9]) == (0, 99)
    assert oracle_mod.locate([0, 0, 400.0])[0] != 0
    assert oracle_mod.locate([0, 0, -1e-12])[0] != 0
    assert oracle_mod.locate([200.0001, 0, 1])[0] != 0


def test_distance_cases(oracle_mod):
    # along +z from the front face of absorber 0: 2.3 to its back plane
    assert oracle_mod.distance([0, 0, 0], [0, 0, 1], 0) == (2.3, 2)
    # gap 1 backwards to its front plane at 2.3
    s, a = oracle_mod.distance([0, 0, 5.0], [0, 0, -1], 1)
    assert a == 2 and s == (2.3 - 5.0) / -1.0
    # transverse: x plane at 200 first
    s, a = oracle_mod.distance([199.0, 0, 1.0], [1.0, 0, 0], 0)
    assert (s, a) == (1.0, 0)
    # ties resolved z, then x, then y
    d = [1 / math.sqrt(3)] * 3
    s, a = oracle_mod.distance([198.0, 198.0, 6.0], d, 1)  # gap 1 ends at z = 8
    assert a == 2 and s == 2.0 / d[0]
    s, a = oracle_mod.distance([198.0, 198.0, 0.0], [math.sqrt(0.5), math.sqrt(0.5), 0.0], 0)
    assert a == 0
    # a point beyond its plane gives a zero-length step, never a negative one
    s, a = oracle_mod.distance([0, 0, 2.3000000001], [0, 0, 1], 0)
    assert s == 0.0 and a == 2
    assert math.copysign(1.0, s) == 1.0


# --------------------------------------------------------------- layouts ----
LEAF_SIZES = {0: [8] * 10 + [4] * 4, 1: [8, 8, 8, 4, 4, 4, 4, 4, 8, 8, 4, 4, 4, 4]}


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("mapping,lanes", [(0, 1), (1, 1), (2, 2), (2, 8), (2, 64), (2, 256)])
def test_mapping_is_a_disjoint_cover(oracle_mod, prec, mapping, lanes):
    C = 512
    nbytes = oracle_mod.buffer_bytes(mapping, lanes, prec, C)
    owner = np.full(nbytes, -1, dtype=np.int64)
    for slot in range(C):
        for leaf in range(14):
            a = oracle_mod.leaf_addr(mapping, lanes, prec, C, slot, leaf)
            sz = oracle_mod.leaf_size(prec, leaf)
            assert sz == LEAF_SIZES[prec][leaf]
            assert a % sz == 0, "natural alignment"
            assert np.all(owner[a:a + sz] == -1), "overlap"
            owner[a:a + sz] = slot * 14 + leaf
    used = int((owner >= 0).sum())
    assert used == C * sum(LEAF_SIZES[prec])
    if mapping == 0:
        assert nbytes == C * (80 if prec else 96)
        # the mixed AoS record carries 4 bytes of padding after numIALeft
        assert nbytes - used == (C * 4 if prec else 0)
    if mapping == 2:
        assert nbytes == used


def test_aosoa2_pattern(oracle_mod):
    """Paper Sec. 4 footnote: fields (A,B,C) with n = 2 are laid out AABBCCAABBCC."""
    C, prec = 8, 0
    seq = []
    for slot in range(C):
        for leaf in range(14):
            seq.append((oracle_mod.leaf_addr(2, 2, prec, C, slot, leaf), leaf, slot))
    seq.sort()
    leaves = [leaf for _, leaf, _ in seq]
    assert leaves[:4] == [0, 0, 1, 1]
    assert leaves[:28] == [x for leaf in range(14) for x in (leaf, leaf)]
    assert [s for _, _, s in seq[:4]] == [0, 1, 0, 1]


def test_soa_arrays_start_on_256_bytes(oracle_mod):
    for C in (1, 3, 1000, 4096):
        for prec in (0, 1):
            for leaf in range(14):
                assert oracle_mod.leaf_addr(1, 1, prec, C, 0, leaf) % 256 == 0
