"""CPU check of the mixed-precision error bound, on emulated arithmetic.

The mixed forms screen candidates with an estimate of the KL key whose cross
term C = sum_i x_i log c_i is formed from 16-bit operands (BF16 or FP16),
each value v split as v = hi + lo + r with hi = v rounded to 16 bits and
lo = (v - hi) rounded to 16 bits (v - hi is exact in FP64), and the three
products lo*hi, hi*lo, hi*hi accumulated in FP32 in an unspecified order.
Every ordering decision is exact only if |C~ - C| stays within the bound the
library states:

    e_rel = 3u^2 + 3u^3 + (3D + 3) 2^-23 (1.0001) (1 + u)^5
    e_abs = D (3 s (pmax + lmax) + 21 s^2) (1 + g) + 6 g D s (pmax + lmax) + 3 D 2^-126
    |C~ - C| <= e_rel / (1 - e_rel) (|C~| + e_abs) + e_abs

with u = 2^-8 (BF16) or 2^-11 (FP16) plus 2^-23 for a conversion that rounds
through FP32 first, s = 2^-133 (BF16) or 2^-24 (FP16) (half the smallest
subnormal spacing, likewise inflated), g = (3D + 3) 2^-23 (1.0001), pmax and
lmax the largest |x_i| and |log x_i| of the input.  The key estimate is
k~ = S(x) - C~ with S(x) = sum_i x_i log x_i folded in FP64, and the
receiver widens the bound by 2^-44 (|S| + |C~| + 1) for the FP64 roundings of
S, of the subtraction and of the canonical fold.

This test rounds to 16 bits by its own bit arithmetic (round to nearest even,
directly from FP64 and through FP32), forms the products exactly, sums them
in FP32 in several orders (ascending, descending, by magnitude both ways,
random, pairwise, and with truncating additions), and checks the bound
against the exact cross term and, after the FP64 steps, against the oracle's
canonical key.  It also plants a mistake (the lo parts dropped) to show that
the check can fail.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

MODES = {"bf16": (8, -133), "fp16": (11, -24)}  # significand bits, log2 of the subnormal spacing


def rne(v, p, qmin):
    """Round float64 array v to p significant bits (nearest, ties to even),
    with spacing never below 2^qmin (the subnormal range); exact in FP64."""
    v = np.asarray(v, dtype=np.float64)
    m, e = np.frexp(np.abs(v))  # |v| = m 2^e, m in [0.5, 1)
    q = np.exp2(np.maximum(e - p, qmin).astype(np.float64))
    out = np.round(np.abs(v) / q) * q  # np.round: half to even; the scaling is exact
    return np.where(v < 0, -out, np.where(v == 0, 0.0, out))


def to16(v, mode, via32):
    p, qmin = MODES[mode]
    if via32:
        v = rne(v, 24, -149)
    return rne(v, p, qmin)


def split(v, mode, via32):
    hi = to16(v, mode, via32)
    lo = to16(v - hi, mode, via32)  # v - hi is exact in FP64
    return hi, lo


def f32_sum(terms, order, rtz=False):
    """Sum FP32-exact terms in FP32 in the given order, each addition rounded
    to nearest even (or toward zero)."""
    acc = np.float32(0.0)
    for t in terms[order]:
        exact = float(acc) + float(t)  # two FP32 values add exactly in FP64
        r = np.float32(exact)
        if rtz and abs(float(r)) > abs(exact):
            r = np.nextafter(r, np.float32(0.0))
        acc = r
    return float(acc)


def f32_pairwise(terms):
    t = [np.float32(x) for x in terms]
    while len(t) > 1:
        t = [np.float32(float(t[i]) + float(t[i + 1])) if i + 1 < len(t) else t[i]
             for i in range(0, len(t), 2)]
    return float(t[0]) if t else 0.0


def exact_dot(x, l):
    """sum_i x_i l_i, correctly rounded to FP64 (x FP32-exact values): l is
    split into two 26/27-bit halves so that each partial product is exact."""
    m, e = np.frexp(l)
    lh = np.ldexp(np.trunc(np.ldexp(m, 26)), e - 26)
    ll = l - lh
    return math.fsum(np.concatenate([x * lh, x * ll]).tolist())


def fma_fold(x, l):
    s = Fraction(0)
    for a, b in zip(x.tolist(), l.tolist()):
        s = Fraction(float(Fraction(a) * Fraction(b) + s))
    return float(s)


def bound_constants(mode, D, pmax, lmax):
    p, _ = MODES[mode]
    u = 2.0 ** -p + 2.0 ** -23
    s = 2.0 ** -133 if mode == "bf16" else 2.0 ** -24
    g = (3 * D + 3) * 2.0 ** -23 * 1.0001
    e_rel = 3 * u * u + 3 * u ** 3 + g * (1 + u) ** 5
    e_abs = (D * (3 * s * (pmax + lmax) + 21 * s * s) * (1 + g) + g * 6 * D * s * (pmax + lmax)
             + 3 * D * 2.0 ** -126)
    return e_rel / (1 - e_rel) * (1 + 2.0 ** -50), e_abs


def rows(kind, n, D, seed):
    """FP32 points on the simplex: Dirichlet(1^D); rows with 30% of their
    coordinates below 2^-14 (FP16 subnormals); rows with one coordinate near 1."""
    rng = np.random.default_rng(seed)
    if kind == "dirichlet":
        return synth.dirichlet(seed, n, D - 1, np.float32)
    if kind == "tiny":
        P = rng.exponential(size=(n, D))
        k = max(1, int(0.3 * D))
        for r in range(n):
            idx = rng.choice(D, k, replace=False)
            P[r, idx] = 0.0
            P[r] /= P[r].sum()
            P[r, idx] = np.exp(rng.uniform(np.log(1e-12), np.log(2.0 ** -14), k))
        return np.maximum(P, 1e-12).astype(np.float32)
    P = np.exp(rng.uniform(np.log(1e-9), np.log(1e-5), size=(n, D)))
    big = rng.integers(0, D, n)
    P[np.arange(n), big] = 1.0 - (P.sum(axis=1) - P[np.arange(n), big])
    return P.astype(np.float32)


def orders(terms, rng):
    m = terms.size
    yield np.arange(m)
    yield np.arange(m)[::-1]
    yield np.argsort(np.abs(terms), kind="stable")
    yield np.argsort(-np.abs(terms), kind="stable")
    yield rng.permutation(m)


def check_pairs(P, mode, via32, drop_lo=False, pairs=60, seed=0):
    n, D = P.shape
    P64 = oracle.widen(P)
    L = oracle.log_table(P64)
    pmax, lmax = float(np.abs(P64).max()), float(np.abs(L).max())
    assert pmax <= 1.0
    epsq, eabs = bound_constants(mode, D, pmax, lmax)
    rng = np.random.default_rng(seed)
    worst = 0.0
    for _ in range(pairs):
        x, c = (int(v) for v in rng.choice(n, 2, replace=False))
        xh, xl = split(P64[x], mode, via32)
        lh, ll = split(L[c], mode, via32)
        if drop_lo:
            xl = np.zeros_like(xl)
            ll = np.zeros_like(ll)
        terms = np.concatenate([xl * lh, xh * ll, xh * lh])  # products of 16-bit values: exact
        assert np.array_equal(terms.astype(np.float32).astype(np.float64), terms)
        C = exact_dot(P64[x], L[c])
        S = fma_fold(P64[x], L[x])
        key = oracle.key(P64, L, x, c)
        sums = []
        for o in orders(terms, rng):
            sums.append(f32_sum(terms, o))
            sums.append(f32_sum(terms, o, rtz=True))
        sums.append(f32_pairwise(terms))
        for Ct in sums:
            bnd = epsq * (abs(Ct) + eabs) + eabs
            err = abs(Ct - C)
            worst = max(worst, (err - abs(C) * 2.0 ** -52) / bnd)
            if not drop_lo:
                assert err - abs(C) * 2.0 ** -52 <= bnd, (x, c, Ct, C, bnd)
                kt = S - Ct  # FP64 subtraction, as in the receiver
                cabs = max(kt - S, 0.0)
                eps = epsq * (cabs + eabs) + eabs + 2.0 ** -44 * (abs(S) + cabs + 1.0)
                assert abs(kt - key) <= eps, (x, c, kt, key, eps)
    return worst


@pytest.mark.parametrize("mode", ["bf16", "fp16"])
@pytest.mark.parametrize("via32", [False, True], ids=["direct", "via_fp32"])
@pytest.mark.parametrize("D", [6, 21, 32, 51, 64])
@pytest.mark.parametrize("kind", ["dirichlet", "tiny", "near1"])
def test_mixed_bound_holds(mode, via32, D, kind):
    P = rows(kind, 120, D, seed=D * 7 + len(kind))
    worst = check_pairs(P, mode, via32, seed=D)
    # the bound is not vacuous: the emulated error reaches a visible share of it
    assert worst > 0.02, worst


@pytest.mark.parametrize("mode", ["bf16", "fp16"])
def test_dropping_the_low_parts_breaks_the_bound(mode):
    # the single-product form's error is ~u|C|, far beyond the split form's bound
    P = rows("dirichlet", 120, 21, seed=5)
    assert check_pairs(P, mode, False, drop_lo=True, seed=1) > 1.0


def test_rounding_helpers():
    # against numpy's own FP16 and FP32 conversions (direct rounding from FP64)
    v = np.random.default_rng(1).standard_normal(20000) * np.exp2(np.random.default_rng(2).integers(-30, 10, 20000))
    assert np.array_equal(rne(v, 11, -24), np.float16(v).astype(np.float64))
    assert np.array_equal(rne(v, 24, -149), np.float32(v).astype(np.float64))
    # BF16 through FP32 by bit arithmetic: add 0x7FFF + lsb, clear the low half
    f = np.float32(v)
    b = f.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    assert np.array_equal(to16(v, "bf16", True), b.view(np.float32).astype(np.float64))
