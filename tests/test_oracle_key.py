"""Pins of the oracle's comparator key: D(x||y) = sum_i x_i log(x_i / y_i)
(Section 2.2), summed over every stored coordinate."""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth


def _table(P):
    P64 = oracle.widen(P)
    return P64, oracle.log_table(P64)


def test_log_table_is_correctly_rounded():
    # Reference: the natural log to 45 significant digits in Python's decimal
    # module, then rounded to the nearest double.  Includes FP32-widened values
    # and the region near 1 where log loses relative accuracy most easily.
    from decimal import Decimal, getcontext
    getcontext().prec = 45
    vals = np.concatenate([
        synth.dirichlet(5, 300, 20, np.float32).ravel().astype(np.float64),
        synth.dirichlet(6, 100, 7, np.float64).ravel(),
        1.0 - 2.0 ** -np.arange(1, 53, dtype=np.float64),
        np.array([1e-12, 1.0, 0.5, 0.75, 2.0 ** -30, 0.7071067811865476, 0.7071067811865475]),
    ])
    L = oracle.log_table(vals)
    for v, l in zip(vals, L):
        assert l == float(Decimal(float(v)).ln()), v


def test_self_divergence_is_exact_zero():
    P64, L = _table(synth.dirichlet(11, 20, 9, np.float64))
    for x in range(20):
        k = oracle.key(P64, L, x, x)
        assert k == 0.0 and math.copysign(1.0, k) == 1.0


def test_two_coordinates_reduce_to_bernoulli_kl():
    # d = 1: KL of Bernoulli(p) from Bernoulli(q), written with ratios.
    rng = np.random.default_rng(3)
    p = rng.uniform(0.01, 0.99, 40)
    P64 = np.stack([p, 1.0 - p], axis=1)
    P64, L = _table(P64)
    for x in range(40):
        for y in range(40):
            a, b = P64[x, 0], P64[y, 0]
            ref = a * math.log(a / b) + (1 - a) * math.log((1 - a) / (1 - b))
            got = oracle.key(P64, L, x, y)
            assert abs(got - ref) <= 1e-14 * max(1.0, abs(ref)) + 1e-16


def test_uniform_second_argument_gives_negentropy_plus_log_d():
    # D(x || uniform) = sum_i x_i log x_i + log D   (entropy identity)
    D = 12
    P = synth.dirichlet(8, 30, D - 1, np.float64)
    P = np.vstack([P, np.full((1, D), 1.0 / D)])
    P64, L = _table(P)
    u = P.shape[0] - 1
    for x in range(30):
        ref = float(np.sum(P64[x] * np.log(P64[x]))) + math.log(D)
        assert abs(oracle.key(P64, L, x, u) - ref) < 1e-14


def test_matches_scipy_relative_entropy_and_is_asymmetric():
    from scipy.special import rel_entr
    P64, L = _table(synth.dirichlet(21, 25, 20, np.float64))
    asym = 0
    for x, y in itertools.product(range(25), range(25)):
        ref = float(np.sum(rel_entr(P64[x], P64[y])))
        got = oracle.key(P64, L, x, y)
        assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref))
        if x != y:
            assert got >= 0.0  # Gibbs' inequality on normalised points
            asym += oracle.key(P64, L, y, x) != got
    assert asym > 500


def test_fp32_storage_keeps_gibbs_up_to_mass_defect():
    # FP32-rounded points need not sum to 1; the key is still >= the mass
    # defect sum(x) - sum(y) minus rounding slack (log-sum inequality).
    P = synth.dirichlet(31, 40, 20, np.float32)
    P64, L = _table(P)
    s = P64.sum(axis=1)
    for x in range(40):
        for y in range(40):
            assert oracle.key(P64, L, x, y) >= (s[x] - s[y]) - 1e-12


def test_ranking_digraph_has_a_three_cycle():
    # Figure 1: six points drawn uniformly from a 14-simplex give a ranking
    # digraph with a 3-cycle xy -> xz ... back to xy, so the comparators cannot
    # come from a metric (the theorem of Section 2.1).  Search seeded draws.
    def has_cycle(P64, L):
        m = P64.shape[0]
        less = lambda x, y, z: oracle.key(P64, L, x, y) < oracle.key(P64, L, x, z)
        for a, b, c in itertools.permutations(range(m), 3):
            # {a,b} -> {a,c} (wrt a), {a,c} -> {b,c} (wrt c), {b,c} -> {a,b} (wrt b)
            if less(a, b, c) and less(c, a, b) and less(b, c, a):
                return True
        return False

    found = sum(has_cycle(*_table(synth.dirichlet(100 + s, 6, 14, np.float64)))
                for s in range(10))
    assert found >= 1
    # A symmetric dissimilarity never gives such a cycle: the same search with
    # the symmetrised key D(x||y) + D(y||x) finds none.
    for s in range(10):
        P64, L = _table(synth.dirichlet(100 + s, 6, 14, np.float64))
        sym = lambda x, y: oracle.key(P64, L, x, y) + oracle.key(P64, L, y, x)
        for a, b, c in itertools.permutations(range(6), 3):
            assert not (sym(a, b) < sym(a, c) and sym(c, a) < sym(c, b) and sym(b, c) < sym(b, a))
