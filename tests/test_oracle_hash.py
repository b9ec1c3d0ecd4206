"""Pins of the oracle's counter-based randomness."""
import numpy as np
import pytest

import oracle
import synth


def test_mix64_matches_published_splitmix64_vector():
    # SplitMix64 (Steele, Lea & Flood 2014) seeded with 1234567: the state
    # advances by the golden gamma and each output is the mix64 finalizer of
    # the state.  These five outputs are the generator's published test vector.
    expected = [6457827717110365317, 3203168211198807973, 9817491932198370423,
                4593380528125082431, 16408922859458223821]
    state = 1234567
    for e in expected:
        state = (state + 0x9E3779B97F4A7C15) % (1 << 64)
        assert oracle.mix64(state) == e


def test_hash_is_composition_of_mixers():
    # H(s,t,a,b) chains three finalizer calls; check against the finalizer itself
    # (pinned above) and the generator's independent implementation.
    M = (1 << 64) - 1
    for s, t, a, b in [(0, 0, 0, 0), (2001, 1, 17, 3), (M, 7, M, 12345)]:
        h = oracle.mix64(s ^ ((t * 0x9E3779B97F4A7C15) & M))
        h = oracle.mix64(h ^ a)
        h = oracle.mix64(h ^ b)
        assert oracle.hash64(s, t, a, b) == h
        assert synth.hash64(s, t, a, b) == h


@pytest.mark.parametrize("m", [1, 2, 3, 10, 999_999, 2**31 - 1, 2**40 + 7])
def test_bound_closed_forms(m):
    top = (1 << 64) - 1
    assert oracle.bound(0, m) == 0
    assert oracle.bound(top, m) == m - 1
    assert oracle.bound(1 << 63, m) == m // 2
    for h in [12345, 1 << 50, (1 << 64) // 3, top - 99]:
        assert oracle.bound(h, m) == (h * m) >> 64
        assert synth.bound(h, m) == (h * m) >> 64


def test_bound_of_hash_is_uniform():
    # chi-square of 60,000 draws over 12 cells (11 dof); 0.1% critical value 31.3
    m, N = 12, 60_000
    counts = np.zeros(m)
    for s in range(N):
        counts[oracle.bound(oracle.hash64(99, 2, 5, s), m)] += 1
    chi2 = ((counts - N / m) ** 2 / (N / m)).sum()
    assert chi2 < 31.3
