"""Pins of two oracle entry points the GPU checks lean on.

* oracle_round_subset: the round's update (Section 3.1, "Update"; Section 4.2)
  for a chosen set of vertices only.  Each vertex's new list reads only the
  round-start snapshot (the independence Section 4.2 uses to spread vertices
  over processors), so its rows, update counts and evaluation counts must be
  those the whole round gives those vertices, and over all vertices they must
  add up to the round's totals.
* The carry-over rule the library applies in late rounds: a vertex whose own
  list did not change, that no list dropped, and whose friends' and
  co-friends' lists did not change has the same candidate set (co-friends,
  friends of friends, friends of co-friends, Section 3.1) as one round
  earlier, so the next round gives it the same list and the same number of
  evaluations.  Checked here on the oracle's own rounds, per vertex.
"""
import numpy as np
import pytest

import oracle
import synth


def _snapshot(seed, n, d, K, gseed, rounds=0):
    P = synth.dirichlet(seed, n, d, np.float32)
    P64 = oracle.widen(P)
    L = oracle.log_table(P64)
    F, keys = oracle.initial_graph(P64, L, K, gseed)
    for _ in range(rounds):
        F, keys, _, _ = oracle.round_step(P64, L, F, keys)
    return P64, L, F, keys


@pytest.mark.parametrize("rounds", [0, 2])
def test_round_subset_all_vertices_is_the_round(rounds):
    P64, L, F, keys = _snapshot(21, 1500, 6, 10, 5, rounds)
    Fn, kn, upd, ev = oracle.round_step(P64, L, F, keys)
    xs = np.arange(F.shape[0])
    Fo, ko, up, evs = oracle.round_subset(P64, L, F, keys, xs, threads=3)
    assert np.array_equal(Fo, Fn)
    assert np.array_equal(ko.view(np.uint64), kn.view(np.uint64))
    assert int(up.sum()) == upd and int(evs.sum()) == ev
    # per vertex: updates are the new entries, evaluations the candidate set's size
    for x in range(0, F.shape[0], 97):
        assert up[x] == len(set(Fn[x].tolist()) - set(F[x].tolist()))
        assert evs[x] == len(oracle.candidates(F, x))


def test_round_subset_rows_of_a_random_subset():
    P64, L, F, keys = _snapshot(22, 2500, 9, 16, 6, 1)
    Fn, kn, _, _ = oracle.round_step(P64, L, F, keys)
    xs = np.random.default_rng(3).permutation(F.shape[0])[:400]
    for threads in (1, 5):
        Fo, ko, up, evs = oracle.round_subset(P64, L, F, keys, xs, threads=threads)
        assert np.array_equal(Fo, Fn[xs])
        assert np.array_equal(ko.view(np.uint64), kn[xs].view(np.uint64))
        for i in range(0, xs.size, 37):
            x = int(xs[i])
            assert up[i] == len(set(Fn[x].tolist()) - set(F[x].tolist()))
            assert evs[i] == len(oracle.candidates(F, x))


def _cofriends(F):
    n, K = F.shape
    co = [[] for _ in range(n)]
    for x in range(n):
        for y in F[x].tolist():
            co[y].append(x)
    return co


@pytest.mark.parametrize("n,d,K,ds,seed", [(3000, 4, 8, 9, 3), (4000, 6, 12, 4, 17)])
def test_carry_over_rule_holds_on_oracle_rounds(n, d, K, ds, seed):
    P64, L, F, keys = _snapshot(ds, n, d, K, seed)
    xs = np.arange(n)
    prev = None   # (F_{r-1}, evaluations of round r-1 per vertex)
    fired = 0
    for _ in range(40):
        Fn, kn, up, ev = oracle.round_subset(P64, L, F, keys, xs)
        if prev is not None:
            Fp, evp = prev
            # flags of the round that produced F from Fp
            gained = np.array([set(F[x].tolist()) != set(Fp[x].tolist()) for x in range(n)])
            dropped = np.zeros(n, dtype=bool)
            for x in np.nonzero(gained)[0]:
                for y in set(Fp[x].tolist()) - set(F[x].tolist()):
                    dropped[y] = True
            co = _cofriends(F)
            for x in range(n):
                same = (not gained[x] and not dropped[x] and not gained[F[x]].any()
                        and not any(gained[w] for w in co[x]))
                if same:
                    fired += 1
                    assert np.array_equal(Fn[x], F[x]), x
                    assert np.array_equal(kn[x].view(np.uint64), keys[x].view(np.uint64)), x
                    assert ev[x] == evp[x], x
        prev = (F, ev)
        F, keys = Fn, kn
        if int(up.sum()) == 0:
            break
    assert int(up.sum()) == 0
    assert fired > 0  # the rule applies to some vertex in late rounds
