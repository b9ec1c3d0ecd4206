"""Pins of the oracle's descent: initial graph (Section 3.2), candidate set and
update (Sections 3.1, 4.2), friend clustering rate and stop rule (Section 3.3)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _setup(seed, n, d, dtype=np.float64):
    P = synth.dirichlet(seed, n, d, dtype)
    P64 = oracle.widen(P)
    return P, P64, oracle.log_table(P64)


def _adjacency(F, n):
    A = np.zeros((n, n), dtype=bool)
    for x in range(n):
        A[x, F[x]] = True
    return A


def _check_lists(P64, L, F, keys):
    n, K = F.shape
    for x in range(n):
        row = F[x]
        assert len(set(row.tolist())) == K and x not in row
        for j in range(K):
            assert keys[x, j] == oracle.key(P64, L, x, int(row[j]))
        order = sorted(zip(keys[x].tolist(), row.tolist()))
        assert [i for _, i in order] == row.tolist()


def test_initial_graph_is_sorted_k_out():
    _, P64, L = _setup(3, 300, 4)
    F, keys = oracle.initial_graph(P64, L, 7, seed=77)
    _check_lists(P64, L, F, keys)


def test_initial_graph_draw_rule():
    # Draw a of x is r = bound(H(seed,1,x,a), n-1), shifted past x; the first
    # K distinct draws form the friend set.
    n, K, seed = 50, 5, 9
    _, P64, L = _setup(4, n, 3)
    F, _ = oracle.initial_graph(P64, L, K, seed)
    for x in range(n):
        chosen, a = [], 0
        while len(chosen) < K:
            r = oracle.bound(oracle.hash64(seed, 1, x, a), n - 1)
            y = r + (r >= x)
            if y not in chosen:
                chosen.append(y)
            a += 1
        assert sorted(chosen) == sorted(F[x].tolist())


def test_initial_in_degree_is_binomial():
    # Random K-out: each other point picks y with probability K/(n-1), so the
    # in-degree is Binomial(n-1, K/(n-1)).  Chi-square over pooled cells.
    from scipy import stats
    n, K = 20_000, 8
    _, P64, L = _setup(5, n, 2)
    F, _ = oracle.initial_graph(P64, L, K, seed=5)
    deg = np.bincount(F.ravel(), minlength=n)
    assert deg.sum() == n * K
    edges = [0, 4, 6, 7, 8, 9, 10, 12, 100]
    obs = np.histogram(deg, bins=edges)[0]
    cdf = stats.binom(n - 1, K / (n - 1)).cdf
    probs = np.diff([0.0] + [cdf(e - 1) for e in edges[1:-1]] + [1.0])
    chi2 = ((obs - n * probs) ** 2 / (n * probs)).sum()
    assert chi2 < stats.chi2(len(obs) - 1).ppf(0.999)


def test_n_equals_k_plus_one_is_exact_at_start():
    n, K = 11, 10
    _, P64, L = _setup(6, n, 5)
    F, keys = oracle.initial_graph(P64, L, K, seed=1)
    bf, bk = oracle.bruteforce(P64, L, K, np.arange(n))
    assert np.array_equal(F, bf) and np.array_equal(keys, bk)


def test_candidate_set_matches_adjacency_algebra():
    # With A the friend adjacency (A[x,y] = y is a friend of x): co-friends of
    # x are column x of A, friends of friends are row x of A*A, friends of
    # co-friends are row x of A^T*A.  Remove x and its friends.
    n, K = 40, 4
    _, P64, L = _setup(7, n, 3)
    F, _ = oracle.initial_graph(P64, L, K, seed=12)
    A = _adjacency(F, n).astype(np.int64)
    reach = (A.T + A @ A + A.T @ A) > 0
    for x in range(n):
        want = set(np.nonzero(reach[x])[0].tolist()) - {x} - set(F[x].tolist())
        assert set(oracle.candidates(F, x).tolist()) == want
    # a co-friend of a friend is NOT a candidate by itself (the join is asymmetric)
    coco = (A @ A.T) > 0
    extra = [(x, y) for x in range(n) for y in np.nonzero(coco[x] & ~reach[x])[0] if y != x]
    assert extra, "this graph should contain co-friends of friends that are not candidates"


def test_round_update_is_best_k_of_friends_and_candidates():
    n, K = 60, 5
    _, P64, L = _setup(8, n, 4)
    F, keys = oracle.initial_graph(P64, L, K, seed=3)
    Fn, kn, upd, ev = oracle.round_step(P64, L, F, keys)
    tot_upd = tot_ev = 0
    for x in range(n):
        U = oracle.candidates(F, x).tolist()
        pool = [(keys[x, j], int(F[x, j])) for j in range(K)]
        pool += [(oracle.key(P64, L, x, z), z) for z in U]
        best = sorted(pool)[:K]
        assert [i for _, i in best] == Fn[x].tolist()
        assert [k for k, _ in best] == kn[x].tolist()
        tot_ev += len(U)
        tot_upd += len(set(Fn[x].tolist()) - set(F[x].tolist()))
    assert (upd, ev) == (tot_upd, tot_ev)


def test_round_that_sees_everyone_gives_exact_knn():
    # If every point meets every other point in a round, the round's output is
    # the exact K-NN graph (Section 2.3), whatever the start.
    n, K = 18, 6
    _, P64, L = _setup(9, n, 5)
    F, keys = oracle.initial_graph(P64, L, K, seed=1)
    covered = all(len(oracle.candidates(F, x)) + K == n - 1 for x in range(n))
    assert covered  # this seed's random 6-out graph reaches everyone in one round
    Fn, kn, _, _ = oracle.round_step(P64, L, F, keys)
    bf, bk = oracle.bruteforce(P64, L, K, np.arange(n))
    assert np.array_equal(Fn, bf) and np.array_equal(kn, bk)


def test_fixed_point_on_small_input_recovers_most_neighbours():
    n, K = 300, 8
    _, P64, L = _setup(10, n, 3)
    F, keys = oracle.initial_graph(P64, L, K, seed=5)
    for _ in range(30):
        Fn, kn, upd, _ = oracle.round_step(P64, L, F, keys)
        assert np.all(kn <= keys)  # rank-wise keys never increase
        F, keys = Fn, kn
        if upd == 0:
            break
    assert upd == 0
    bf, _ = oracle.bruteforce(P64, L, K, np.arange(n))
    recall = np.mean([len(set(a) & set(b)) / K for a, b in zip(F.tolist(), bf.tolist())])
    assert recall >= 0.95


def test_threads_do_not_change_results():
    P, _, _ = _setup(11, 3000, 6, np.float32)
    a = oracle.build_graph(P, 6, 12, seed=99, threads=1)
    b = oracle.build_graph(P, 6, 12, seed=99, threads=8)
    assert a.rounds == b.rounds and np.array_equal(a.idx, b.idx)
    assert np.array_equal(a.keys.view(np.uint64), b.keys.view(np.uint64))
    assert np.array_equal(a.updates, b.updates) and np.array_equal(a.hits, b.hits)


def test_sampled_fcr_within_binomial_interval_of_exhaustive():
    n, K = 2000, 10
    _, P64, L = _setup(12, n, 5)
    F, keys = oracle.initial_graph(P64, L, K, seed=6)
    for _ in range(2):
        F, keys, _, _ = oracle.round_step(P64, L, F, keys)
    h, p = oracle.fcr_exhaustive(F)
    A = _adjacency(F, n)
    link = A | A.T
    ref = sum(int(link[F[x, a], F[x, b]]) for x in range(n) for a in range(K)
              for b in range(a + 1, K))
    assert h == ref and p == n * K * (K - 1) // 2
    rate = h / p
    M = 40_000
    got = oracle.fcr(F, seed=6, rnd=2, M=M) / M
    assert abs(got - rate) < 4.5 * math.sqrt(rate * (1 - rate) / M) + 2e-3


def test_fcr_sampling_rule():
    n, K, seed, r, M = 30, 4, 123, 3, 200
    _, P64, L = _setup(13, n, 3)
    F, _ = oracle.initial_graph(P64, L, K, seed=1)
    link = _adjacency(F, n)
    link = link | link.T
    hits = 0
    for s in range(M):
        x = oracle.bound(oracle.hash64(seed, 2, r, s), n)
        a = oracle.bound(oracle.hash64(seed, 3, r, s), K)
        bp = oracle.bound(oracle.hash64(seed, 4, r, s), K - 1)
        b = bp + (bp >= a)
        assert a != b
        hits += int(link[F[x, a], F[x, b]])
    assert oracle.fcr(F, seed, r, M) == hits


def test_stop_rule_on_hand_built_sequences():
    # Section 3.3 (iv): stop at the first round whose rate does not increase.
    def rounds_until_stop(hits, updates, max_rounds=100):
        for r in range(1, len(hits)):
            if oracle.should_stop(hits[r - 1], hits[r], updates[r], r, max_rounds):
                return r
        return None
    assert rounds_until_stop([5, 50, 300, 420, 419], [0, 9, 9, 9, 9]) == 4
    assert rounds_until_stop([5, 50, 300, 300], [0, 9, 9, 9]) == 3  # equal does not increase
    assert rounds_until_stop([5, 50, 300, 400], [0, 9, 0, 9]) == 2  # fixed point
    assert rounds_until_stop([5, 6, 7, 8, 9], [0, 1, 1, 1, 1], max_rounds=3) == 3


def test_argument_and_domain_errors():
    P = synth.dirichlet(14, 10, 3, np.float32)
    assert oracle.build_graph(P, 3, 10, 1).status == oracle.ERR_ARG  # K > n-1
    assert oracle.build_graph(P, 3, 1, 1).status == oracle.ERR_ARG  # K < 2
    bad = P.copy()
    bad[3, 2] = 0.0
    assert oracle.build_graph(bad, 3, 4, 1).status == oracle.ERR_DOMAIN
    bad[3, 2] = np.nan
    assert oracle.build_graph(bad, 3, 4, 1).status == oracle.ERR_DOMAIN


def test_paper_table3_first_row_statistics():
    # Table 3, first row: n = 2e4 points on the 9-simplex (10 coordinates),
    # K = 16 stopped after 5 rounds (bound 2*ceil(log_K n) = 8) with final
    # clustering coefficient 0.271, and accuracy typically 95% or better.
    # Our draws differ from the paper's, so these are loose statistical checks.
    with open(os.path.join(GOLDEN, "paper_table3.json")) as f:
        row = json.load(f)["rows"][0]
    n, K, D = row["n"], row["K"], row["coordinates"]
    P = synth.dirichlet(4242, n, D - 1, np.float64)
    M = n
    res = oracle.build_graph(P, D - 1, K, seed=4343, M=M)
    assert res.status == oracle.OK
    assert res.rounds <= row["round_bound"]
    assert abs(res.rounds - row["rounds"]) <= 2
    fcc = res.hits[-1] / M
    assert abs(fcc - row["fcc"]) < 0.05
    P64 = oracle.widen(P)
    L = oracle.log_table(P64)
    qs = synth.subsample(4343, n, 200)
    bf, _ = oracle.bruteforce(P64, L, K, qs)
    acc = np.mean([len(set(res.idx[q].tolist()) & set(b.tolist())) / K for q, b in zip(qs, bf)])
    assert acc >= 0.9


# ---------------------------------------------------------------------------
# Other terminations (Section 1.2, Table 1, and Section 1.3, item (b)): "no possible update"
# and Dong et al.'s delta-proportion rule.  All rules follow one trajectory
# and differ only in the round they stop at.
# ---------------------------------------------------------------------------
def test_stop_rules_on_hand_built_sequences():
    n, K = 1000, 10
    # fixed point: only a round without updates (or the cap) stops
    assert oracle.stop_rule(1, 0.0, n, K, 50, 40, 7, 3, 100) == (False, False)
    assert oracle.stop_rule(1, 0.0, n, K, 50, 60, 0, 3, 100) == (True, False)
    assert oracle.stop_rule(1, 0.0, n, K, 50, 60, 7, 100, 100) == (True, True)
    # delta: updates <= delta n K = 100
    assert oracle.stop_rule(2, 0.01, n, K, 50, 40, 101, 3, 100) == (False, False)
    assert oracle.stop_rule(2, 0.01, n, K, 50, 60, 100, 3, 100) == (True, False)
    assert oracle.stop_rule(2, 0.01, n, K, 50, 60, 101, 9, 9) == (True, True)
    # the statistical criterion is the default rule
    assert oracle.stop_rule(0, 0.0, n, K, 50, 50, 7, 3, 100) == (True, False)
    assert oracle.stop_rule(0, 0.0, n, K, 50, 51, 7, 3, 100) == (False, False)


def test_fixed_point_rule_reaches_a_fixed_point():
    P = synth.dirichlet(515, 400, 4, np.float64)
    fp = oracle.build_graph(P, 4, 6, seed=21, stop_rule=oracle.STOP_FIXED_POINT)
    assert fp.status == oracle.OK and fp.updates[-1] == 0
    P64 = oracle.widen(P)
    L = oracle.log_table(P64)
    Fn, kn, upd, _ = oracle.round_step(P64, L, fp.idx, fp.keys)
    assert upd == 0 and np.array_equal(Fn, fp.idx) and np.array_equal(kn, fp.keys)
    # the statistical rule stops on the same trajectory, no later
    st = oracle.build_graph(P, 4, 6, seed=21)
    assert st.rounds <= fp.rounds
    assert np.array_equal(st.updates, fp.updates[:st.rounds + 1])
    assert np.array_equal(st.hits, fp.hits[:st.rounds + 1])


def test_delta_rule_stops_at_first_small_round():
    n, d, K = 600, 5, 8
    P = synth.dirichlet(616, n, d, np.float64)
    fp = oracle.build_graph(P, d, K, seed=22, stop_rule=oracle.STOP_FIXED_POINT)
    for delta in (0.05, 0.01, 0.001):
        first = next(r for r in range(1, fp.rounds + 1) if fp.updates[r] <= delta * n * K)
        dl = oracle.build_graph(P, d, K, seed=22, stop_rule=oracle.STOP_DELTA, delta=delta)
        assert dl.status == oracle.OK and dl.rounds == first
        cut = oracle.build_graph(P, d, K, seed=22, stop_rule=oracle.STOP_FIXED_POINT, max_rounds=first)
        assert np.array_equal(dl.idx, cut.idx) and np.array_equal(dl.keys, cut.keys)


def test_stop_rule_arguments():
    P = synth.dirichlet(3, 50, 3, np.float64)
    assert oracle.build_graph(P, 3, 4, 1, stop_rule=3).status == oracle.ERR_ARG
    assert oracle.build_graph(P, 3, 4, 1, stop_rule=2, delta=-1.0).status == oracle.ERR_ARG
