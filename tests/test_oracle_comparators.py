"""Pins of the oracle's other comparators.  The method needs only a total
order on S \\ {x} for each x (Section 2.1, a ranking system; Section 1.3 (a));
besides D(x||y) the oracle offers D(y||x), sum (sqrt x_i - sqrt y_i)^2
(Hellinger) and sum (x_i - y_i)^2 (Euclidean), each folded in ascending
coordinate order with one fma per term."""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth

KL, REV, HEL, L2 = oracle.CMP_KL, oracle.CMP_KL_REVERSE, oracle.CMP_HELLINGER, oracle.CMP_L2
ALL = [KL, REV, HEL, L2]


def _table(P):
    P64 = oracle.widen(P)
    return P64, oracle.log_table(P64)


def test_reverse_is_kl_with_the_points_exchanged():
    P64, L = _table(synth.dirichlet(71, 40, 9, np.float32))
    for x, y in itertools.permutations(range(12), 2):
        r = oracle.key(P64, L, x, y, REV)
        k = oracle.key(P64, L, y, x, KL)
        assert np.float64(r).view(np.uint64) == np.float64(k).view(np.uint64)
    # and it is not the forward divergence
    assert oracle.key(P64, L, 0, 1, REV) != oracle.key(P64, L, 0, 1, KL)


def test_reverse_closed_forms():
    # two coordinates: D(y||x) for Bernoulli(p) at x and Bernoulli(q) at y
    for p, q in [(0.3, 0.7), (0.01, 0.5), (0.9, 0.2)]:
        P64 = np.array([[p, 1 - p], [q, 1 - q]])
        L = oracle.log_table(P64)
        want = q * math.log(q / p) + (1 - q) * math.log((1 - q) / (1 - p))
        assert oracle.key(P64, L, 0, 1, REV) == pytest.approx(want, rel=1e-14, abs=1e-17)
    # x uniform: D(y||u) = sum y log y + log D
    D = 7
    y = synth.dirichlet(72, 1, D - 1, np.float64)[0]
    P64 = np.vstack([np.full(D, 1.0 / D), y])
    L = oracle.log_table(P64)
    want = float(np.sum(y * np.log(y))) + math.log(D)
    assert oracle.key(P64, L, 0, 1, REV) == pytest.approx(want, rel=1e-13)


def test_euclidean_against_numpy_and_exact_cases():
    P64, L = _table(synth.dirichlet(73, 30, 12, np.float32))
    for x, y in [(0, 1), (3, 17), (29, 5)]:
        want = float(np.sum((P64[x] - P64[y]) ** 2))
        assert oracle.key(P64, L, x, y, L2) == pytest.approx(want, rel=1e-14)
    # small integers: every step exact
    P = np.array([[1.0, 2.0, 3.0, -4.0], [4.0, 6.0, 3.0, 0.0]])
    assert oracle.key(P, np.zeros_like(P), 0, 1, L2) == 9.0 + 16.0 + 0.0 + 16.0


def test_hellinger_against_closed_forms():
    # perfect squares: sqrt exact, so the value is exact
    P = np.array([[0.25, 0.75 - 0.0, 0.0], [0.0625, 0.5625, 0.375]])
    want = (0.5 - 0.25) ** 2 + (math.sqrt(0.75) - 0.75) ** 2 + (0.0 - math.sqrt(0.375)) ** 2
    assert oracle.key(P, np.zeros_like(P), 0, 1, HEL) == pytest.approx(want, rel=1e-15)
    # disjoint supports: sum x + sum y
    P = np.array([[0.5, 0.5, 0.0, 0.0], [0.0, 0.0, 0.25, 0.75]])
    assert oracle.key(P, np.zeros_like(P), 0, 1, HEL) == 2.0
    # sum (sqrt x - sqrt y)^2 = sum x + sum y - 2 sum sqrt(x y)  (Bhattacharyya form)
    P64, L = _table(synth.dirichlet(74, 20, 15, np.float64))
    for x, y in [(0, 1), (7, 12)]:
        bc = float(np.sum(np.sqrt(P64[x] * P64[y])))
        want = float(P64[x].sum() + P64[y].sum()) - 2 * bc
        assert oracle.key(P64, L, x, y, HEL) == pytest.approx(want, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("cmp", [HEL, L2])
def test_symmetric_comparators_are_exactly_symmetric_and_zero_on_self(cmp):
    P64, L = _table(synth.dirichlet(75, 25, 10, np.float32))
    for x, y in itertools.combinations(range(25), 2):
        a, b = oracle.key(P64, L, x, y, cmp), oracle.key(P64, L, y, x, cmp)
        assert np.float64(a).view(np.uint64) == np.float64(b).view(np.uint64)
    for x in range(25):
        assert oracle.key(P64, L, x, x, cmp) == 0.0


def _ranking_digraph_has_cycle(P64, L, cmp):
    """Arcs xy -> xz when y precedes z for x; a cycle exists iff a DFS finds a
    back edge."""
    n = P64.shape[0]
    nodes = [(a, b) for a in range(n) for b in range(a + 1, n)]
    idx = {e: i for i, e in enumerate(nodes)}
    adj = [[] for _ in nodes]
    for x in range(n):
        others = [y for y in range(n) if y != x]
        order = sorted(others, key=lambda y: (oracle.key(P64, L, x, y, cmp), y))
        for i, y in enumerate(order):
            for z in order[i + 1:]:
                adj[idx[tuple(sorted((x, y)))]].append(idx[tuple(sorted((x, z)))])
    color = [0] * len(nodes)

    def dfs(u):
        color[u] = 1
        for w in adj[u]:
            if color[w] == 1 or (color[w] == 0 and dfs(w)):
                return True
        color[u] = 2
        return False

    return any(color[u] == 0 and dfs(u) for u in range(len(nodes)))


@pytest.mark.parametrize("cmp", [HEL, L2])
def test_metric_comparators_give_acyclic_ranking_digraphs(cmp):
    # Section 2.1 theorem: the ranking digraph is acyclic iff the comparators
    # come from a metric; sqrt of both keys is a metric (Euclidean distance of
    # the points, or of their square roots).
    for s in range(6):
        P64, L = _table(synth.dirichlet(300 + s, 7, 3, np.float64))
        assert not _ranking_digraph_has_cycle(P64, L, cmp)


def test_reverse_kl_ranking_digraph_has_a_cycle():
    # the reverse divergence is not metrizable either (Section 2.2's argument
    # applies to it): some seeded draw of six points shows a cycle
    found = False
    for s in range(200):
        P64, L = _table(synth.dirichlet(400 + s, 6, 3, np.float64))
        if _ranking_digraph_has_cycle(P64, L, REV):
            found = True
            break
    assert found


@pytest.mark.parametrize("cmp", [HEL, L2])
def test_bruteforce_matches_kd_tree(cmp):
    spatial = pytest.importorskip("scipy.spatial")
    P64, L = _table(synth.dirichlet(76, 800, 6, np.float32))
    X = np.sqrt(P64) if cmp == HEL else P64
    qs = np.arange(0, 800, 37)
    K = 9
    idx, keys = oracle.bruteforce(P64, L, K, qs, cmp=cmp)
    dist, nb = spatial.cKDTree(X).query(X[qs], k=K + 1)
    assert np.array_equal(nb[:, 0], qs)  # the query itself first
    assert np.array_equal(idx, nb[:, 1:])
    assert np.allclose(np.sqrt(keys), dist[:, 1:], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("cmp", ALL)
def test_round_that_sees_everyone_gives_exact_knn(cmp):
    # n = 2K + 2 with a complete start: every candidate set covers S \ {x}
    n, K, d = 14, 6, 4
    P64, L = _table(synth.dirichlet(77 + cmp, n, d, np.float64))
    F0, k0 = oracle.initial_graph(P64, L, K, 5, cmp=cmp)
    F, k = F0, k0
    for _ in range(6):
        F, k, _, _ = oracle.round_step(P64, L, F, k, cmp=cmp)
    bf, bk = oracle.bruteforce(P64, L, K, np.arange(n), cmp=cmp)
    assert np.array_equal(F, bf) and np.array_equal(k, bk)


@pytest.mark.parametrize("cmp", ALL)
def test_descent_lists_are_sorted_best_k_of_their_keys(cmp):
    n, d, K = 500, 5, 8
    P = synth.dirichlet(78, n, d, np.float64)
    r = oracle.build_graph(P, d, K, 9, cmp=cmp, stop_rule=oracle.STOP_FIXED_POINT)
    assert r.status == oracle.OK and r.updates[-1] == 0
    P64, L = _table(P)
    for x in range(0, n, 50):
        row = r.idx[x]
        assert len(set(row.tolist())) == K and x not in row
        for j, y in enumerate(row):
            assert r.keys[x, j] == oracle.key(P64, L, x, int(y), cmp)
        assert all((r.keys[x, j], row[j]) < (r.keys[x, j + 1], row[j + 1]) for j in range(K - 1))
    # a different comparator gives a different graph
    if cmp != KL:
        assert not np.array_equal(r.idx, oracle.build_graph(P, d, K, 9).idx)


def test_domains_of_the_comparators():
    d, K = 3, 2
    P = np.full((6, 4), 0.25)
    P[2, 1] = 0.0
    assert oracle.build_graph(P, d, K, 1, cmp=KL).status == oracle.ERR_DOMAIN
    assert oracle.build_graph(P, d, K, 1, cmp=REV).status == oracle.ERR_DOMAIN
    assert oracle.build_graph(P, d, K, 1, cmp=HEL).status == oracle.OK
    P[3, 0] = -0.5
    assert oracle.build_graph(P, d, K, 1, cmp=HEL).status == oracle.ERR_DOMAIN
    assert oracle.build_graph(P, d, K, 1, cmp=L2).status == oracle.OK
    P[4, 2] = np.inf
    assert oracle.build_graph(P, d, K, 1, cmp=L2).status == oracle.ERR_DOMAIN
    assert oracle.build_graph(P, d, K, 1, cmp=7).status == oracle.ERR_ARG
