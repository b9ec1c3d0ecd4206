"""A round restricted to a share of the receivers (knnd_ctx_round_share): the
per-vertex tasks of a synchronous round read only the round-start graph
(Section 4.2 spreads them over processors), so the share's lists must be
exactly those of the full round, every other list must be carried over, and
the shares of a partition must add up to the full round's counts.
"""
import numpy as np
import pytest

import oracle
import paper_2202_00517_amd as knnd
import synth

pytestmark = pytest.mark.gpu

FORMS = [(0, knnd.KNND_PREC_FP64), (knnd.KNND_FLAG_PULL, knnd.KNND_PREC_FP64),
         (0, knnd.KNND_PREC_MIXED_BF16), (0, knnd.KNND_PREC_MIXED_FP16),
         (knnd.KNND_FLAG_ATOMIC_CSR, knnd.KNND_PREC_FP64), (knnd.KNND_FLAG_ATOMIC_CSR, knnd.KNND_PREC_MIXED_BF16)]
FORM_IDS = ["hub", "pull", "bf16", "fp16", "atomic_csr", "atomic_csr_bf16"]


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


def _ctx_after_rounds(P, d, K, seed, prm, rounds):
    c = knnd.Context(P, d, K, seed, prm)
    c.init_graph()
    for _ in range(rounds):
        c.round()
    return c


@pytest.mark.parametrize("form", FORMS, ids=FORM_IDS)
def test_shares_partition_the_full_round(form):
    n, d, K, seed = 20000, 10, 20, 61
    P = synth.dirichlet(60, n, d, np.float32)
    prm = knnd.default_params(flags=form[0], precision=form[1])
    say(f"share rounds n={n} d={d} K={K} form={form}")
    # round 2 from a real descent state (edges flagged by round 1)
    with _ctx_after_rounds(P, d, K, seed, prm, 1) as c:
        S_idx, S_kl = c.get_graph()
        full = c.round()
        F_idx, F_kl = c.get_graph()
    cuts = [0, 1, 977, 2500, 7919, 10000, 15013, 19999, n]
    upd = ev = 0
    for a, b in zip(cuts[:-1], cuts[1:]):
        with _ctx_after_rounds(P, d, K, seed, prm, 1) as c:
            st = c.round_share(a, b - a)
            assert c.rounds == 2
            gi, gk = c.get_graph()
            # a share round lists only the reverse edges it reads; the
            # context's co-friend lists afterwards are whole again
            rp, col = c.cofriends()
        src = np.repeat(np.arange(n), K)
        deg = np.bincount(np.asarray(gi).ravel(), minlength=n)
        assert np.array_equal(rp, np.concatenate([[0], np.cumsum(deg)])), (a, b)
        assert np.array_equal(col, src[np.lexsort((src, np.asarray(gi).ravel()))].astype(np.int32)), (a, b)
        own = np.zeros(n, dtype=bool)
        own[a:b] = True
        assert np.array_equal(gi[own], F_idx[own]), (a, b)
        assert np.array_equal(bits(gk[own]), bits(F_kl[own])), (a, b)
        assert np.array_equal(gi[~own], S_idx[~own]), (a, b)
        assert np.array_equal(bits(gk[~own]), bits(S_kl[~own])), (a, b)
        upd += st["updates"]
        ev += st["evals_alg"]
    assert (upd, ev) == (full["updates"], full["evals_alg"])


def test_share_against_the_oracle_and_the_next_round():
    # the share's rows against the oracle's update of those vertices, and a
    # full round after the share round against the oracle's round from the
    # graph it left (that round skips no pair: receivers outside the share
    # evaluated nothing, so an old edge no longer vouches for its pairs)
    n, d, K, seed = 6000, 7, 12, 62
    P = synth.dirichlet(63, n, d, np.float32)
    P64 = oracle.widen(P)
    L = oracle.log_table(P64)
    a, m = 1234, 1500
    with _ctx_after_rounds(P, d, K, seed, knnd.default_params(), 1) as c:
        S_idx, S_kl = c.get_graph()
        st = c.round_share(a, m)
        gi, gk = c.get_graph()
        xs = np.arange(a, a + m)
        oi, ok, up, evs = oracle.round_subset(P64, L, S_idx, S_kl, xs)
        assert np.array_equal(gi[xs], oi) and np.array_equal(bits(gk[xs]), bits(ok))
        assert (st["updates"], st["evals_alg"]) == (int(up.sum()), int(evs.sum()))
        st2 = c.round()
        hi, hk = c.get_graph()
    o2i, o2k, u2, e2 = oracle.round_step(P64, L, gi, gk)
    assert np.array_equal(hi, o2i) and np.array_equal(bits(hk), bits(o2k))
    assert (st2["updates"], st2["evals_alg"]) == (u2, e2)


def _hub_snapshot(P, K, hub, seed):
    """Every point lists `hub` among its friends, so that receiver has n-1
    co-friends; rows sorted by the oracle's keys."""
    P64 = oracle.widen(P)
    L = oracle.log_table(P64)
    n = P.shape[0]
    rng = np.random.default_rng(seed)
    F = np.empty((n, K), dtype=np.int32)
    keys = np.empty((n, K), dtype=np.float64)
    for x in range(n):
        row = [] if x == hub else [hub]
        while len(row) < K:
            y = int(rng.integers(0, n))
            if y != x and y not in row:
                row.append(y)
        pairs = sorted((oracle.key(P64, L, x, y), y) for y in row)
        F[x] = [y for _, y in pairs]
        keys[x] = [k for k, _ in pairs]
    return P64, L, F, keys


@pytest.mark.parametrize("form", FORMS, ids=FORM_IDS)
def test_share_holding_a_hub_receiver(form):
    # the hub receiver (n-1 co-friends) overflows the guarded LDS class and is
    # redone in the global-memory class; the other share has none
    n, d, K = 30000, 4, 4
    hub = n // 3
    P = synth.dirichlet(64, n, d, np.float32)
    P64, L, F, k = _hub_snapshot(P, K, hub, 65)
    prm = knnd.default_params(flags=form[0], precision=form[1])
    for a, m in [(hub - 100, 300), (0, 5000)]:
        say(f"hub share form={form} first={a} count={m}")
        with knnd.Context(P, d, K, 5, prm) as c:
            c.set_graph(F, k, 0)
            st = c.round_share(a, m)
            gi, gk = c.get_graph()
        xs = np.arange(a, a + m)
        oi, ok, up, evs = oracle.round_subset(P64, L, F, k, xs)
        assert np.array_equal(gi[xs], oi) and np.array_equal(bits(gk[xs]), bits(ok))
        assert (st["updates"], st["evals_alg"]) == (int(up.sum()), int(evs.sum()))
        rest = np.ones(n, dtype=bool)
        rest[xs] = False
        assert np.array_equal(gi[rest], F[rest]) and np.array_equal(bits(gk[rest]), bits(k[rest]))


def test_share_argument_errors():
    n, d, K = 500, 3, 5
    P = synth.dirichlet(66, n, d, np.float32)
    with knnd.Context(P, d, K, 1) as c:
        with pytest.raises(knnd.KnndError) as e:
            c.round_share(0, 10)  # no graph yet
        assert e.value.status == knnd.KNND_ERR_ARG
        c.init_graph()
        for a, m in [(-1, 10), (0, 0), (n - 5, 6), (n, 1)]:
            with pytest.raises(knnd.KnndError) as e:
                c.round_share(a, m)
            assert e.value.status == knnd.KNND_ERR_ARG
        assert c.rounds == 0
        st = c.round_share(n - 1, 1)
        assert c.rounds == 1 and st["evals_alg"] > 0
