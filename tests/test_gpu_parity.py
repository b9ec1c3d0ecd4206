"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar: neighbor lists and per-round counts bit-exact; keys compared as FP64
bits (the tolerance allowed for keys is 1e-12 relative; the canonical key
definition makes them identical, so the test demands identity).
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import paper_2202_00517_amd as knnd
import synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


def assert_same_graph(gi, gk, oi, ok, what):
    gi = np.asarray(gi)
    bad = np.nonzero((gi != oi).any(axis=1))[0]
    assert bad.size == 0, f"{what}: {bad.size} rows differ, first x={bad[:5].tolist()}"
    kb = np.nonzero((bits(gk) != bits(ok)).any(axis=1))[0]
    assert kb.size == 0, f"{what}: keys differ in {kb.size} rows, first x={kb[:5].tolist()}"


def full_compare(P, d, K, seed, M=0, flags=0, max_rounds=100, precision=0, stop_rule=0, delta=0.0,
                 cmp=0):
    say(f"full build n={P.shape[0]} d={d} K={K} seed={seed} {P.dtype} M={M} flags={flags} "
        f"precision={precision} stop_rule={stop_rule} delta={delta} cmp={cmp}")
    prm = knnd.default_params(fcr_samples=M, flags=flags, max_rounds=max_rounds,
                              precision=precision, stop_rule=stop_rule, delta=delta, comparator=cmp)
    g = knnd.knnd_build_ex(P, d, K, seed, prm)
    o = oracle.build_graph(P, d, K, seed, M=M, max_rounds=max_rounds, stop_rule=stop_rule,
                           delta=delta, cmp=cmp)
    assert g["status"] == o.status
    assert g["rounds"] == o.rounds, (g["rounds"], o.rounds)
    for r in range(o.rounds + 1):
        s = g["stats"][r]
        assert s["fcr_hits"] == o.hits[r], (r, s, o.hits[r])
        if r:
            assert (s["updates"], s["evals_alg"]) == (o.updates[r], o.evals[r]), (r, s)
    assert_same_graph(g["idx"], g["kl"], o.idx, o.keys, "final graph")
    return g, o


# ---------------------------------------------------------------------------
# a0: log table and initial graph
# ---------------------------------------------------------------------------
def test_log_table_bit_exact():
    specials = np.array([1.0, 1e-12, 0.5, 0.75, 2.0 ** -30, 0.7071067811865476, 0.7071067811865475,
                         1.4142135623730951, 1.0 - 2.0 ** -53, 1e-310, 5e-324, 3.0, 1e300,
                         0.999999, 1e-5, 0.1, 0.2, 0.3], dtype=np.float64)
    near1 = 1.0 - 2.0 ** -np.arange(1, 55, dtype=np.float64)
    vals = np.concatenate([specials, near1, np.random.default_rng(1).uniform(1e-9, 1.0, 4000)])
    D = 8
    vals = vals[: (vals.size // D) * D].reshape(-1, D)
    say(f"log table of {vals.size} special/random values")
    with knnd.Context(vals, D - 1, 2, 1) as c:
        L = c.log_table()
    ref = oracle.log_table(vals)
    assert np.array_equal(bits(L), bits(ref))
    for cfg in ("n2000_d5_k10", "n100000_d10_k20"):
        cf = synth.WORKLOADS[cfg]
        P = synth.dirichlet(cf["data_seed"], cf["n"], cf["d"], cf["dtype"])
        say(f"log table {cfg}")
        with knnd.Context(P, cf["d"], cf["K"], cf["seed"]) as c:
            L = c.log_table()
        assert np.array_equal(bits(L), bits(oracle.log_table(oracle.widen(P))))


@pytest.mark.parametrize("n,d,K,dtype", [(2000, 5, 10, np.float64), (5000, 10, 20, np.float32),
                                         (65, 3, 64, np.float32), (11, 2, 10, np.float32),
                                         (777, 1, 2, np.float64)])
def test_initial_graph_bit_exact(n, d, K, dtype):
    P = synth.dirichlet(500 + n, n, d, dtype)
    seed = 900 + n
    say(f"initial graph n={n} d={d} K={K} {np.dtype(dtype).name}")
    with knnd.Context(P, d, K, seed) as c:
        st = c.init_graph()
        gi, gk = c.get_graph()
    P64 = oracle.widen(P)
    L = oracle.log_table(P64)
    oi, ok = oracle.initial_graph(P64, L, K, seed)
    assert_same_graph(gi, gk, oi, ok, "initial graph")
    assert st["fcr_hits"] == oracle.fcr(oi, seed, 0, min(n, 10000))


# ---------------------------------------------------------------------------
# a1..a5: one round from the oracle's own snapshot
# ---------------------------------------------------------------------------
def one_round(P, d, K, seed, F0=None, k0=None, flags=0, precision=0, cmp=0):
    P64 = oracle.widen(P)
    L = oracle.log_table(P64) if cmp in (0, 1) else np.zeros_like(P64)
    if F0 is None:
        F0, k0 = oracle.initial_graph(P64, L, K, seed, cmp=cmp)
    say(f"one round n={P.shape[0]} d={d} K={K} flags={flags} precision={precision} cmp={cmp}")
    prm = knnd.default_params(flags=flags, precision=precision, comparator=cmp)
    with knnd.Context(P, d, K, seed, prm) as c:
        c.set_graph(F0, k0, 0)
        st = c.round()
        gi, gk = c.get_graph()
    oi, ok, upd, ev = oracle.round_step(P64, L, F0, k0, cmp=cmp)
    assert_same_graph(gi, gk, oi, ok, "round 1")
    assert (st["updates"], st["evals_alg"]) == (upd, ev)
    assert st["fcr_hits"] == oracle.fcr(oi, seed, 1, min(P.shape[0], 10000))
    return st


# Checkpoint and resume: a round's state is its lists, keys and round index
# (every random draw is a hash of the seed and indices), so a descent saved
# after round r and resumed in a fresh context follows the uninterrupted one
# exactly: the same lists, keys, update, evaluation and FCR counts in every
# later round (only the evaluations performed differ: the resumed round
# counts every edge as new and skips no pair).
def _resume_case(P, d, K, seed, prm, save_at, total):
    with knnd.Context(P, d, K, seed, prm) as c:
        c.init_graph()
        ref = []
        for r in range(1, total + 1):
            st = c.round()
            if r == save_at:
                si, sk = c.get_graph()
            ref.append(st)
        fi, fk = c.get_graph()
    with knnd.Context(P, d, K, seed, prm) as c:
        c.set_graph(si, sk, save_at)
        got = [c.round() for _ in range(save_at + 1, total + 1)]
        gi, gk = c.get_graph()
    for a, b in zip(ref[save_at:], got):
        assert (a["updates"], a["evals_alg"], a["fcr_hits"]) == (b["updates"], b["evals_alg"], b["fcr_hits"]), (a, b)
    assert np.array_equal(fi, gi) and np.array_equal(bits(fk), bits(gk))


@pytest.mark.parametrize("form", [(0, knnd.KNND_PREC_FP64), (0, knnd.KNND_PREC_MIXED_BF16),
                                  (knnd.KNND_FLAG_PULL, knnd.KNND_PREC_FP64)], ids=["hub", "bf16", "pull"])
@pytest.mark.parametrize("save_at", [1, 3])
def test_resume_from_a_saved_round(form, save_at):
    P = synth.dirichlet(41, 20000, 10, np.float32)
    say(f"resume after round {save_at}, form {form}")
    _resume_case(P, 10, 16, 5, knnd.default_params(flags=form[0], precision=form[1]), save_at, 6)


JOIN_FORMS = [0, knnd.KNND_FLAG_PULL]
# (flags, precision): exact hub form, pull form, BF16 and FP16 mixed forms
FORMS = [(0, knnd.KNND_PREC_FP64), (knnd.KNND_FLAG_PULL, knnd.KNND_PREC_FP64),
         (0, knnd.KNND_PREC_MIXED_BF16), (0, knnd.KNND_PREC_MIXED_FP16)]
FORM_IDS = ["hub", "pull", "bf16", "fp16"]


@pytest.mark.parametrize("form", FORMS, ids=FORM_IDS)
@pytest.mark.parametrize("n,d,K", [(11, 3, 10), (200, 1, 2), (1000, 6, 16), (3001, 20, 30),
                                   (4097, 60, 64), (20000, 10, 20)])
def test_one_round_bit_exact(n, d, K, form):
    one_round(synth.dirichlet(n + 7, n, d, np.float32), d, K, seed=n, flags=form[0],
              precision=form[1])


def _hub_snapshot(P, K, hub, seed):
    """Every point lists `hub` among its friends (the hub's own list is random),
    so one receiver has n-1 co-friends.  Rows sorted by the oracle's keys."""
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
    return F, keys


@pytest.mark.parametrize("form", FORMS, ids=FORM_IDS)
@pytest.mark.parametrize("n,d,K", [(3000, 6, 8), (7000, 5, 4), (18005, 4, 4), (30000, 4, 4),
                                   (40000, 4, 4)])
def test_hub_receiver_large_tables(n, d, K, form):
    # The receiver with n-1 co-friends lands in the 16384-slot LDS class
    # (n=3000 and 7000), in the 32768-slot class with about 18000 distinct
    # candidates, more than 16384 (n=18005), in the 32768-slot class whose
    # guard hands it to the global-memory class (n=30000), and directly in the
    # global-memory class (n=40000).
    P = synth.dirichlet(n + 11, n, d, np.float32)
    F, k = _hub_snapshot(P, K, hub=n // 3, seed=n)
    one_round(P, d, K, seed=5, F0=F, k0=k, flags=form[0], precision=form[1])


@pytest.mark.parametrize("form", FORMS, ids=FORM_IDS)
def test_exact_ties_break_by_index(form):
    # 20 distinct points, each repeated 12 times: many keys tie exactly
    base = synth.dirichlet(31, 20, 5, np.float32)
    P = np.repeat(base, 12, axis=0)
    full_compare(P, 5, 8, seed=17, flags=form[0], precision=form[1])


# ---------------------------------------------------------------------------
# whole descent (all rounds, stop test) against the oracle
# ---------------------------------------------------------------------------
def test_n2000_d5_k10_full():
    c = synth.WORKLOADS["n2000_d5_k10"]
    P = synth.dirichlet(c["data_seed"], c["n"], c["d"], c["dtype"])
    full_compare(P, c["d"], c["K"], c["seed"])


def test_random_small_workloads_full():
    rng = np.random.default_rng(2024)
    for i in range(24):
        n = int(rng.integers(30, 5000))
        d = int(rng.integers(1, 61))
        K = int(rng.integers(2, min(64, n - 1) + 1))
        dtype = np.float32 if rng.random() < 0.7 else np.float64
        P = synth.dirichlet(3000 + i, n, d, dtype)
        flags, prec = FORMS[i % len(FORMS)]
        full_compare(P, d, K, seed=4000 + i, flags=flags, precision=prec)


@pytest.mark.parametrize("form", JOIN_FORMS, ids=["hub", "pull"])
def test_skipping_old_paths_changes_nothing(form):
    P = synth.dirichlet(8, 6000, 9, np.float32)
    a = knnd.knnd_build_ex(P, 9, 16, 33, knnd.default_params(flags=form))
    b = knnd.knnd_build_ex(P, 9, 16, 33, knnd.default_params(flags=form | knnd.KNND_FLAG_NO_SKIP))
    assert a["rounds"] == b["rounds"]
    assert np.array_equal(a["idx"], b["idx"]) and np.array_equal(bits(a["kl"]), bits(b["kl"]))
    for sa, sb in zip(a["stats"], b["stats"]):
        assert (sa["updates"], sa["fcr_hits"], sa["evals_alg"]) == \
            (sb["updates"], sb["fcr_hits"], sb["evals_alg"])
    assert sum(s["evals_performed"] for s in a["stats"]) < sum(s["evals_performed"] for s in b["stats"])
    if form == knnd.KNND_FLAG_PULL:
        assert b["stats"][1]["evals_performed"] == b["stats"][1]["evals_alg"]
    else:  # the hub form computes every candidate occurrence except x itself
        n, K = 6000, 16
        assert b["stats"][1]["evals_performed"] == n * K * (2 * K + 1) - n * K


STOP_CASES = [(knnd.KNND_STOP_FIXED_POINT, 0.0), (knnd.KNND_STOP_DELTA, 0.01),
              (knnd.KNND_STOP_DELTA, 0.001), (knnd.KNND_STOP_DELTA, 0.0)]


@pytest.mark.parametrize("form", [FORMS[0], FORMS[2]], ids=["hub", "bf16"])
@pytest.mark.parametrize("rule,delta", STOP_CASES, ids=["fixed_point", "delta1e-2", "delta1e-3", "delta0"])
@pytest.mark.parametrize("n,d,K,ds,seed", [(3001, 20, 30, 5, 7), (20000, 10, 20, 6, 8), (5000, 4, 8, 9, 3)])
def test_stop_rules_full(n, d, K, ds, seed, rule, delta, form):
    P = synth.dirichlet(ds, n, d, np.float32)
    g, o = full_compare(P, d, K, seed, flags=form[0], precision=form[1], stop_rule=rule, delta=delta)
    if rule == knnd.KNND_STOP_FIXED_POINT or delta == 0.0:
        assert g["stats"][g["rounds"]]["updates"] == 0


# Receivers whose neighbourhood did not change keep their list and evaluation
# count (the candidate set is the same, Section 3.1): the fixed-point descent
# reaches rounds with few changes, where the carry-over fires; its lists, key
# bits and every per-round count equal the oracle's and those of the same
# descent with the carry-over switched off.
@pytest.mark.parametrize("form", [FORMS[0], FORMS[2]], ids=["hub", "bf16"])
@pytest.mark.parametrize("n,d,K,ds,seed", [(20000, 10, 20, 6, 8), (5000, 4, 8, 9, 3)])
def test_carry_over_fires_and_matches(n, d, K, ds, seed, form):
    P = synth.dirichlet(ds, n, d, np.float32)
    g, o = full_compare(P, d, K, seed, flags=form[0], precision=form[1],
                        stop_rule=knnd.KNND_STOP_FIXED_POINT)
    carried = [s["carried"] for s in g["stats"]]
    assert max(carried) > 0, carried
    for s in g["stats"]:
        assert 0 <= s["evals_carried"] <= s["evals_alg"]
        assert (s["carried"] == 0) == (s["evals_carried"] == 0)
    h = knnd.knnd_build_ex(P, d, K, seed, knnd.default_params(
        flags=form[0] | knnd.KNND_FLAG_NO_CARRY, precision=form[1],
        stop_rule=knnd.KNND_STOP_FIXED_POINT))
    assert h["rounds"] == g["rounds"]
    assert all(s["carried"] == 0 and s["evals_carried"] == 0 for s in h["stats"])
    for a, b in zip(g["stats"], h["stats"]):
        assert (a["updates"], a["fcr_hits"], a["evals_alg"]) == (b["updates"], b["fcr_hits"], b["evals_alg"])
    assert np.array_equal(g["idx"], h["idx"])
    assert np.array_equal(bits(g["kl"]), bits(h["kl"]))


def test_stop_rule_round_cap_warns():
    P = synth.dirichlet(9, 5000, 4, np.float32)
    g, o = full_compare(P, 4, 8, 3, max_rounds=4, stop_rule=knnd.KNND_STOP_FIXED_POINT)
    assert g["status"] == knnd.KNND_WARN_MAX_ROUNDS and g["rounds"] == 4


# Reverse neighbours (Section 3.1): the co-friend lists a round builds from
# its snapshot, against their construction from the lists themselves; two
# builds agree bit for bit (rowptr is a count and a scan, and the interface
# sorts each segment; the join leaves the order inside a segment free).
@pytest.mark.parametrize("flags", [0, knnd.KNND_FLAG_ATOMIC_CSR], ids=["bucketed", "atomic"])
def test_cofriend_lists(flags):
    P = synth.dirichlet(3, 20000, 6, np.float32)
    with knnd.Context(P, 6, 12, 5, knnd.default_params(flags=flags)) as c:
        c.init_graph()
        c.round()
        idx, _ = c.get_graph()
        rp1, col1 = c.cofriends()
        rp2, col2 = c.cofriends()
    idx = np.asarray(idx)
    n, K = idx.shape
    src = np.repeat(np.arange(n), K)
    deg = np.bincount(idx.ravel(), minlength=n)
    assert np.array_equal(rp1, np.concatenate([[0], np.cumsum(deg)]))
    order = np.lexsort((src, idx.ravel()))  # by target, then source
    assert np.array_equal(col1, src[order].astype(np.int32))
    assert np.array_equal(rp1, rp2) and np.array_equal(col1, col2)


@pytest.mark.parametrize("n,d,K,seed", [(20000, 10, 20, 8), (3001, 20, 30, 7)])
def test_atomic_reverse_neighbour_build(n, d, K, seed):
    # the per-edge atomic CSR build (used above 2^25 points) gives the same descent
    P = synth.dirichlet(6, n, d, np.float32)
    full_compare(P, d, K, seed, flags=knnd.KNND_FLAG_ATOMIC_CSR, precision=knnd.KNND_PREC_MIXED_BF16)


def test_round_cap_and_fcr_sample_size():
    P = synth.dirichlet(9, 4000, 8, np.float32)
    full_compare(P, 8, 12, seed=3, max_rounds=2)
    full_compare(P, 8, 12, seed=3, M=4000 * 3)


def test_device_pointers_match_host_path():
    import torch
    P = synth.dirichlet(10, 7000, 12, np.float32)
    h = knnd.knnd_build_ex(P, 12, 24, 44)
    g = knnd.knnd_build_ex(torch.from_numpy(P).cuda(), 12, 24, 44)
    torch.cuda.synchronize()
    assert g["rounds"] == h["rounds"]
    assert np.array_equal(g["idx"].cpu().numpy(), h["idx"])
    assert np.array_equal(bits(g["kl"].cpu().numpy()), bits(h["kl"]))


def test_basic_entry_point():
    P = synth.dirichlet(12, 2500, 4, np.float32)
    idx, upd, rounds, st = knnd.knnd_build(P, 4, 9, 123, max_rounds=50)
    o = oracle.build_graph(P, 4, 9, 123, max_rounds=50)
    assert st == o.status and rounds == o.rounds
    assert np.array_equal(idx, o.idx)
    assert np.array_equal(upd, o.updates[1:])


def test_domain_errors():
    P = synth.dirichlet(13, 100, 3, np.float32)
    for bad in (0.0, -0.1, np.nan, np.inf):
        Q = P.copy()
        Q[17, 2] = bad
        with pytest.raises(knnd.KnndError) as e:
            knnd.knnd_build_ex(Q, 3, 4, 1)
        assert e.value.status == knnd.KNND_ERR_DOMAIN


# ---------------------------------------------------------------------------
# full-size workloads against the oracle's stored digests
# ---------------------------------------------------------------------------
def _golden(name):
    path = os.path.join(GOLDEN, f"oracle_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as f:
        return json.load(f)


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def check_against_golden(cfg, precision=0):
    gold = _golden(cfg)
    c = synth.WORKLOADS[cfg]
    P = synth.dirichlet(c["data_seed"], c["n"], c["d"], c["dtype"])
    say(f"{cfg} full size vs stored oracle digests, precision {precision}")
    g = knnd.knnd_build_ex(P, c["d"], c["K"], c["seed"], knnd.default_params(precision=precision))
    assert g["status"] == gold["status"]
    assert g["rounds"] == gold["rounds"]
    assert [s["fcr_hits"] for s in g["stats"]] == gold["fcr_hits"]
    assert [s["updates"] for s in g["stats"]][1:] == gold["updates"][1:]
    assert [s["evals_alg"] for s in g["stats"]][1:] == gold["evals_alg"][1:]
    assert _digest(g["idx"]) == gold["idx_sha256"]
    assert _digest(g["kl"]) == gold["kl_sha256"]
    return g, P


def test_n100000_d10_k20_full_size():
    check_against_golden("n100000_d10_k20")


@pytest.mark.parametrize("form", FORMS, ids=FORM_IDS)
def test_n100000_d10_k20_live_oracle(form):
    c = synth.WORKLOADS["n100000_d10_k20"]
    P = synth.dirichlet(c["data_seed"], c["n"], c["d"], c["dtype"])
    g, _ = full_compare(P, c["d"], c["K"], c["seed"], flags=form[0], precision=form[1])
    resc = sum(s["rescues"] for s in g["stats"])
    if form[1] != knnd.KNND_PREC_FP64:
        alg = sum(s["evals_alg"] for s in g["stats"])
        say(f"n=100000 d=10 K=20 {FORM_IDS[FORMS.index(form)]}: rescued {resc} of {alg} evaluations "
            f"({100.0 * resc / alg:.2f}%)")
        assert 0 < resc < alg
    else:
        assert resc == 0


MIXED = [knnd.KNND_PREC_MIXED_BF16, knnd.KNND_PREC_MIXED_FP16]


@pytest.mark.parametrize("prec", MIXED, ids=["bf16", "fp16"])
def test_mixed_off_the_simplex_runs_exact(prec):
    # coordinates above 1 make some products x_i log c_i positive, where the
    # mixed error bound does not hold: the library must run the exact form
    P = synth.dirichlet(77, 3000, 6, np.float32) * np.float32(3.0)
    g, _ = full_compare(P, 6, 8, seed=9, precision=prec)
    assert all(s["rescues"] == 0 for s in g["stats"])


@pytest.mark.parametrize("prec", MIXED, ids=["bf16", "fp16"])
def test_mixed_tiny_coordinates(prec):
    # most coordinates far below the FP16 normal range (down to the 1e-12
    # clamp), so the subnormal part of the error bound matters
    base = synth.dirichlet(78, 4000, 15, np.float64) ** 6
    base = base / base.sum(axis=1, keepdims=True)
    P = np.maximum(base, 1e-12).astype(np.float32)
    assert (P < 2.0 ** -14).mean() > 0.3
    g, _ = full_compare(P, 15, 12, seed=10, precision=prec)
    assert sum(s["rescues"] for s in g["stats"]) > 0


def test_n1000000_d20_k30_mixed_bf16_full_size():
    g, _ = check_against_golden("n1000000_d20_k30", knnd.KNND_PREC_MIXED_BF16)
    resc = sum(s["rescues"] for s in g["stats"])
    alg = sum(s["evals_alg"] for s in g["stats"])
    say(f"n=1e6 d=20 K=30 bf16: rescued {resc} of {alg} evaluations ({100.0 * resc / alg:.2f}%)")


def test_n200000_d50_k20_mixed_fp16_full_size():
    g, _ = check_against_golden("n200000_d50_k20", knnd.KNND_PREC_MIXED_FP16)
    resc = sum(s["rescues"] for s in g["stats"])
    alg = sum(s["evals_alg"] for s in g["stats"])
    say(f"n=200000 d=50 K=20 fp16: rescued {resc} of {alg} evaluations ({100.0 * resc / alg:.2f}%)")


def test_n1000000_d20_k30_full_size():
    g, P = check_against_golden("n1000000_d20_k30")
    c = synth.WORKLOADS["n1000000_d20_k30"]
    # sampled rows recomputed key by key with the oracle's key function
    P64 = oracle.widen(P)
    L = oracle.log_table(P64)
    xs = synth.subsample(99, c["n"], 300)
    for x in xs:
        for j in range(c["K"]):
            assert g["kl"][x, j] == oracle.key(P64, L, int(x), int(g["idx"][x, j]))


def test_n1000000_d20_k30_round1_sampled_receivers():
    # Round 1 at full size from the oracle's own initial graph, on 2000 receivers.
    c = synth.WORKLOADS["n1000000_d20_k30"]
    P = synth.dirichlet(c["data_seed"], c["n"], c["d"], c["dtype"])
    P64 = oracle.widen(P)
    L = oracle.log_table(P64)
    F0, k0 = oracle.initial_graph(P64, L, c["K"], c["seed"])
    say("n=1e6 d=20 K=30 round 1 from the oracle snapshot")
    with knnd.Context(P, c["d"], c["K"], c["seed"]) as ctx:
        st0 = ctx.init_graph()
        gi, gk = ctx.get_graph()
        assert_same_graph(gi, gk, F0, k0, "n=1e6 d=20 K=30 initial graph")
        st1 = ctx.round()
        gi, gk = ctx.get_graph()
    xs = synth.subsample(7, c["n"], 2000)
    oi, ok, _, _ = oracle.round_subset(P64, L, F0, k0, xs)
    assert_same_graph(gi[xs], gk[xs], oi, ok, "n=1e6 d=20 K=30 round 1 sample")
    gold = _golden("n1000000_d20_k30")
    assert st0["fcr_hits"] == gold["fcr_hits"][0]
    assert (st1["updates"], st1["evals_alg"], st1["fcr_hits"]) == \
        (gold["updates"][1], gold["evals_alg"][1], gold["fcr_hits"][1])


def test_n200000_d50_k20_full_size_and_recall():
    g, P = check_against_golden("n200000_d50_k20")
    c = synth.WORKLOADS["n200000_d50_k20"]
    P64 = oracle.widen(P)
    L = oracle.log_table(P64)
    gold = _golden("n200000_d50_k20")
    qs = synth.subsample(c["seed"], c["n"], gold["recall_queries"])
    bf, bk = oracle.bruteforce(P64, L, c["K"], qs)
    hits = sum(len(set(g["idx"][q].tolist()) & set(b.tolist())) for q, b in zip(qs, bf))
    say(f"n=200000 d=50 K=20 recall@{c['K']} on {qs.size} queries: {hits / (qs.size * c['K']):.4f}")
    # the oracle's graph has the same recall, written by make_golden.py
    assert hits == gold["recall_hits"]
    # the library's exhaustive search, bounded by the descent's K-th keys
    ei, ek = knnd.knnd_exact_knn(P, c["d"], c["K"], qs.astype(np.int32), tau=g["kl"][qs, -1])
    assert np.array_equal(ei, bf)
    assert np.array_equal(bits(ek), bits(bk))


# ---------------------------------------------------------------------------
# Exhaustive search (knnd_exact_knn) against the oracle's brute force
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,d,K,dtype", [(5000, 9, 16, np.float32), (3001, 20, 30, np.float32),
                                         (700, 3, 64, np.float64), (12000, 59, 20, np.float32),
                                         (65, 1, 64, np.float32)])
def test_exact_knn_matches_oracle(n, d, K, dtype):
    P = synth.dirichlet(n + 5, n, d, dtype)
    P64 = oracle.widen(P)
    L = oracle.log_table(P64)
    qs = synth.subsample(n, n, min(n, 203))
    say(f"exact knn n={n} d={d} K={K} {np.dtype(dtype).name}, {qs.size} queries")
    bf, bk = oracle.bruteforce(P64, L, K, qs)
    ei, ek = knnd.knnd_exact_knn(P, d, K, qs.astype(np.int32))
    assert np.array_equal(ei, bf)
    assert np.array_equal(bits(ek), bits(bk))


def test_exact_knn_ties_and_bound_refinement():
    # 2 distinct points, 5000 copies each: every query has 4999 keys of exactly
    # zero; a bound of 0.0 admits all of them (more than one 4096-entry buffer
    # holds), so the bound must be tightened until the ties are settled by index
    base = synth.dirichlet(91, 2, 6, np.float32)
    P = np.repeat(base, 5000, axis=0)
    P64 = oracle.widen(P)
    L = oracle.log_table(P64)
    qs = np.array([0, 1, 4999, 5000, 9999, 7321], dtype=np.int64)
    bf, bk = oracle.bruteforce(P64, L, 12, qs)
    for tau in (None, np.zeros(qs.size)):
        ei, ek = knnd.knnd_exact_knn(P, 6, 12, qs.astype(np.int32), tau=tau)
        assert np.array_equal(ei, bf)
        assert np.array_equal(bits(ek), bits(bk))


def test_exact_knn_device_pointers_and_errors():
    torch = pytest.importorskip("torch")
    P = synth.dirichlet(17, 2000, 7, np.float32)
    qs = synth.subsample(5, 2000, 64).astype(np.int32)
    hi, hk = knnd.knnd_exact_knn(P, 7, 10, qs)
    di, dk = knnd.knnd_exact_knn(torch.from_numpy(P).cuda(), 7, 10, torch.from_numpy(qs).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(hi, di.cpu().numpy())
    assert np.array_equal(bits(hk), bits(dk.cpu().numpy()))
    with pytest.raises(knnd.KnndError) as e:  # a bound below the K-th key
        knnd.knnd_exact_knn(P, 7, 10, qs, tau=np.full(qs.size, -1.0))
    assert e.value.status == knnd.KNND_ERR_ARG
    with pytest.raises(knnd.KnndError) as e:  # query out of range
        knnd.knnd_exact_knn(P, 7, 10, np.array([3, 2000], dtype=np.int32))
    assert e.value.status == knnd.KNND_ERR_ARG


# ---------------------------------------------------------------------------
# Batched instances (knnd_build_batched): each instance must come out exactly
# as the oracle's descent of that instance alone.
# ---------------------------------------------------------------------------
def _compare_instance(g, P, d, K, seed, what, stop_rule=0, delta=0.0, cmp=0):
    o = oracle.build_graph(P, d, K, seed, stop_rule=stop_rule, delta=delta, cmp=cmp)
    assert g["status"] == o.status, what
    assert g["rounds"] == o.rounds, (what, g["rounds"], o.rounds)
    for r in range(o.rounds + 1):
        s = g["stats"][r]
        assert s["fcr_hits"] == o.hits[r], (what, r)
        if r:
            assert (s["updates"], s["evals_alg"]) == (o.updates[r], o.evals[r]), (what, r, s)
    assert_same_graph(g["idx"], g["kl"], o.idx, o.keys, what)


# (n, d, K, data seed, seed): several K, coordinates that share a padded
# group (d+1 = 13, 14, 16) or not, tiny and uneven n, n = K + 1
BATCH_MIX = [(900, 12, 8, 11, 21), (2500, 13, 8, 12, 22), (1300, 15, 8, 13, 23), (33, 3, 8, 14, 24),
             (4000, 5, 16, 15, 25), (17, 2, 16, 16, 26), (3100, 20, 16, 17, 27), (700, 7, 4, 18, 28),
             (5000, 9, 32, 19, 29), (64, 30, 32, 20, 30), (1200, 1, 2, 21, 31), (6000, 19, 16, 22, 32)]


@pytest.mark.parametrize("prec,flags", [(knnd.KNND_PREC_FP64, 0), (knnd.KNND_PREC_MIXED_BF16, 0),
                                        (knnd.KNND_PREC_FP64, knnd.KNND_FLAG_PULL)], ids=["plain", "bf16", "pull"])
def test_batched_mix_vs_oracle(prec, flags):
    inst = [(synth.dirichlet(ds, n, d, np.float32), d, K, s) for n, d, K, ds, s in BATCH_MIX]
    say(f"batched: {len(inst)} instances, precision {prec}, flags {flags}")
    st, outs = knnd.knnd_build_batched(inst, knnd.default_params(precision=prec, flags=flags))
    assert st == knnd.KNND_OK
    for (P, d, K, s), g in zip(inst, outs):
        _compare_instance(g, P, d, K, s, f"instance n={P.shape[0]} d={d} K={K}")


# Rounds replayed from captured graphs (the default) against the same rounds
# enqueued kernel by kernel: every instance identical, bit for bit.  Groups
# of this mix stop at different rounds, so the graphs are captured again
# while the call runs.
@pytest.mark.parametrize("prec", [knnd.KNND_PREC_FP64, knnd.KNND_PREC_MIXED_BF16], ids=["plain", "bf16"])
def test_batched_graph_replay_matches_eager(prec):
    inst = [(synth.dirichlet(ds, n, d, np.float32), d, K, s) for n, d, K, ds, s in BATCH_MIX]
    say(f"batched: graph replay vs eager, precision {prec}")
    st1, a = knnd.knnd_build_batched(inst, knnd.default_params(precision=prec))
    st2, b = knnd.knnd_build_batched(inst, knnd.default_params(precision=prec, flags=knnd.KNND_FLAG_NO_GRAPH))
    assert st1 == st2 == knnd.KNND_OK
    assert max(g["rounds"] for g in a) >= 4
    for x, y in zip(a, b):
        assert (x["status"], x["rounds"]) == (y["status"], y["rounds"])
        for sx, sy in zip(x["stats"], y["stats"]):
            for f in ("updates", "fcr_hits", "evals_alg", "evals_performed", "rescues"):
                assert sx[f] == sy[f], f
        assert np.array_equal(x["idx"], y["idx"])
        assert np.array_equal(bits(x["kl"]), bits(y["kl"]))


# The autotuner: under KNND_PREC_AUTO each group's join runs the exact or the
# BF16 mixed form, whichever its first-round trials measured faster (the
# exact form on either hub kernel); every choice gives the oracle's result.
# Its choices are appended to the file KNND_TUNE_CACHE names.
def test_batched_autotuned_vs_oracle(tmp_path, monkeypatch):
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("KNND_TUNE_CACHE", str(path))
    inst = [(synth.dirichlet(ds, n, d, np.float32), d, K, s) for n, d, K, ds, s in BATCH_MIX]
    say("batched: autotuned precision and hub kernel")
    st, outs = knnd.knnd_build_batched(inst, knnd.default_params(precision=knnd.KNND_PREC_AUTO))
    assert st == knnd.KNND_OK
    for (P, d, K, s), g in zip(inst, outs):
        _compare_instance(g, P, d, K, s, f"instance n={P.shape[0]} d={d} K={K}")
    lines = [ln for ln in path.read_text().splitlines() if "prec=3" in ln and "batched=1" in ln]
    assert lines, "no tuned shape recorded"
    for ln in lines:
        key, choice, trials = (x.strip() for x in ln.split("|"))
        mixed, lds, hpw, rwave, opt = (int(v) for v in choice.split())
        assert len(trials.split()) >= 2 and not (mixed and lds) and hpw in (1, 2, 4) and rwave in (0, 1, 2)
        assert opt in (0, 1)
    # a second call reuses the cached choices (no trials) and gives the same result
    st2, again = knnd.knnd_build_batched(inst, knnd.default_params(precision=knnd.KNND_PREC_AUTO))
    assert st2 == st
    for a, b in zip(outs, again):
        assert np.array_equal(a["idx"], b["idx"]) and np.array_equal(bits(a["kl"]), bits(b["kl"]))


# Every schedule the tuner can pick gives the oracle's result (forced one at
# a time; a schedule that is not a candidate for a group leaves it tuned).
@pytest.mark.parametrize("force", ["0 0 1 0 0", "0 0 2 0 1", "0 0 4 1 0", "0 1 1 2 1", "1 0 1 0 0", "1 0 1 0 1"],
                         ids=["reg", "reg_hpw2_opt", "reg_hpw4_wave1", "lds_wave2_opt", "mixed", "mixed_opt"])
def test_batched_forced_schedules_vs_oracle(force, monkeypatch):
    monkeypatch.setenv("KNND_TUNE_FORCE", force)
    inst = [(synth.dirichlet(ds, n, d, np.float32), d, K, s) for n, d, K, ds, s in BATCH_MIX]
    say(f"batched: forced schedule {force}")
    st, outs = knnd.knnd_build_batched(inst, knnd.default_params(precision=knnd.KNND_PREC_AUTO))
    assert st == knnd.KNND_OK
    for (P, d, K, s), g in zip(inst, outs):
        _compare_instance(g, P, d, K, s, f"instance n={P.shape[0]} d={d} K={K}")


# Single descents under forced schedules with one wave per small receiver
# (small K fills the 512- and 1024-slot classes), and the fixed-point rule so
# that late rounds carry unchanged receivers over as well.
@pytest.mark.parametrize("force", ["0 0 1 2 0", "0 0 4 1 1", "0 0 2 2 0"],
                         ids=["wave2", "hpw4_wave1_opt", "hpw2_wave2"])
@pytest.mark.parametrize("n,d,K,ds,seed", [(5000, 4, 8, 9, 3), (20000, 10, 10, 6, 8), (777, 2, 5, 4, 4)])
def test_single_forced_wave_receivers_vs_oracle(n, d, K, ds, seed, force, monkeypatch):
    monkeypatch.setenv("KNND_TUNE_FORCE", force)
    P = synth.dirichlet(ds, n, d, np.float32)
    full_compare(P, d, K, seed, precision=knnd.KNND_PREC_AUTO)
    full_compare(P, d, K, seed, precision=knnd.KNND_PREC_AUTO, stop_rule=knnd.KNND_STOP_FIXED_POINT)


# Guarded 4096-slot tables: at K = 32 most receivers exceed the exact bound
# of that table (T just above 2048) and, optimistically sized, fit it; those
# that do not are redone in the 8192-slot class (round 1 lists every
# distinct candidate, so some overflow the list).
@pytest.mark.parametrize("force", ["0 0 1 0 1", "1 0 1 0 1"], ids=["exact_opt", "mixed_opt"])
def test_single_forced_guarded_4096_vs_oracle(force, monkeypatch):
    monkeypatch.setenv("KNND_TUNE_FORCE", force)
    P = synth.dirichlet(31, 20000, 10, np.float32)
    full_compare(P, 10, 32, 9, precision=knnd.KNND_PREC_AUTO)
    P = synth.dirichlet(32, 3001, 20, np.float32)
    full_compare(P, 20, 30, 7, precision=knnd.KNND_PREC_AUTO)


@pytest.mark.parametrize("n,d,K,ds,seed", [(3001, 20, 30, 5, 7), (20000, 10, 20, 6, 8)])
def test_single_autotuned_vs_oracle(n, d, K, ds, seed):
    P = synth.dirichlet(ds, n, d, np.float32)
    full_compare(P, d, K, seed, precision=knnd.KNND_PREC_AUTO)


# Other stop rules (Section 1.2, Table 1, and Section 1.3, item (b)): same rounds, another
# stopping round; each instance stops on its own n.
@pytest.mark.parametrize("rule,delta", [(knnd.KNND_STOP_FIXED_POINT, 0.0), (knnd.KNND_STOP_DELTA, 0.002)],
                         ids=["fixed_point", "delta"])
def test_batched_stop_rules_vs_oracle(rule, delta):
    inst = [(synth.dirichlet(ds, n, d, np.float32), d, K, s) for n, d, K, ds, s in BATCH_MIX]
    say(f"batched: stop rule {rule} delta {delta}")
    st, outs = knnd.knnd_build_batched(inst, knnd.default_params(precision=knnd.KNND_PREC_MIXED_BF16,
                                                                 stop_rule=rule, delta=delta))
    assert st == knnd.KNND_OK
    for (P, d, K, s), g in zip(inst, outs):
        _compare_instance(g, P, d, K, s, f"instance n={P.shape[0]} d={d} K={K}", rule, delta)


def test_batched_device_pointers_match_host():
    torch = pytest.importorskip("torch")
    inst = [(synth.dirichlet(ds, n, d, np.float32), d, K, s) for n, d, K, ds, s in BATCH_MIX[:6]]
    say("batched: device pointers")
    _, host = knnd.knnd_build_batched(inst)
    dev_inst = [(torch.from_numpy(P).cuda(), d, K, s) for P, d, K, s in inst]
    st, dev = knnd.knnd_build_batched(dev_inst)
    torch.cuda.synchronize()
    assert st == knnd.KNND_OK
    for h, g in zip(host, dev):
        assert h["rounds"] == g["rounds"]
        assert np.array_equal(h["idx"], g["idx"].cpu().numpy())
        assert np.array_equal(h["kl"].view(np.uint64), g["kl"].cpu().numpy().view(np.uint64))


def test_batched_round_cap_stops_every_instance():
    inst = [(synth.dirichlet(ds, n, d, np.float32), d, K, s) for n, d, K, ds, s in BATCH_MIX[:5]]
    st, outs = knnd.knnd_build_batched(inst, knnd.default_params(max_rounds=1))
    assert st in (knnd.KNND_OK, knnd.KNND_WARN_MAX_ROUNDS)
    for (P, d, K, s), g in zip(inst, outs):
        o = oracle.build_graph(P, d, K, s, max_rounds=1)
        assert g["rounds"] == 1 and g["status"] == o.status
        assert_same_graph(g["idx"], g["kl"], o.idx, o.keys, "capped instance")


@pytest.mark.parametrize("prec", [knnd.KNND_PREC_FP64, knnd.KNND_PREC_MIXED_BF16], ids=["plain", "bf16"])
def test_512_instances_batched_full_size(prec):
    gold = _golden(synth.BATCH_WORKLOAD)["instances"]
    inst = []
    for b in range(synth.BATCH_INSTANCES):
        n, d, K, ds, s = synth.instance(synth.BATCH_BASE_SEED, b)
        inst.append((synth.dirichlet(ds, n, d, np.float32), d, K, s))
    say(f"512 instances: {len(inst)} instances vs stored oracle digests, precision {prec}")
    st, outs = knnd.knnd_build_batched(inst, knnd.default_params(precision=prec))
    assert st == knnd.KNND_OK
    for b, (g, o) in enumerate(zip(outs, gold)):
        assert (g["status"], g["rounds"]) == (o["status"], o["rounds"]), b
        assert [s["updates"] for s in g["stats"][1:]] == o["updates"][1:], b
        assert [s["fcr_hits"] for s in g["stats"]] == o["fcr_hits"], b
        assert [s["evals_alg"] for s in g["stats"][1:]] == o["evals_alg"][1:], b
        assert _digest(g["idx"]) == o["idx_sha256"], b
        assert _digest(g["kl"]) == o["kl_sha256"], b


# ---------------------------------------------------------------------------
# The paper's printed statistics (Section 4, Tables 3 and 4), reproduced on
# the GPU path with other random draws: tolerance bands, not equality.
# ---------------------------------------------------------------------------
def test_paper_tables_statistics_on_gpu():
    torch = pytest.importorskip("torch")
    from paper_2202_00517_amd import paper_tables as pt
    t3 = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_table3.json")))["rows"]
    t4 = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_table4.json")))
    for i, p in enumerate(t3):  # n = 2e4, 2e5 and 2e6, 10 coordinates
        r = pt.run_row(p["n"], p["coordinates"], p["K"], 3100 + i, 3200 + i, torch, knnd.KNND_PREC_MIXED_BF16)
        say(f"table 3 row {i}: {r}")
        assert r["rounds"] <= p["round_bound"] and abs(r["rounds"] - p["rounds"]) <= 2
        assert abs(r["fcc"] - p["fcc"]) < 0.05
        assert r["accuracy_2000"] >= 0.85
    acc = {}
    for i, p in enumerate(t4["rows"]):
        r = pt.run_row(t4["n"], p["coordinates"], p["K"], 4100 + i, 4200 + i, torch, knnd.KNND_PREC_MIXED_BF16)
        say(f"table 4 row {i}: {r}")
        assert r["rounds"] <= r["round_bound"]
        assert abs(r["fcc"] - p["fcc"]) < 0.03
        assert abs(r["accuracy_2000"] - p["accuracy"]) < 0.25
        acc[(p["K"], p["coordinates"])] = r["accuracy_2000"]
    # accuracy declines with dimension, and K = 64 is more accurate than K = 16
    for K in (16, 64):
        assert acc[(K, 10)] > acc[(K, 40)] and acc[(K, 20)] > acc[(K, 60)]
    for c in (10, 20, 40, 60):
        assert acc[(64, c)] > acc[(16, c)]


# ---------------------------------------------------------------------------
# Other comparators (Section 2.1: any family of per-point total orders):
# reverse KL, Hellinger and Euclidean keys, bit for bit against the oracle.
# ---------------------------------------------------------------------------
CMPS = [knnd.KNND_CMP_KL_REVERSE, knnd.KNND_CMP_HELLINGER, knnd.KNND_CMP_L2]
CMP_IDS = ["reverse_kl", "hellinger", "l2"]


def _gauss(seed, n, D, dtype=np.float32):
    """Seeded standard normal points (any sign): inputs for the Euclidean comparator."""
    return np.random.default_rng(seed).standard_normal((n, D)).astype(dtype)


def test_feature_tables_bit_exact():
    # square roots (Hellinger) over many binades, zeros and subnormals; the
    # identity table (Euclidean) on values of any sign
    rng = np.random.default_rng(3)
    vals = np.concatenate([np.array([0.0, 1.0, 4.0, 2.0, 0.5, 5e-324, 1e-310, 2.0 ** -1022, 1e300,
                                     np.nextafter(1.0, 2.0), np.nextafter(1.0, 0.0)]),
                           np.ldexp(rng.uniform(0.5, 1.0, 20000), rng.integers(-1074, 1000, 20000)),
                           rng.uniform(0.0, 1.0, 4000)])
    D = 8
    vals = vals[: (vals.size // D) * D].reshape(-1, D)
    say(f"sqrt table of {vals.size} values")
    prm = knnd.default_params(comparator=knnd.KNND_CMP_HELLINGER)
    with knnd.Context(vals, D - 1, 2, 1, prm) as c:
        L = c.log_table()
    assert np.array_equal(bits(L), bits(np.sqrt(vals)))
    G = _gauss(4, 500, D, np.float64)
    prm = knnd.default_params(comparator=knnd.KNND_CMP_L2)
    with knnd.Context(G, D - 1, 2, 1, prm) as c:
        L = c.log_table()
    assert np.array_equal(bits(L), bits(G))


@pytest.mark.parametrize("cmp", CMPS, ids=CMP_IDS)
@pytest.mark.parametrize("n,d,K,dtype", [(2000, 5, 10, np.float64), (5000, 10, 20, np.float32),
                                         (65, 3, 64, np.float32)])
def test_comparator_initial_graph_bit_exact(n, d, K, dtype, cmp):
    P = synth.dirichlet(600 + n, n, d, dtype)
    seed = 910 + n
    prm = knnd.default_params(comparator=cmp)
    with knnd.Context(P, d, K, seed, prm) as c:
        c.init_graph()
        gi, gk = c.get_graph()
    P64 = oracle.widen(P)
    L = oracle.log_table(P64)
    oi, ok = oracle.initial_graph(P64, L, K, seed, cmp=cmp)
    assert_same_graph(gi, gk, oi, ok, "initial graph")


@pytest.mark.parametrize("form", FORMS[:3], ids=FORM_IDS[:3])
@pytest.mark.parametrize("cmp", CMPS, ids=CMP_IDS)
@pytest.mark.parametrize("n,d,K", [(3001, 20, 30), (1000, 6, 16), (700, 70, 8), (200, 1, 2)])
def test_comparator_one_round_bit_exact(n, d, K, cmp, form):
    P = synth.dirichlet(700 + n + d, n, d, np.float32)
    one_round(P, d, K, 33 + n, flags=form[0], precision=form[1], cmp=cmp)


@pytest.mark.parametrize("form", FORMS[:3], ids=FORM_IDS[:3])
@pytest.mark.parametrize("cmp", CMPS, ids=CMP_IDS)
@pytest.mark.parametrize("n,d,K,ds,seed", [(3001, 20, 30, 5, 7), (20000, 10, 20, 6, 8),
                                           (2500, 80, 12, 10, 4)])
def test_comparator_full(n, d, K, ds, seed, cmp, form):
    P = synth.dirichlet(ds, n, d, np.float32)
    g, o = full_compare(P, d, K, seed, flags=form[0], precision=form[1], cmp=cmp)
    assert g["stats"][1]["rescues"] == 0  # no mixed form for these keys


@pytest.mark.parametrize("form", FORMS[:2], ids=FORM_IDS[:2])
def test_euclidean_on_points_of_any_sign(form):
    G = _gauss(5, 6000, 12)
    full_compare(G, 11, 16, 17, flags=form[0], cmp=knnd.KNND_CMP_L2,
                 stop_rule=knnd.KNND_STOP_FIXED_POINT)


def test_comparator_domains():
    P = synth.dirichlet(8, 300, 4, np.float32)
    P[7, 2] = 0.0
    for cmp, want in [(knnd.KNND_CMP_KL_REVERSE, knnd.KNND_ERR_DOMAIN), (knnd.KNND_CMP_HELLINGER, knnd.KNND_OK),
                      (knnd.KNND_CMP_L2, knnd.KNND_OK)]:
        prm = knnd.default_params(comparator=cmp)
        if want == knnd.KNND_OK:
            assert knnd.knnd_build_ex(P, 4, 8, 1, prm)["status"] == knnd.KNND_OK
        else:
            with pytest.raises(knnd.KnndError) as e:
                knnd.knnd_build_ex(P, 4, 8, 1, prm)
            assert e.value.status == want
    P[9, 1] = -0.25
    with pytest.raises(knnd.KnndError) as e:
        knnd.knnd_build_ex(P, 4, 8, 1, knnd.default_params(comparator=knnd.KNND_CMP_HELLINGER))
    assert e.value.status == knnd.KNND_ERR_DOMAIN


@pytest.mark.parametrize("cmp", CMPS, ids=CMP_IDS)
def test_batched_comparators_vs_oracle(cmp):
    inst = [(synth.dirichlet(ds, n, d, np.float32), d, K, s) for n, d, K, ds, s in BATCH_MIX]
    say(f"batched: comparator {cmp}")
    st, outs = knnd.knnd_build_batched(inst, knnd.default_params(comparator=cmp))
    assert st == knnd.KNND_OK
    for (P, d, K, s), g in zip(inst, outs):
        _compare_instance(g, P, d, K, s, f"instance n={P.shape[0]} d={d} K={K}", cmp=cmp)


@pytest.mark.parametrize("cmp", CMPS, ids=CMP_IDS)
@pytest.mark.parametrize("n,d,K,dtype", [(5000, 9, 16, np.float32), (3001, 20, 30, np.float64),
                                         (1500, 100, 8, np.float32)])
def test_comparator_exact_knn_matches_oracle(n, d, K, dtype, cmp):
    P = synth.dirichlet(800 + n, n, d, dtype)
    qs = synth.subsample(77, n, 300).astype(np.int32)
    say(f"exact knn n={n} d={d} K={K} cmp={cmp}")
    ei, ek = knnd.knnd_exact_knn(P, d, K, qs, comparator=cmp)
    P64 = oracle.widen(P)
    oi, ok = oracle.bruteforce(P64, oracle.log_table(P64), K, qs.astype(np.int64), cmp=cmp)
    assert_same_graph(ei, ek, oi, ok, "exact knn")


# ---------------------------------------------------------------------------
# Device memory cache: reused blocks hold stale data from earlier calls;
# results must not depend on it.
# ---------------------------------------------------------------------------
def test_memory_cache_reuse_and_release():
    P = synth.dirichlet(31, 20000, 10, np.float32)
    Q = synth.dirichlet(32, 20000, 10, np.float32)
    prm = knnd.default_params(precision=knnd.KNND_PREC_MIXED_BF16)
    say("cache: build P, build Q (reusing P's blocks), release, build P again")
    a = knnd.knnd_build_ex(P, 10, 20, 5, prm)
    b = knnd.knnd_build_ex(Q, 10, 20, 5, prm)
    assert knnd.release_cache() == knnd.KNND_OK
    c = knnd.knnd_build_ex(P, 10, 20, 5, prm)
    o = oracle.build_graph(Q, 10, 20, 5)
    assert_same_graph(b["idx"], b["kl"], o.idx, o.keys, "second build")
    assert np.array_equal(a["idx"], c["idx"]) and np.array_equal(bits(a["kl"]), bits(c["kl"]))
    # a smaller build then a larger one on reused blocks
    d = knnd.knnd_build_ex(P[:5000], 10, 20, 5, prm)
    e = knnd.knnd_build_ex(P, 10, 20, 5, prm)
    o = oracle.build_graph(P[:5000], 10, 20, 5)
    assert_same_graph(d["idx"], d["kl"], o.idx, o.keys, "small build")
    assert np.array_equal(a["idx"], e["idx"])


# ---------------------------------------------------------------------------
# Dimension boundaries: the MFMA operand width (32 or 64 coordinates; above 64
# the exact hub form runs) and the LDS limit of the hub form ((K+1) rows of
# D doubles over 64 KB: the pull form runs).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", MIXED, ids=["bf16", "fp16"])
@pytest.mark.parametrize("d", [31, 32, 63, 64])
def test_mixed_at_operand_width_boundaries(d, prec):
    P = synth.dirichlet(900 + d, 3000, d, np.float32)
    g, _ = full_compare(P, d, 16, 41 + d, precision=prec)
    if d + 1 > 64:
        assert sum(s["rescues"] for s in g["stats"]) == 0  # exact hub form


def test_high_dimension_runs_the_pull_form():
    d, K = 200, 40  # (K+1) * 201 * 8 bytes > 64 KB
    P = synth.dirichlet(905, 1500, d, np.float32)
    full_compare(P, d, K, 43, precision=knnd.KNND_PREC_MIXED_BF16)


@pytest.mark.parametrize("prec", MIXED, ids=["bf16", "fp16"])
def test_mixed_near_duplicates_resolved_by_rescue(prec):
    # clusters of near-duplicates: keys inside a cluster differ far below the
    # 16-bit operands' resolution, so only the FP64 rescue orders them
    base = synth.dirichlet(910, 400, 9, np.float64)
    rng = np.random.default_rng(911)
    P = np.repeat(base, 8, axis=0) * (1.0 + 1e-7 * rng.standard_normal((3200, 10)))
    P = (P / P.sum(axis=1, keepdims=True)).astype(np.float32)
    g, _ = full_compare(P, 9, 12, 47, precision=prec)
    assert sum(s["rescues"] for s in g["stats"]) > 0


@pytest.mark.parametrize("prec", [knnd.KNND_PREC_MIXED_BF16, knnd.KNND_PREC_MIXED_FP16], ids=["bf16", "fp16"])
def test_mixed_large_rescue_sets(prec):
    # two clusters of 1200 near-duplicates at K = 30: in round 1 a receiver
    # lists the hundreds of candidates from its own cluster, whose key
    # intervals all contain the K-th bound, so its rescue set exceeds the
    # fast path's 256 and the keys are formed in the block's final merge
    base = synth.dirichlet(912, 2, 9, np.float64)
    rng = np.random.default_rng(913)
    P = np.repeat(base, 1200, axis=0) * (1.0 + 1e-6 * rng.standard_normal((2400, 10)))
    P = (P / P.sum(axis=1, keepdims=True)).astype(np.float32)
    g, _ = full_compare(P, 9, 30, 48, precision=prec)
    # more than 256 rescues per receiver on average in some round: at least
    # one receiver took the large-rescue path
    assert max(s["rescues"] for s in g["stats"]) > 256 * 2400
