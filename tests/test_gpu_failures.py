"""Failure injection on the GPU: each device allocation of a call is made to
fail in turn (knnd_test_fail_alloc).  A buffer the method needs ends the call
with KNND_ERR_NOMEM; an optional one (the hub and mixed forms' buffers, the
neighbourhood-tracking flags) makes it run another form with the same lists,
keys and counts.  Either way every device block goes back to the library's
cache (no live blocks once the call has returned)."""
import numpy as np
import pytest

import paper_2202_00517_amd as knnd
import synth

pytestmark = pytest.mark.gpu

MAX_ALLOCS = 400  # (a batched call of three groups makes about 150)


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    knnd.inject_alloc_failure(0)


def bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


def _sweep(call, check, what):
    """Run call() with the k-th allocation failing, k = 1, 2, ... until a call
    no longer reaches the armed failure; check every successful result."""
    outcomes = []
    base, _ = knnd.memory_stats()  # (contexts other tests left alive)
    for k in range(1, MAX_ALLOCS + 1):
        knnd.inject_alloc_failure(k)
        try:
            res, st = call(), knnd.KNND_OK
        except knnd.KnndError as e:
            res, st = None, e.status
        left = knnd.inject_alloc_failure(0)
        live, _ = knnd.memory_stats()
        assert live == base, f"{what}: {live - base} bytes still in use after a failure at allocation {k}"
        if left > 0:  # fewer than k allocations: the failure never fired
            assert st == knnd.KNND_OK, (what, k, st)
            check(res)
            say(f"{what}: {k - 1} allocations, outcomes {sorted(set(outcomes))}")
            return outcomes
        assert st in (knnd.KNND_OK, knnd.KNND_ERR_NOMEM), (what, k, st)
        if st == knnd.KNND_OK:
            check(res)
        outcomes.append(st)
    pytest.fail(f"{what}: more than {MAX_ALLOCS} allocations")


def _same_descent(ref):
    def check(g):
        assert g["rounds"] == ref["rounds"]
        assert np.array_equal(np.asarray(g["idx"]), np.asarray(ref["idx"]))
        assert np.array_equal(bits(np.asarray(g["kl"])), bits(np.asarray(ref["kl"])))
        for a, b in zip(g["stats"], ref["stats"]):
            assert (a["updates"], a["evals_alg"], a["fcr_hits"]) == (b["updates"], b["evals_alg"], b["fcr_hits"])
    return check


@pytest.mark.parametrize("form", [(0, knnd.KNND_PREC_FP64), (0, knnd.KNND_PREC_MIXED_BF16),
                                  (0, knnd.KNND_PREC_AUTO), (knnd.KNND_FLAG_PULL, knnd.KNND_PREC_FP64),
                                  (knnd.KNND_FLAG_ATOMIC_CSR, knnd.KNND_PREC_MIXED_FP16)],
                         ids=["hub", "bf16", "auto", "pull", "atomic_fp16"])
@pytest.mark.parametrize("device", [False, True], ids=["host", "device"])
def test_single_descent_allocation_failures(form, device):
    import torch
    P = synth.dirichlet(71, 3001, 20, np.float32)
    pts = torch.from_numpy(P).cuda() if device else P
    prm = lambda: knnd.default_params(flags=form[0], precision=form[1])
    ref = knnd.knnd_build_ex(pts, 20, 30, 7, prm())
    ref = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in ref.items()}

    def call():
        g = knnd.knnd_build_ex(pts, 20, 30, 7, prm())
        return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in g.items()}

    out = _sweep(call, _same_descent(ref), f"single descent {form} device={device}")
    assert knnd.KNND_ERR_NOMEM in out  # the required buffers fail cleanly
    if form[0] != knnd.KNND_FLAG_PULL:
        assert knnd.KNND_OK in out  # an optional buffer's failure falls back to another form


def test_batched_allocation_failures():
    inst = [(synth.dirichlet(ds, n, d, np.float32), d, K, s)
            for n, d, K, ds, s in [(900, 12, 8, 11, 21), (4000, 5, 16, 15, 25), (1500, 9, 32, 19, 29)]]
    prm = lambda: knnd.default_params(precision=knnd.KNND_PREC_AUTO)
    st, ref = knnd.knnd_build_batched(inst, prm())
    assert st == knnd.KNND_OK

    def call():
        s, outs = knnd.knnd_build_batched(inst, prm())
        assert s == knnd.KNND_OK
        return outs

    def check(outs):
        for a, b in zip(outs, ref):
            _same_descent(b)(a)

    out = _sweep(call, check, "batched")
    assert knnd.KNND_ERR_NOMEM in out


def test_context_and_exact_search_allocation_failures():
    P = synth.dirichlet(72, 2500, 9, np.float32)
    qs = synth.subsample(5, 2500, 200).astype(np.int32)
    ref_i, ref_k = knnd.knnd_exact_knn(P, 9, 12, qs)

    def exact():
        return knnd.knnd_exact_knn(P, 9, 12, qs)

    def check_exact(r):
        assert np.array_equal(r[0], ref_i) and np.array_equal(bits(r[1]), bits(ref_k))

    assert knnd.KNND_ERR_NOMEM in _sweep(exact, check_exact, "exact search")

    with knnd.Context(P, 9, 12, 3, knnd.default_params(precision=knnd.KNND_PREC_MIXED_BF16)) as c:
        c.init_graph()
        want = [c.round() for _ in range(3)]
        wi, wk = c.get_graph()

    def steps():
        with knnd.Context(P, 9, 12, 3, knnd.default_params(precision=knnd.KNND_PREC_MIXED_BF16)) as c:
            c.init_graph()
            got = [c.round() for _ in range(3)]
            gi, gk = c.get_graph()
        return got, gi, gk

    def check_steps(r):
        got, gi, gk = r
        assert [(s["updates"], s["evals_alg"]) for s in got] == [(s["updates"], s["evals_alg"]) for s in want]
        assert np.array_equal(gi, wi) and np.array_equal(bits(gk), bits(wk))

    assert knnd.KNND_ERR_NOMEM in _sweep(steps, check_steps, "step interface")
