"""knnd_build_noalloc (every device buffer in the library's fixed scratch
array) against knnd_build_ex on the same inputs, through the C ABI: lists and
key bits identical, every per-round count equal; two calls in a row on one
device (the second on a smaller input, so it runs on the contents the first
left in the scratch array), in the hub, mixed and pull forms; and an input
too large for the array is refused before any device work."""
import ctypes

import numpy as np
import pytest

import paper_2202_00517_amd as knnd
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def _bits(t):
    return t.cpu().numpy().view(np.uint64)


def _compare(P, d, K, seed, params):
    import torch
    Pd = torch.from_numpy(P).cuda()
    print(f"noalloc n={P.shape[0]} d={d} K={K} seed={seed} precision={params.precision} "
          f"flags={params.flags}", flush=True)
    a = knnd.knnd_build_ex(Pd, d, K, seed, params)
    b = knnd.knnd_build_noalloc(Pd, d, K, seed, params)
    torch.cuda.synchronize()
    assert a["status"] == b["status"] == knnd.KNND_OK
    assert a["rounds"] == b["rounds"]
    for r in range(a["rounds"] + 1):
        sa, sb = a["stats"][r], b["stats"][r]
        for f in ("updates", "fcr_hits", "evals_alg", "carried", "evals_carried"):
            assert sa[f] == sb[f], (r, f, sa[f], sb[f])
    assert torch.equal(a["idx"], b["idx"])
    assert np.array_equal(_bits(a["kl"]), _bits(b["kl"]))
    return b


@pytest.mark.parametrize("prec,flags", [(knnd.KNND_PREC_FP64, 0), (knnd.KNND_PREC_MIXED_BF16, 0),
                                        (knnd.KNND_PREC_FP64, knnd.KNND_FLAG_PULL)],
                         ids=["hub", "bf16", "pull"])
def test_noalloc_matches_build_ex_twice(prec, flags):
    P1 = synth.dirichlet(41, 8000, 10, np.float32)
    P2 = synth.dirichlet(42, 3000, 6, np.float32)
    _compare(P1, 10, 16, 7, knnd.default_params(precision=prec, flags=flags))
    _compare(P2, 6, 12, 8, knnd.default_params(precision=prec, flags=flags))


def test_noalloc_fixed_point_with_carry_over():
    # a long descent: the carry-over of unchanged neighbourhoods allocates its
    # flags from the scratch array too
    P = synth.dirichlet(9, 5000, 4, np.float32)
    b = _compare(P, 4, 8, 3, knnd.default_params(stop_rule=knnd.KNND_STOP_FIXED_POINT))
    assert max(s["carried"] for s in b["stats"]) > 0


def test_noalloc_refuses_inputs_beyond_the_scratch_array():
    import torch
    n, d, K = 400_000, 20, 30  # about 1 GB of buffers in the smallest form
    P = torch.full((n, d + 1), 1.0 / (d + 1), dtype=torch.float32, device="cuda")
    idx = torch.empty((n, K), dtype=torch.int32, device="cuda")
    p = knnd.default_params()
    r = ctypes.c_int32(-7)
    st = knnd.lib().knnd_build_noalloc(P.data_ptr(), n, d, K, 1, ctypes.byref(p),
                                       torch.cuda.current_stream().cuda_stream, idx.data_ptr(),
                                       None, None, ctypes.byref(r))
    assert st == knnd.KNND_ERR_NOMEM
    assert r.value == -7
