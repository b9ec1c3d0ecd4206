"""Benchmark: comparator evaluations per second and time-to-graph of
comparator-based K-NN descent with the KL comparator, n=1e6 points of the
20-simplex (21 FP32 coordinates), K=30, on one MI355X.

One step = one whole descent through the C ABI (knnd_build_ex) on points
already resident in HBM: validation and log table, random K-out start, every
round (reverse neighbors, candidate join, KL keys, merge, FCR sample) until
the stop test fires, lists copied to the caller's device buffer.

value = sum over rounds of evals_alg (one KL key per receiver and distinct
non-friend candidate, the oracle's count) / time-to-graph.

The default precision is mixed (BF16 MFMA screen with FP64 rescue, bit-exact
output); the plain FP64 descent of the same workload is timed beside it and
reported under "plain" so the line carries both sides of the comparison.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision mixed|plain]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "comparator evals/sec + time-to-graph (n=1e6,d=20,K=30), mixed vs plain"
HBM_PEAK_GBS = 8000.0
MFMA_16BIT_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 / FP16 matrix peak
FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector peak


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_recv_c3.json")
KERNEL_SOURCES = ["paper_2202_00517_amd/csrc/knnd_kernels.hip", "paper_2202_00517_amd/csrc/knnd_device.h"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(precision):
    """HBM bytes per receiver pass from the rocprofv3 FETCH_SIZE / WRITE_SIZE
    runs recorded under profiles/, or None when the kernel sources changed
    since those counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    if rec.get("source_sha256") != kernel_source_digest():
        return None
    return rec.get("bytes_per_launch", {}).get(precision)


def read_tuner_file(path):
    """The join schedules the library's tuner chose (one line per workload
    shape: the shape, the choice, the measured milliseconds of each
    candidate's first-round join)."""
    out = []
    try:
        with open(path) as f:
            for line in f:
                parts = [x.strip() for x in line.split("|")]
                if len(parts) == 3:
                    out.append({"shape": parts[0], "choice": parts[1], "trials_ms": parts[2]})
    except OSError:
        pass
    return out


def batched_leg(knnd, synth, torch, steps):
    """The batched workload (512 instances of uneven n, d, K) as one batched
    call (rounds after the third replayed from captured graphs, each group a
    branch of its own; join schedules chosen by the library's tuner on the
    warm-up call) with the tuner also choosing each group's precision form
    (KNND_PREC_AUTO: exact FP64 or split BF16 with FP64 rescue, the same
    lists either way); device-resident points.  Also timed: the exact form
    throughout, the same with rounds enqueued kernel by kernel (no graphs),
    and the instances one by one through knnd_build_ex."""
    import tempfile
    tune_file = os.path.join(tempfile.mkdtemp(prefix="knnd_tune_"), "tune.txt")
    os.environ["KNND_TUNE_CACHE"] = tune_file
    inst = []
    for b in range(synth.BATCH_INSTANCES):
        n, d, K, ds, s = synth.instance(synth.BATCH_BASE_SEED, b)
        inst.append((torch.from_numpy(synth.dirichlet(ds, n, d, np.float32)).cuda(), d, K, s))

    def timed_calls(prm, reps):
        knnd.knnd_build_batched(inst, prm)  # warm-up (tunes on first use of a shape)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            _, outs = knnd.knnd_build_batched(inst, prm)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps, outs

    prm = knnd.default_params(precision=knnd.KNND_PREC_FP64)
    batched_s, outs = timed_calls(prm, steps)
    auto_s, outs_auto = timed_calls(knnd.default_params(precision=knnd.KNND_PREC_AUTO), steps)
    eager_s, _ = timed_calls(knnd.default_params(precision=knnd.KNND_PREC_FP64, flags=knnd.KNND_FLAG_NO_GRAPH),
                             max(1, steps // 2))
    evals = sum(s["evals_alg"] for o in outs for s in o["stats"])
    t = time.perf_counter()
    ev1 = 0
    for P, d, K, s in inst:
        o = knnd.knnd_build_ex(P, d, K, s, prm)
        ev1 += sum(x["evals_alg"] for x in o["stats"])
    torch.cuda.synchronize()
    single_s = time.perf_counter() - t
    assert ev1 == evals, "batched and one-by-one evaluation counts differ"
    for a, b in zip(outs, outs_auto):  # the tuned precision form gives the same lists
        assert np.array_equal(a["idx"].cpu().numpy(), b["idx"].cpu().numpy()), "tuned form differs"
    return {"workload": f"{len(inst)} instances, n in [500, 20000], d+1 in [4, 21], K in {{8,16,32}}, "
                        f"base seed {synth.BATCH_BASE_SEED}, {sum(p.shape[0] for p, *_ in inst)} points",
            "batched_ms": round(1e3 * auto_s, 2), "value": evals / auto_s, "unit": "evals/s",
            "form": "precision form and join schedules per group chosen by the library's tuner",
            "exact_form_ms": round(1e3 * batched_s, 2), "no_graph_ms": round(1e3 * eager_s, 2),
            "one_by_one_ms": round(1e3 * single_s, 2),
            "speedup_exact_over_one_by_one": round(single_s / batched_s, 3),
            "evals_alg": evals, "max_rounds": max(o["rounds"] for o in outs), "tuner": read_tuner_file(tune_file)}


def share_leg(knnd, Pd, d, K, seed, precision, shares=8, reps=3):
    """One GPU's share of a descent split by receivers over `shares` GPUs:
    round 2 (from the graph a full round 1 left) restricted to the first
    1/shares of the receivers, against the same round over all of them.  The
    share builds the reverse lists it reads (edges from or to its receivers)
    and runs every hub, as each GPU would after an all-gather of the lists.
    Device time of
    the round from the library's HIP events; median of `reps`."""
    n = Pd.shape[0]
    prm = knnd.default_params(precision=precision)
    cnt = (n + shares - 1) // shares
    full, part = [], []
    for _ in range(reps):
        for out in (full, part):
            with knnd.Context(Pd, d, K, seed, prm) as c:
                c.init_graph()
                c.round()
                out.append(c.round() if out is full else c.round_share(0, cnt))

    def med(rows, key):
        v = sorted(r[key] for r in rows)
        return round(v[len(v) // 2], 3)

    return {"receivers": f"first 1/{shares} ({cnt} of {n}), round 2",
            "round_ms_full": med(full, "ms"), "round_ms_share": med(part, "ms"),
            "share_over_full": round(med(part, "ms") / med(full, "ms"), 4),
            "hub_ms_full": med(full, "ms_hub"), "hub_ms_share": med(part, "ms_hub"),
            "recv_ms_full": med(full, "ms_recv"), "recv_ms_share": med(part, "ms_recv"),
            "evals_alg_full": full[0]["evals_alg"], "evals_alg_share": part[0]["evals_alg"]}


def copy_calibration():
    """A plain device copy of 1 GiB: the reference for scaling FETCH_SIZE and
    WRITE_SIZE (run under rocprofv3 --pmc)."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    log("copied 1 GiB")


def eval_bytes(D, mixed):
    """Algorithmic bytes of one comparator evaluation (steps a2+a3): the
    gather of the candidate's row, D 16-bit values (mixed) or D FP64 logs
    (plain), plus its 4-byte id."""
    return D * (2 if mixed else 8) + 4


def eval_flops(D, mixed):
    """Algorithmic arithmetic of one evaluation's key: D multiply-adds of the
    cross term on the matrix cores (mixed), or D subtractions and D
    multiply-adds in FP64 (plain)."""
    return 2 * D if mixed else 3 * D


def kernel_rooflines(rounds, D, mixed):
    """Per-kernel achieved fractions of the roofline that bounds each, from
    the per-evaluation units above times the evaluations each round performs
    (evals_alg minus the count carried over unchanged) and the kernels' HIP
    event times summed over the timed rounds."""
    ev = sum(s["evals_alg"] - s.get("evals_carried", 0) for s in rounds)
    recv_s = sum(s["ms_recv"] for s in rounds) * 1e-3
    hub_s = sum(s["ms_hub"] for s in rounds) * 1e-3
    join_s = sum(s["ms_join"] for s in rounds) * 1e-3
    nr = len(rounds)
    byt = ev * eval_bytes(D, mixed)
    fl = ev * eval_flops(D, mixed)

    def hbm(name, secs):
        a = byt / secs / 1e9
        return {"kernel": name, "bound": "hbm", "unit": "GB/s", "per_eval": eval_bytes(D, mixed),
                "achieved": round(a, 2), "peak": HBM_PEAK_GBS, "frac": round(a / HBM_PEAK_GBS, 5),
                "avg_launch_ms": round(1e3 * secs / nr, 3), "work_per_launch": int(byt / nr)}

    peak = MFMA_16BIT_PEAK_TFLOPS if mixed else FP64_PEAK_TFLOPS
    a = fl / hub_s / 1e12
    hub = {"kernel": "k_hub_mfma (split 16-bit cross terms on MFMA)" if mixed else "k_hub_reg (FP64 keys)",
           "bound": "mfma" if mixed else "fp64", "unit": "TFLOP/s", "per_eval": eval_flops(D, mixed),
           "achieved": round(a, 3), "peak": peak, "frac": round(a / peak, 6),
           "avg_launch_ms": round(1e3 * hub_s / nr, 3), "work_per_launch": int(fl / nr)}
    return [hbm("receiver pass: k_recv (every table-size class) + k_merge", recv_s),
            hbm("join: hub kernel + receiver pass", join_s), hub]


def recv_bytes(n, K, D, mixed, rescues, psize=4):
    """Algorithmic HBM bytes of one receiver pass (every size class of
    k_recv, one round), as the kernel's algorithm moves them:
      per receiver  its list ids and keys read (K*12), rowptr pair (16), the
                    new list written (K*12)
      per edge      the co-friend entry (col 4 B + slot 1 B) read twice: as a
                    candidate and as the row of its friends
      per occurrence (n(K + 2K^2) in all: co-friends, friends of friends,
                    friends of co-friends) one 4-byte id for the K^2 + cK row
                    entries and one key slot (8 B FP64 key; 4 B FP32 cross
                    term in the mixed form)
      mixed form    S(x), x's row and logs per receiver, and the candidate's
                    FP64 log row per rescue
    This is the receiver design's own traffic model (reported as
    design_bytes), not the per-evaluation unit of the roofline."""
    s = 4 if mixed else 8
    b = n * (K * 24 + 16) + n * K * (10 + s) + 2 * n * K * K * (4 + s)
    if mixed:
        b += n * (8 + D * (psize + 8)) + rescues * D * 8
    return b


def cpu_baseline(P, d, K, seed, receivers, threads):
    """The oracle's round 1 on a sample of receivers of the same workload."""
    import oracle
    import synth
    P64 = oracle.widen(P)
    L = oracle.log_table(P64, threads)
    F0, k0 = oracle.initial_graph(P64, L, K, seed, threads)
    xs = synth.subsample(seed, P.shape[0], receivers)
    t = time.perf_counter()
    _, _, _, ev = oracle.round_subset(P64, L, F0, k0, xs, threads)
    secs = time.perf_counter() - t
    return {"value": float(ev.sum()) / secs, "unit": "evals/s", "cores": threads,
            "kind": "oracle",
            "sample": f"round 1 of this workload for {receivers} receivers drawn without "
                      f"replacement ({int(ev.sum())} evaluations, {secs:.1f} s, "
                      f"{threads} threads; log table and start graph not timed)"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    """Threads for the CPU oracle: the host's hardware concurrency, capped at
    16 (the CPU share that goes with one GPU on a shared host)."""
    return min(16, os.cpu_count() or 1)


def oracle_descents(names):
    """The CPU oracle (unchanged) timed on whole descents of the named
    workloads, from points in host memory to final lists: per-round seconds
    and evaluations per second, with the host's threads and, for n <= 10000,
    with one thread as well."""
    import oracle
    import synth
    threads = host_threads()
    out = {"kind": "oracle", "cpu": cpu_model(), "hardware_concurrency": os.cpu_count(),
           "threads": threads, "runs": []}
    for name in names:
        cf = synth.WORKLOADS[name]
        P = synth.dirichlet(cf["data_seed"], cf["n"], cf["d"], cf["dtype"])
        for t in ([threads, 1] if cf["n"] <= 10000 else [threads]):
            log(f"oracle: {name}, {t} threads")
            t0 = time.perf_counter()
            r = oracle.build_graph(P, cf["d"], cf["K"], cf["seed"], threads=t)
            secs = time.perf_counter() - t0
            out["runs"].append({"workload": name, "n": cf["n"], "d": cf["d"], "K": cf["K"], "threads": t,
                                "rounds": r.rounds, "seconds": round(secs, 3),
                                "round_seconds": [round(float(s), 3) for s in r.seconds[1:]],
                                "evals_alg": int(r.evals.sum()),
                                "evals_per_s": float(r.evals.sum()) / secs})
    return out


def oracle_timing(names):
    print(json.dumps(oracle_descents(names)), flush=True)


# The other workloads, timed beside the headline one: (name, precision).
CONFIG_LEGS = [("n2000_d5_k10", "plain"), ("n100000_d10_k20", "plain"),
               ("n200000_d50_k20", "mixed_fp16"), ("n200000_d50_k20", "plain")]
RECALL_QUERIES = 2000


def config_leg(knnd, torch, name, precision, reps=5):
    """One workload on the device: time-to-graph (device-resident points,
    median of `reps` after one warm-up), end-to-end time (host points in, host
    lists out; median of 3), evaluations per second and the rescue rate.  For
    the 50-coordinate workload also recall@K against exhaustive search on
    RECALL_QUERIES sampled points."""
    import synth
    cf = synth.WORKLOADS[name]
    n, d, K, seed = cf["n"], cf["d"], cf["K"], cf["seed"]
    P = synth.dirichlet(cf["data_seed"], n, d, cf["dtype"])
    Pd = torch.from_numpy(P).cuda()
    prec = {"plain": knnd.KNND_PREC_FP64, "mixed_bf16": knnd.KNND_PREC_MIXED_BF16,
            "mixed_fp16": knnd.KNND_PREC_MIXED_FP16}[precision]
    stream = torch.cuda.current_stream().cuda_stream

    def run():
        return knnd.knnd_build_ex(Pd, d, K, seed, knnd.default_params(precision=prec), stream=stream)

    out = run()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        t = time.perf_counter()
        out = run()
        torch.cuda.synchronize()
        times.append(1e3 * (time.perf_counter() - t))
    e2e = []
    for _ in range(3):
        t = time.perf_counter()
        knnd.knnd_build_ex(P, d, K, seed, knnd.default_params(precision=prec), with_kl=False)
        e2e.append(1e3 * (time.perf_counter() - t))
    st = out["stats"][1:]
    ev = sum(s["evals_alg"] for s in st)
    evaluated = sum(s["evals_alg"] - s["evals_carried"] for s in st)
    resc = sum(s["rescues"] for s in st)
    ms = sorted(times)[reps // 2]
    rec = {"workload": name, "n": n, "d": d, "K": K, "points": np.dtype(cf["dtype"]).name,
           "precision": precision, "rounds": out["rounds"], "time_to_graph_ms": round(ms, 3),
           "end_to_end_ms": round(sorted(e2e)[1], 3), "evals_alg": ev, "evals_per_s": ev / (ms * 1e-3),
           "per_round_ms": [round(s["ms"], 3) for s in st]}
    if precision != "plain":
        rec["rescues"] = resc
        rec["rescue_rate"] = resc / evaluated if evaluated else 0.0
    if name == "n200000_d50_k20":
        qs = synth.subsample(seed, n, RECALL_QUERIES)
        ei, _ = knnd.knnd_exact_knn(Pd, d, K, torch.from_numpy(qs.astype(np.int32)).cuda(), with_kl=False)
        got = out["idx"][torch.from_numpy(qs).cuda()].cpu().numpy()
        ex = ei.cpu().numpy()
        hits = sum(len(set(a.tolist()) & set(b.tolist())) for a, b in zip(got, ex))
        rec["recall"] = {"at": K, "queries": RECALL_QUERIES, "hits": hits,
                         "value": hits / (RECALL_QUERIES * K)}
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "plain"])
    ap.add_argument("--no-plain", action="store_true",
                    help="with --precision mixed, skip timing the plain descent beside it")
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-instances comparison")
    ap.add_argument("--cpu-receivers", type=int, default=400_000)
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads (device legs and oracle descents)")
    ap.add_argument("--no-share", action="store_true",
                    help="skip the one-GPU-share round (1/8 of the receivers)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB on the device (reference run for HBM counters)")
    ap.add_argument("--oracle-timing", default=None, metavar="WORKLOADS",
                    help="only time the CPU oracle's whole descent on these workloads "
                         "(comma-separated names, e.g. n2000_d5_k10,n100000_d10_k20), with the "
                         "host threads and, for n <= 10000, with one thread")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.oracle_timing:
        oracle_timing(args.oracle_timing.split(","))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2202_00517_amd as knnd
    import synth

    cfg = dict(synth.WORKLOADS["n1000000_d20_k30"])
    cfg["n"] = args.n
    n, d, K, seed = cfg["n"], cfg["d"], cfg["K"], cfg["seed"]
    D = d + 1
    log(f"generating {n} x {D} Dirichlet points")
    P = synth.dirichlet(cfg["data_seed"], n, d, np.float32)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    Pd = torch.from_numpy(P).to(dev)
    stream = torch.cuda.current_stream(dev)
    mixed = args.precision == "mixed"
    prec = knnd.KNND_PREC_MIXED_BF16 if mixed else knnd.KNND_PREC_FP64

    def timed(precision, tag):
        prm = knnd.default_params(precision=precision)

        def step():
            return knnd.knnd_build_ex(Pd, d, K, seed, prm, stream=stream.cuda_stream)

        for i in range(args.warmup):
            out = step()
            log(f"[{tag}] warmup {i}: rounds={out['rounds']}")
        torch.cuda.synchronize()
        results = []
        t0 = time.perf_counter()
        for i in range(args.steps):
            ts = time.perf_counter()
            out = step()
            torch.cuda.synchronize()
            results.append((out, time.perf_counter() - ts))
            log(f"[{tag}] step {i}: {1e3 * results[-1][1]:.1f} ms, rounds={out['rounds']}")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        evals = [sum(s["evals_alg"] for s in o["stats"]) for o, _ in results]
        assert len(set(evals)) == 1, "evaluation counts differ between identical runs"
        return results, elapsed, evals[0]

    results, elapsed, ev = timed(prec, args.precision)
    evals = [ev]
    ms_per_step = 1e3 * elapsed / args.steps
    value = evals[0] / (elapsed / args.steps)
    last = results[-1][0]
    plain = None
    if mixed and not args.no_plain:
        pres, pel, pev = timed(knnd.KNND_PREC_FP64, "plain")
        pl = pres[-1][0]
        same = (np.array_equal(pl["idx"].cpu().numpy(), last["idx"].cpu().numpy())
                and np.array_equal(pl["kl"].cpu().numpy(), last["kl"].cpu().numpy()))
        assert pev == ev and same, "mixed and plain descents differ"
        plain = {"value": pev / (pel / args.steps), "unit": "evals/s",
                 "ms_per_step": 1e3 * pel / args.steps,
                 "speedup_mixed_over_plain": pel / elapsed,
                 "identical_graph": bool(same)}

    # end to end: host points in, host lists out (H2D of the points, the
    # descent, D2H of the lists), the same call the step makes otherwise
    prm_e2e = knnd.default_params(precision=prec)
    e2e = []
    for _ in range(3):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        knnd.knnd_build_ex(P, d, K, seed, prm_e2e, with_kl=False)
        e2e.append(1e3 * (time.perf_counter() - ts))
    e2e_ms = sorted(e2e)[1]

    # roofline of the dominant kernel: the receiver pass (k_recv, one launch
    # per table-size class, then k_merge; steps a2-a5 on the receiver side),
    # timed with HIP events on the library's stream around its launches in
    # every timed round; one "launch" is one round's pass.  Algorithmic bytes:
    # eval_bytes per evaluation.  The receiver design's own traffic model and
    # the rocprofv3-measured bytes are reported beside it.
    rounds = [s for o, _ in results for s in o["stats"][1:]]
    kernels = kernel_rooflines(rounds, D, mixed)
    design = sum(recv_bytes(n, K, D, mixed, s["rescues"]) for s in rounds) / len(rounds)
    traffic = measured_traffic(args.precision)
    rk = kernels[0]
    roofline = {"bound": "hbm", "achieved": rk["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": rk["frac"], "traffic": traffic, "kernel": rk["kernel"] + ", one round",
                "avg_launch_ms": rk["avg_launch_ms"], "bytes_per_launch": rk["work_per_launch"],
                "bytes_per_eval": eval_bytes(D, mixed), "design_bytes": int(design),
                "traffic_over_design": round(traffic / design, 3) if traffic else None,
                "traffic_over_algorithmic": round(traffic / rk["work_per_launch"], 3) if traffic else None}
    steps_ms = sorted(1e3 * t for _, t in results)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": f"Dirichlet(1^{D}) points on the {d}-simplex, FP32 storage, "
                               f"n={n}, K={K}, seed={seed}, whole descent to the stop test",
                   "n": n, "d": d, "K": K, "precision": args.precision},
        "time_to_graph_ms": ms_per_step,
        "end_to_end_ms": round(e2e_ms, 2),
        "rounds": last["rounds"],
        "evals_alg": evals[0],
        "median_ms_per_step": steps_ms[len(steps_ms) // 2],
        "per_round_ms": [round(s["ms"], 3) for s in last["stats"]],
        "rescues": sum(s["rescues"] for s in last["stats"]),
        "roofline": roofline,
        "kernels": kernels,
    }
    if plain is not None:
        line["plain"] = plain
    if not args.no_share:
        log("one GPU's share: round 2 over 1/8 of the receivers vs all of them")
        line["share"] = share_leg(knnd, Pd, d, K, seed, prec)
    if not args.no_batched:
        log("batched instances: one batched call vs one by one")
        line["batched"] = batched_leg(knnd, synth, torch, args.steps)
    if not args.no_configs:
        line["per_config"] = []
        for name, prec_name in CONFIG_LEGS:
            log(f"workload {name}, {prec_name}")
            line["per_config"].append(config_leg(knnd, torch, name, prec_name))
    if not args.no_cpu_baseline:
        threads = host_threads()
        log(f"cpu baseline: oracle round 1 on {args.cpu_receivers} receivers, {threads} threads")
        line["cpu_baseline"] = cpu_baseline(P, d, K, seed, args.cpu_receivers, threads)
        line["cpu_baseline"]["cpu"] = cpu_model()
        line["cpu_baseline"]["hardware_concurrency"] = os.cpu_count()
        if not args.no_configs:
            line["oracle_descents"] = oracle_descents(sorted({c for c, _ in CONFIG_LEGS},
                                                             key=lambda c: synth.WORKLOADS[c]["n"]))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
