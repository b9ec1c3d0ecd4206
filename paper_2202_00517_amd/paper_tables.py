"""The statistics of the paper's Tables 3 and 4 (Section 4), measured with
this library on one GPU: rounds to the stop test against 2 ceil(log_K n),
final friend clustering coefficient, device time of the first and last
round, and accuracy (the share of the true K nearest neighbours found) on a
sample of six points, as the paper reports it, and on 2000 points.  The true
neighbours come from knnd_exact_knn, bounded by the descent's own K-th keys.

Inputs are synthetic Dirichlet(1,...,1) points (the paper's workload), FP32
storage, generated with fixed seeds; the paper's random draws are not
reproducible, so its rounds, FCC and accuracy are context, not targets.

`--table stop` runs the other terminations of Section 1.2 (Table 1) and
Section 1.3 (item (b)) on the n = 1e6, 21-coordinate, K = 30 workload: the
statistical FCR test, Dong et al.'s delta-proportion rule at two deltas, and
the fixed point, each with its rounds, time to graph, evaluations and
accuracy.

`--table cmp` runs the same workload under each comparator the library
offers (Section 2.1: any per-point total order): rounds, time to graph,
evaluations per second and accuracy against the exact search under the same
comparator.

    python -m paper_2202_00517_amd.paper_tables [--table 3|4|stop|cmp|all] [--json out.json]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_2202_00517_amd as knnd  # noqa: E402
import synth  # noqa: E402

GOLDEN = os.path.join(ROOT, "tests", "golden")


def _sample(seed, n, m):
    return synth.subsample(seed, n, m).astype(np.int32)


def accuracy(idx, P, d, K, queries, kl_bound, torch, comparator=0):
    """Mean share of the exact K nearest neighbours that the lists hold."""
    true_idx, _ = knnd.knnd_exact_knn(P, d, K, torch.from_numpy(queries).to(P.device),
                                      tau=kl_bound, with_kl=False, comparator=comparator)
    got = idx[torch.from_numpy(queries).to(P.device).long()].cpu().numpy()
    tru = true_idx.cpu().numpy()
    return float(np.mean([len(set(a.tolist()) & set(b.tolist())) / K for a, b in zip(got, tru)]))


def run_row(n, coords, K, data_seed, seed, torch, precision, stop_rule=0, delta=0.0, comparator=0):
    d = coords - 1
    P = torch.from_numpy(synth.dirichlet(data_seed, n, d, np.float32)).cuda()
    prm = knnd.default_params(precision=precision, stop_rule=stop_rule, delta=delta, comparator=comparator)
    t = time.perf_counter()
    out = knnd.knnd_build_ex(P, d, K, seed, prm)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    M = min(n, 10000)
    st = out["stats"]
    row = {"n": n, "coordinates": coords, "K": K, "rounds": out["rounds"],
           "round_bound": 2 * math.ceil(math.log(n) / math.log(K)),
           "fcc": st[-1]["fcr_hits"] / M, "first_round_ms": round(st[1]["ms"], 2),
           "last_round_ms": round(st[-1]["ms"], 2), "time_to_graph_ms": round(1e3 * wall, 1),
           "evals_alg": int(sum(s["evals_alg"] for s in st)), "last_updates": int(st[-1]["updates"]),
           "status": out["status"], "device_ms": round(sum(s["ms"] for s in st), 1)}
    row["evals_per_s"] = row["evals_alg"] / (row["device_ms"] * 1e-3)
    idx, kl = out["idx"], out["kl"]
    for name, m in (("accuracy_6", 6), ("accuracy_2000", 2000)):
        q = _sample(seed + m, n, m)
        bound = kl[torch.from_numpy(q).to(P.device).long(), K - 1]
        row[name] = round(accuracy(idx, P, d, K, q, bound, torch, comparator), 4)
    del P, out
    torch.cuda.empty_cache()
    return row


def table3(torch, precision):
    with open(os.path.join(GOLDEN, "paper_table3.json")) as f:
        paper = json.load(f)["rows"]
    rows = []
    for i, p in enumerate(paper):
        r = run_row(p["n"], p["coordinates"], p["K"], 3100 + i, 3200 + i, torch, precision)
        r["paper"] = {k: p[k] for k in ("rounds", "fcc", "first_round_s", "last_round_s")}
        print(json.dumps(r), flush=True)
        rows.append(r)
    return rows


def table4(torch, precision):
    with open(os.path.join(GOLDEN, "paper_table4.json")) as f:
        tab = json.load(f)
    rows = []
    for i, p in enumerate(tab["rows"]):
        r = run_row(tab["n"], p["coordinates"], p["K"], 4100 + i, 4200 + i, torch, precision)
        r["paper"] = {k: p[k] for k in ("fcc", "accuracy")}
        print(json.dumps(r), flush=True)
        rows.append(r)
    return rows


STOP_RULES = [("FCR test (paper)", knnd.KNND_STOP_FCR, 0.0), ("delta = 0.01", knnd.KNND_STOP_DELTA, 0.01),
              ("delta = 0.001", knnd.KNND_STOP_DELTA, 0.001), ("fixed point", knnd.KNND_STOP_FIXED_POINT, 0.0)]


def stop_rules(torch, precision, n=1000000, coords=21, K=30):
    rows = []
    for name, rule, delta in STOP_RULES:
        r = run_row(n, coords, K, 5100, 5200, torch, precision, rule, delta)
        r["rule"] = name
        print(json.dumps(r), flush=True)
        rows.append(r)
    return rows


COMPARATORS = [("KL D(x||y)", knnd.KNND_CMP_KL), ("reverse KL D(y||x)", knnd.KNND_CMP_KL_REVERSE),
               ("Hellinger", knnd.KNND_CMP_HELLINGER), ("Euclidean", knnd.KNND_CMP_L2)]


def comparators(torch, n=1000000, coords=21, K=30):
    """Every comparator in the FP64 form, and KL also in the requested mixed form."""
    rows = []
    for name, cmp in COMPARATORS:
        for prec in ([knnd.KNND_PREC_FP64, knnd.KNND_PREC_MIXED_BF16] if cmp == knnd.KNND_CMP_KL
                     else [knnd.KNND_PREC_FP64]):
            r = run_row(n, coords, K, 5100, 5200, torch, prec, comparator=cmp)
            r["comparator"] = name
            r["precision"] = "split BF16 mixed" if prec else "FP64"
            print(json.dumps(r), flush=True)
            rows.append(r)
    return rows


def markdown_cmp(rows):
    if not rows:
        return ""
    r0 = rows[0]
    lines = [f"Comparators (n = {r0['n']:.0e}, {r0['coordinates']} coordinates, K = {r0['K']}):", "",
             "| comparator | form | rounds | evaluations | device ms | evals/s | time to graph ms | accuracy 2000 pts |",
             "|---|---|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| {r['comparator']} | {r['precision']} | {r['rounds']} | {r['evals_alg']:.3e} | "
                     f"{r['device_ms']} | {r['evals_per_s']:.3e} | {r['time_to_graph_ms']} | {r['accuracy_2000']:.4f} |")
    return "\n".join(lines)


def markdown_stop(rows):
    if not rows:
        return ""
    r0 = rows[0]
    lines = [f"Stop rules (n = {r0['n']:.0e}, {r0['coordinates']} coordinates, K = {r0['K']}):", "",
             "| rule | rounds | updates in last round | evaluations | time to graph ms | accuracy 2000 pts |",
             "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| {r['rule']} | {r['rounds']} | {r['last_updates']} | {r['evals_alg']:.3e} | "
                     f"{r['time_to_graph_ms']} | {r['accuracy_2000']:.4f} |")
    return "\n".join(lines)


def markdown(t3, t4):
    lines = []
    if t3:
        lines += ["Table 3 (10 coordinates):", "",
                  "| n | K | rounds (paper) | 2⌈log_K n⌉ | FCC (paper) | 1st / last round ms | accuracy 6 pts | accuracy 2000 pts |",
                  "|---|---|---|---|---|---|---|---|"]
        for r in t3:
            p = r["paper"]
            lines.append(f"| {r['n']:.0e} | {r['K']} | {r['rounds']} ({p['rounds']}) | {r['round_bound']} | "
                         f"{r['fcc']:.3f} ({p['fcc']:.3f}) | {r['first_round_ms']} / {r['last_round_ms']} | "
                         f"{r['accuracy_6']:.3f} | {r['accuracy_2000']:.4f} |")
        lines.append("")
    if t4:
        lines += ["Table 4 (n = 2e5):", "",
                  "| K | coordinates | rounds | FCC (paper) | accuracy 6 pts (paper) | accuracy 2000 pts |",
                  "|---|---|---|---|---|---|"]
        for r in t4:
            p = r["paper"]
            lines.append(f"| {r['K']} | {r['coordinates']} | {r['rounds']} | {r['fcc']:.3f} ({p['fcc']:.2f}) | "
                         f"{r['accuracy_6']:.3f} ({p['accuracy']:.2f}) | {r['accuracy_2000']:.4f} |")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--table", default="all", choices=["3", "4", "stop", "cmp", "all"])
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp16", "plain"])
    ap.add_argument("--json", default=None)
    args = ap.parse_args()
    import torch
    prec = {"bf16": knnd.KNND_PREC_MIXED_BF16, "fp16": knnd.KNND_PREC_MIXED_FP16,
            "plain": knnd.KNND_PREC_FP64}[args.precision]
    t3 = table3(torch, prec) if args.table in ("3", "all") else []
    t4 = table4(torch, prec) if args.table in ("4", "all") else []
    sr = stop_rules(torch, prec) if args.table in ("stop", "all") else []
    cr = comparators(torch) if args.table in ("cmp", "all") else []
    print(markdown(t3, t4), flush=True)
    print(markdown_stop(sr), flush=True)
    print(markdown_cmp(cr), flush=True)
    if args.json:
        with open(args.json, "w") as f:
            json.dump({"table3": t3, "table4": t4, "stop_rules": sr, "comparators": cr}, f, indent=1)


if __name__ == "__main__":
    main()
