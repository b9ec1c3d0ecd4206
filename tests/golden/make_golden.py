"""Write tests/golden/oracle_<workload>.json: the CPU oracle's result on the
full-size synthetic workloads, as SHA-256 digests of the final neighbor lists
(int32, little-endian) and keys (FP64 bits) plus every per-round count.

Calls only oracle/ (and the input generator).  Usage:
    python tests/golden/make_golden.py n1000000_d20_k30 n200000_d50_k20 batch512
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


# Workloads whose accuracy is recorded: recall@K of the final graph against
# exhaustive search (the share of the true K nearest found, Section 4) on
# RECALL_QUERIES points drawn without replacement by the tag-7 hash from the
# workload's seed.
RECALL_WORKLOADS = {"n200000_d50_k20"}
RECALL_QUERIES = 2000


def recall_hits(P, idx, K, seed):
    P64 = oracle.widen(P)
    L = oracle.log_table(P64)
    qs = synth.subsample(seed, P.shape[0], RECALL_QUERIES)
    bf, _ = oracle.bruteforce(P64, L, K, qs)
    return int(sum(len(set(idx[q].tolist()) & set(b.tolist())) for q, b in zip(qs, bf)))


def run_single(name):
    c = synth.WORKLOADS[name]
    P = synth.dirichlet(c["data_seed"], c["n"], c["d"], c["dtype"])
    t = time.time()
    res = oracle.build_graph(P, c["d"], c["K"], c["seed"])
    secs = time.time() - t
    extra = {}
    if name in RECALL_WORKLOADS:
        extra = {"recall_queries": RECALL_QUERIES,
                 "recall_hits": recall_hits(P, res.idx, c["K"], c["seed"])}
    return {
        "workload": f"n={c['n']} d={c['d']} K={c['K']} "
                    f"{np.dtype(c['dtype']).name} points, data seed {c['data_seed']}, seed {c['seed']}",
        "status": res.status,
        "rounds": res.rounds,
        "updates": res.updates.tolist(),
        "fcr_hits": res.hits.tolist(),
        "evals_alg": res.evals.tolist(),
        "idx_sha256": digest(res.idx),
        "kl_sha256": digest(res.keys),
        "oracle_seconds": secs,
        **extra,
    }


def run_batched():
    out = []
    t = time.time()
    for b in range(synth.BATCH_INSTANCES):
        n, d, K, ds, s = synth.instance(synth.BATCH_BASE_SEED, b)
        P = synth.dirichlet(ds, n, d, np.float32)
        res = oracle.build_graph(P, d, K, s)
        out.append({"n": n, "d": d, "K": K, "status": res.status, "rounds": res.rounds,
                    "updates": res.updates.tolist(), "fcr_hits": res.hits.tolist(),
                    "evals_alg": res.evals.tolist(), "idx_sha256": digest(res.idx),
                    "kl_sha256": digest(res.keys)})
    return {"workload": f"{synth.BATCH_INSTANCES} instances from base seed {synth.BATCH_BASE_SEED}",
            "instances": out, "oracle_seconds": time.time() - t}


def main(names):
    for name in names:
        if name == synth.BATCH_WORKLOAD:
            rec = run_batched()
        else:
            rec = run_single(name)
        path = os.path.join(HERE, f"oracle_{name}.json")
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
        print(f"wrote {path} ({rec.get('oracle_seconds', 0):.1f} s)", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(synth.WORKLOADS) + [synth.BATCH_WORKLOAD])
