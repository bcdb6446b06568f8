"""Write ``rmat24_expected.json``: the CPU oracle's results on the R-MAT
scale-24 workload, as SHA-256 digests of whole output arrays plus the
scalar results.

Calls only ``graphgen`` (the input) and ``oracle`` (the results); run from
the repository root:

    python tests/golden/make_rmat24_expected.py

About 10 minutes and 30 GB of host memory, single-threaded oracle.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

LABEL_SEED, LABEL_K = 11, 4096


def digest(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(np.asarray(a, dtype=dtype)).tobytes()).hexdigest()


def graph_digest(g):
    return {"row_ptr": digest(g.row_ptr, np.int64), "col": digest(g.col, np.int32), "w": digest(g.w, np.int32)}


def main():
    t = time.time()
    g = gg.config("rmat24")
    print(f"generated n={g.n} nnz={g.nnz} in {time.time() - t:.0f}s", flush=True)
    out = {"workload": "rmat24", "n": g.n, "nnz": g.nnz, "graph": graph_digest(g), "local_move": []}
    for labels_desc, labels in (("singletons", None),
                                (f"random_labels(n, {LABEL_K}, {LABEL_SEED})", gg.random_labels(g.n, LABEL_K, LABEL_SEED))):
        t = time.time()
        r = oracle.local_move(g.row_ptr, g.col, g.w, labels)
        out["local_move"].append({"labels_in": labels_desc, "labels": digest(r.labels, np.int32),
                                  "deg": digest(r.deg, np.int64), "e_own": digest(r.e_own, np.int64)})
        print(f"local_move from {labels_desc} in {time.time() - t:.0f}s", flush=True)
    t = time.time()
    lab = gg.random_labels(g.n, LABEL_K, LABEL_SEED)
    m, k = oracle.renumber(lab)
    rp, cl, w = oracle.contract(g.row_ptr, g.col, g.w, m[lab], k)
    out["aggregate"] = {"labels_in": f"random_labels(n, {LABEL_K}, {LABEL_SEED})", "n_new": k,
                        "renumbered": digest(m[lab], np.int32), "row_ptr": digest(rp, np.int64),
                        "col": digest(cl, np.int32), "w": digest(w, np.int64)}
    del rp, cl, w
    print(f"aggregate in {time.time() - t:.0f}s: {k} communities", flush=True)
    t = time.time()
    r = oracle.louvain(g.row_ptr, g.col, g.w)
    out["run"] = {"labels": digest(r.labels, np.int32), "q_int": str(r.q_int), "q": r.q, "status": int(r.status),
                  "levels": [{k: (str(v) if k == "q_int" else int(v)) for k, v in lv.items()} for lv in r.levels]}
    print(f"run in {time.time() - t:.0f}s: {len(r.levels)} levels, Q = {r.q:.6f}", flush=True)
    with open(os.path.join(HERE, "rmat24_expected.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
