#!/usr/bin/env python3
"""Writes the stored FP64 oracle trajectories of the two workloads too large
for the oracle to run inside a test:

  c3_lloyd_trajectory.npz   sparse tf-idf rows, n = 1,000,000, d = 100,000,
                            ~150 stored entries per row, k = 1,000, 50 steps
  c4_lloyd_trajectory.npz   dense von Mises-Fisher rows, n = 2,000,000,
                            d = 256, k = 4,096, 20 steps

Both are plain spherical Lloyd (Section 5 of the paper) from the seeded
initial rows, computed by ``oracle/`` only (the CSR oracle with transposed
centres for c3, the numpy dense oracle for c4) on inputs from ``datagen/``.
Stored per checkpoint step t: the changed-row count, the objective
sum_j |S(j)| after the update, a SHA-256 of the whole int32 assignment, the
assignment of sampled rows with a flag for rows whose top-2 gap is at most
1e-5, and FP64 centre coordinates of sampled clusters (c3: the 256 largest
magnitudes and 256 seeded others; c4: all 256).  A SHA-256 of the generated
input pins the generator.

Run on a CPU (no GPU involved):  python tests/golden/make_full_size.py [c3|c4]
c3 takes about an hour on 8 cores, c4 about ten minutes.
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import datagen  # noqa: E402
import oracle  # noqa: E402
from oracle import dense as odense  # noqa: E402

GAP = 1e-5


def sha(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def input_sha_csr(X) -> str:
    return sha(np.array([X.n, X.d], np.int64), X.row_ptr, X.col, X.val)


def input_sha_dense(X) -> str:
    return sha(np.array(X.shape, np.int64), X)


def log(*a):
    print(*a, flush=True)


def make_c3(path):
    t0 = time.time()
    X, init, cfg = datagen.sparse_workload("c3")
    C0 = datagen.init_centers_csr(X, init)
    log("c3 generated: n=%d nnz=%d (%.0fs)" % (X.n, X.nnz, time.time() - t0))
    checkpoints = [1, 2, 10, 25, 50]
    rng = np.random.default_rng(3003)
    rows = np.sort(rng.choice(X.n, 20000, replace=False))
    clusters = np.sort(rng.choice(cfg.k, 8, replace=False))
    rec = {k: [] for k in ("step", "assign_sha", "a_sample", "inband", "objective",
                           "centre_cols", "centre_vals")}
    changed_all = []

    def on_step(t, a, C, s1, s2, changed, obj):
        changed_all.append(changed)
        log("c3 step %d: changed %d objective %s (%.0fs)" % (t, changed, obj,
                                                            time.time() - t0))
        if t not in checkpoints:
            return
        rec["step"].append(t)
        rec["assign_sha"].append(sha(a.astype(np.int32)))
        rec["a_sample"].append(a[rows].astype(np.int16))
        rec["inband"].append(np.packbits((s1 - s2)[rows] <= GAP))
        rec["objective"].append(np.nan if obj is None else obj)
        cols = np.empty((len(clusters), 512), np.int32)
        vals = np.empty((len(clusters), 512))
        crng = np.random.default_rng(7000 + t)
        for q, j in enumerate(clusters):
            c = C[j]
            top = np.argsort(-np.abs(c), kind="stable")[:256]
            rest = np.setdiff1d(np.arange(X.d), top)
            pick = np.concatenate([top, crng.choice(rest, 256, replace=False)])
            cols[q] = pick
            vals[q] = c[pick]
        rec["centre_cols"].append(cols)
        rec["centre_vals"].append(vals)

    a, C, it, conv = oracle.lloyd_trajectory(X, C0, cfg.max_iter, on_step)
    np.savez_compressed(
        path, input_sha=input_sha_csr(X), init_rows=init, n=X.n, d=X.d, nnz=X.nnz, k=cfg.k,
        max_iter=cfg.max_iter, iterations=it, converged=conv,
        changed=np.array(changed_all, np.int64), sample_rows=rows, clusters=clusters,
        gap=GAP, **{k: np.array(v) for k, v in rec.items()})
    log("wrote %s (%d steps, converged %d, %.0fs)" % (path, it, conv, time.time() - t0))


def make_c4(path):
    t0 = time.time()
    cfg = datagen.C4
    X = datagen.dense_vmf(cfg["n"], cfg["d"], cfg["n_means"], cfg["seed"])
    init = datagen.init_rows(X.shape[0], cfg["k"], cfg["seed"])
    C0 = X[init].copy()
    log("c4 generated: n=%d d=%d (%.0fs)" % (X.shape[0], X.shape[1], time.time() - t0))
    steps = 20
    rng = np.random.default_rng(4004)
    rows = np.sort(rng.choice(X.shape[0], cfg["subsample"], replace=False))
    clusters = np.sort(rng.choice(cfg["k"], 4, replace=False))
    rec = {k: [] for k in ("step", "assign_sha", "a_sample", "inband", "objective",
                           "centre_vals", "changed")}

    def on_step(t, a, C, s1, s2, changed, obj):
        log("c4 step %d: changed %d objective %s (%.0fs)" % (t, changed, obj,
                                                            time.time() - t0))
        rec["step"].append(t)
        rec["changed"].append(changed)
        rec["assign_sha"].append(sha(a.astype(np.int32)))
        rec["a_sample"].append(a[rows].astype(np.int16))
        rec["inband"].append(np.packbits((s1 - s2)[rows] <= GAP))
        rec["objective"].append(np.nan if obj is None else obj)
        rec["centre_vals"].append(C[clusters].copy())

    a, C, it, conv = odense.lloyd_trajectory(X, C0, steps, on_step)
    np.savez_compressed(
        path, input_sha=input_sha_dense(X), init_rows=init, n=X.shape[0], d=X.shape[1],
        k=cfg["k"], max_iter=steps, iterations=it, converged=conv, sample_rows=rows,
        clusters=clusters, gap=GAP, **{k: np.array(v) for k, v in rec.items()})
    log("wrote %s (%d steps, %.0fs)" % (path, it, time.time() - t0))


def main():
    which = sys.argv[1:] or ["c4", "c3"]
    for w in which:
        path = os.path.join(HERE, "%s_lloyd_trajectory.npz" % w)
        {"c3": make_c3, "c4": make_c4}[w](path)


if __name__ == "__main__":
    main()
