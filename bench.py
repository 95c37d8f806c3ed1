#!/usr/bin/env python3
"""Benchmark: Lloyd-equivalent iterations/s of accelerated spherical k-means
on one MI355X, against the plain GPU FP32 Lloyd fit at identical assignments.

Default run (no flags): the headline is the large sparse workload -- n =
1,000,000 synthetic tf-idf documents, d = 100,000 terms, ~150 stored entries
per row (log-normal lengths, Zipf(1.1) terms, tf-idf weights, unit rows),
k = 1,000 centres initialised from 1,000 seeded random documents, 50
assignment steps, Hamerly with FP32 similarities.  The same run then measures
the other workloads as secondary records under "workloads": the dense
embeddings (n = 2,000,000 von Mises-Fisher rows, d = 256, k = 4,096, BF16
matrix cores), the 256 batched problems, and the mid-size sparse workload
(n = 100,000, d = 50,000, k = 100, run to no-change).  Inputs are generated
on the host and copied to the GPU before any timing starts.

A step is one complete fit (every assignment step, centre update, movement,
bound update and test).  W untimed warm-up fits, then K timed fits between
synchronisations; value = assignment steps executed / fit time
("Lloyd-equivalent": every variant performs exactly the assignment steps of
Lloyd with identical results, checked in every run).  Timed fits run without
per-launch events; the dominant kernel's average launch time comes from one
separate fit with HIP events recorded around its launches inside the library.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X FP32 vector
PEAK_BF16_TFLOPS = 2500.0     # MI355X dense BF16 matrix
PEAK_HBM_GBS = 8000.0         # MI355X HBM3E
METRIC = "Lloyd-equivalent iters/s and sims/s vs plain GPU Lloyd at identical assignments"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Kernel sources whose change invalidates a stored counter measurement.
KERNEL_SOURCES = {
    "k_assign_csr": ["kernels_assign.hip", "skm_device.h", "skm_internal.h"],
    "k_dense_sim": ["kernels_dense.hip", "skm_internal.h"],
}


def source_digest(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2107_04074_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, variant):
    """Bytes per launch of `kernel` that L2 fetched from and wrote to the
    fabric (Infinity Cache or HBM), from the committed counter summary
    profiles/<kernel>_<workload>_<variant>_traffic.md (FETCH_SIZE + WRITE_SIZE
    per dispatch, scaled by a plain-copy calibration).  None when there is no
    summary or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "%s_%s_%s_traffic.md" % (kernel, workload, variant))
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ":" in line:
                key, val = line[2:].split(":", 1)
                fields[key.strip()] = val.strip().strip("`")
    if fields.get("source_digest") != source_digest(kernel):
        return None
    return {"bytes_per_launch": float(fields["hbm_bytes_per_launch"]),
            "file": os.path.relpath(path, ROOT)}


def walk_layout_choices(probs):
    """Row-walk layouts the compiled tuning table (csrc/walk_tuning.h,
    written by tune_walk.py) picks for these CSR problems with the FP32
    copy: problems per (padded width, row-length class, layout)."""
    import re
    path = os.path.join(ROOT, "paper_2107_04074_amd", "csrc", "walk_tuning.h")
    text = open(path).read()
    bounds = [int(v) for v in re.search(r"kWalkTuneRowBound\[[^\]]*\]\s*=\s*\{([^}]*)\}",
                                       text).group(1).split(",")]
    body = re.search(r"kWalkTune\[kWalkTuneRowClasses\]\[kWalkTuneWidths\]\s*=\s*\{(.*?)\};",
                     text, re.S).group(1)
    table = [[int(v) for v in r.split(",")] for r in re.findall(r"\{([^{}]*)\}", body)]
    counts = {}
    for X, k, _, _ in probs:
        kp = 16
        while kp < k:
            kp *= 2
        if kp > 256:
            continue
        rc = 0
        while rc < len(bounds) and X.nnz >= bounds[rc] * X.n:
            rc += 1
        lay = table[rc][kp.bit_length() - 5]
        key = "kp%d_rowclass%d_%s" % (kp, rc, "alternative" if lay else "default")
        counts[key] = counts.get(key, 0) + 1
    return {"table": table, "tuner": "paper_2107_04074_amd/tune_walk.py",
            "problems": dict(sorted(counts.items()))}


def split(v, dense):
    """'<variant>' with an optional precision suffix: '_fp32' (FP32
    similarities), '_bf16' (dense: BF16 matrix cores), '_fp16' (CSR: FP16
    centre copy for the row walk); every precision gives the same exact
    assignments."""
    for suf, p in (("_fp32", 0), ("_bf16", 1), ("_fp16", 2)):
        if v.endswith(suf):
            return v[:-len(suf)], p
    return v, (1 if dense else 0)


def timed(fn, reps):
    """Best wall time of `reps` runs of fn (after the caller's warm-up)."""
    import torch
    best, out = None, None
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        best = dt if best is None else min(best, dt)
    return best, out


class Problem:
    """One sparse or dense workload resident on the GPU, with workspaces per
    variant."""

    def __init__(self, name, dev):
        import datagen
        from paper_2107_04074_amd import skm
        self.skm, self.dev, self.name = skm, dev, name
        t0 = time.time()
        self.dense = name == "c4"
        self.Xh = self.X = None
        if self.dense:
            c4 = datagen.C4
            self.Xh = datagen.dense_vmf(c4["n"], c4["d"], c4["n_means"], c4["seed"])
            init = datagen.init_rows(self.Xh.shape[0], c4["k"], c4["seed"])
            self.C0 = self.Xh[init].copy()
            self.Xd = skm.DeviceDense.from_host(self.Xh, dev)
            self.k, self.max_iter = c4["k"], 20
            self.n, self.d, self.nnz = self.Xh.shape[0], self.Xh.shape[1], self.Xh.size
        else:
            self.X, init, cfg = datagen.sparse_workload(name)
            self.C0 = datagen.init_centers_csr(self.X, init)
            self.Xd = skm.DeviceCSR.from_host(self.X, dev)
            self.k, self.max_iter = cfg.k, cfg.max_iter
            self.n, self.d, self.nnz = self.X.n, self.X.d, self.X.nnz
        import torch
        self.C0d = torch.from_numpy(self.C0).to(dev)
        self.ws = {}
        log("generated %s: n=%d d=%d nnz=%d k=%d in %.1fs" % (name, self.n, self.d, self.nnz,
                                                             self.k, time.time() - t0))

    def workspace(self, v):
        import torch
        if v not in self.ws:
            base, prec = split(v, self.dense)
            self.ws[v] = torch.empty(self.skm.workspace_size(self.Xd, self.k, base,
                                                             precision=prec),
                                     dtype=torch.uint8, device=self.dev)
        return self.ws[v]

    def fit(self, v, profile=0, per_iter=False, schedule=0, max_iter=None):
        base, prec = split(v, self.dense)
        return self.skm.fit(self.Xd, self.k, self.C0d, base, max_iter or self.max_iter,
                            workspace=self.workspace(v), want_centers=False, per_iter=per_iter,
                            profile=profile, precision=prec, schedule=schedule)

    def release(self):
        self.ws.clear()
        self.Xd = self.C0d = None


def kernel_roofline(P, st_prof, variant):
    """Roofline record of the dominant kernel from one profiled fit: the CSR
    row walk (FP32 FMA chains over gathered centre rows) or the dense MFMA
    similarity pass.  Algorithmic FLOP = 2 k per stored entry walked (dense:
    2 k d per row); compulsory bytes = the walked rows' CSR (8 B per entry +
    8 B row pointer + 12 B of per-row bounds) plus one read of the centre
    copy (4 d k_pad B) -- what an ideal kernel must move once."""
    launches = max(st_prof.sim_kernel_launches, 1)
    avg_s = st_prof.sim_kernel_ms / 1e3 / launches
    nnz_l = st_prof.sim_kernel_nnz / launches
    rows_l = st_prof.sim_kernel_rows / launches
    flops = 2.0 * P.k * nnz_l
    achieved = flops / avg_s / 1e12 if avg_s > 0 else 0.0
    base, prec = split(variant, P.dense)
    if P.dense:
        peak = PEAK_BF16_TFLOPS if prec == 1 else PEAK_FP32_TFLOPS
        kern, bound = "k_dense_sim", "mfma"
        compulsory = rows_l * (2.0 if prec == 1 else 4.0) * 256 + 2.0 * 4096 * 256
    else:
        peak, kern, bound = PEAK_FP32_TFLOPS, "k_assign_csr", "alu"
        kpad = 1 << max(4, (P.k - 1).bit_length())  # centre copy width: power of two >= 16
        compulsory = 8.0 * nnz_l + 20.0 * rows_l + (4.0 if prec != 2 else 2.0) * P.d * kpad
    traffic = measured_traffic(kern, P.name, variant)
    rec = {
        "kernel": kern, "bound": bound, "achieved": round(achieved, 3), "peak": peak,
        "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
        "traffic": traffic["bytes_per_launch"] if traffic else None,
        "traffic_source": traffic["file"] if traffic else None,
        "avg_launch_us": round(avg_s * 1e6, 3), "launches": st_prof.sim_kernel_launches,
        "flops_per_launch": flops,
        "compulsory_bytes_per_launch": compulsory,
        "compulsory_GBps": round(compulsory / avg_s / 1e9, 1) if avg_s > 0 else 0.0,
        "compulsory_frac_of_hbm_peak": round(compulsory / avg_s / 8.0e12, 4) if avg_s > 0
        else 0.0,
    }
    if not P.dense:
        # every walked entry gathers one whole centre row (no reuse): the
        # bytes the walk pulls through the vector-memory path
        operand = (4.0 if prec != 2 else 2.0) * nnz_l * kpad
        rec["operand_bytes_per_launch"] = operand
        rec["operand_GBps"] = round(operand / avg_s / 1e9, 1) if avg_s > 0 else 0.0
    if traffic and avg_s > 0:
        # L2 <-> fabric bytes (FETCH_SIZE + WRITE_SIZE): served by the 256 MB
        # Infinity Cache or HBM, so an upper bound of HBM traffic
        rec["fabric_GBps"] = round(traffic["bytes_per_launch"] / avg_s / 1e9, 1)
        rec["fabric_frac_of_hbm_peak"] = round(traffic["bytes_per_launch"] / avg_s / 8.0e12, 4)
    return rec


def run_single(P, variant, steps, warmup, table, skip_baseline):
    """Headline-style record of one workload: the timed variant against the
    plain GPU FP32 Lloyd fit, a comparison table, per-step pruning."""
    import torch
    base_v = "lloyd_fp32" if P.dense else "lloyd"
    a_ref = st_ref = st_l = lloyd_s = None
    if not skip_baseline:
        a_ref, _, _, st_ref = P.fit(base_v)
        lloyd_s, (_, _, _, st_l) = timed(lambda: P.fit(base_v), 2)
        log("%s lloyd: %d steps, %.3f ms/fit" % (P.name, st_l.iterations, lloyd_s * 1e3))
    for _ in range(warmup):
        P.fit(variant)
    torch.cuda.synchronize()
    stats = []
    t_start = time.perf_counter()
    for _ in range(steps):
        a_v, _, _, st = P.fit(variant)
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    identical = None if a_ref is None else (
        bool(torch.equal(a_v, a_ref)) and all(s.iterations == st_ref.iterations for s in stats))
    # launch statistics of the dominant kernel from one more fit with events
    _, _, _, st_prof = P.fit(variant, profile=1)
    torch.cuda.synchronize()

    variants = {}
    for v in table:
        P.fit(v)
        best, (a_x, _, _, st_x) = timed(lambda: P.fit(v), 2)
        variants[v] = {"ms_per_fit": round(best * 1e3, 3),
                       "iters_per_s": round(st_x.iterations / best, 3),
                       "speedup_vs_gpu_lloyd": None if lloyd_s is None else
                       round(lloyd_s / best, 3),
                       "sims_fraction": round(st_x.sims_point_center /
                                              (P.n * P.k * st_x.iterations), 4),
                       "identical": None if a_ref is None else
                       bool(torch.equal(a_x, a_ref)) and st_x.iterations == st_ref.iterations}
        log("%s %-18s %9.3f ms/fit  sims %.3f  identical %s" % (
            P.name, v, best * 1e3, variants[v]["sims_fraction"], variants[v]["identical"]))

    # similarities computed per assignment step, as a fraction of Lloyd's n k
    # (tightenings count as computed, so the fraction can exceed 1), with the
    # default schedule and with the bound tests at every step (the paper's)
    vb, _ = split(variant, P.dense)
    _, _, _, st_pi = P.fit(variant, per_iter=True)
    sims_frac = [round(float(x) / (P.n * P.k), 4) for x in st_pi.sims_per_iter[:st_pi.iterations]]
    sims_frac_tested = None
    if vb != "lloyd":
        _, _, _, st_ps = P.fit(variant, per_iter=True, schedule=1)
        sims_frac_tested = [round(float(x) / (P.n * P.k), 4)
                            for x in st_ps.sims_per_iter[:st_ps.iterations]]
    torch.cuda.synchronize()
    iters = sum(s.iterations for s in stats)
    sims = sum(s.sims_point_center for s in stats)
    lloyd_equiv_sims = P.n * P.k * iters
    st = stats[-1]
    base, prec = split(variant, P.dense)
    return {
        "value": round(iters / elapsed, 3),
        "ms_per_step": round(elapsed / steps * 1e3, 4),
        "dtype": {0: "f32", 1: "bf16", 2: "f32"}[prec],
        "config": {"workload": "%s: spherical k-means %s, n=%d d=%d nnz=%d k=%d, seeded "
                               "random-row init, %s" % (
                                   P.name, variant, P.n, P.d, P.nnz, P.k,
                                   ("%d assignment steps at most (stops early when nothing "
                                    "changes)" % P.max_iter) if P.max_iter < 1000 else
                                   "run to no-change"),
                   "variant": variant, "n": P.n, "d": P.d, "nnz": P.nnz, "k": P.k,
                   "max_iter": P.max_iter, "parallelism": "single GPU",
                   "similarity_arithmetic": {0: "fp32 FMA", 1: "bf16 MFMA, fp32 accumulate",
                                             2: "fp16 centre copy, fp32 FMA"}[prec]},
        "iterations_per_fit": st.iterations,
        "converged": st.converged,
        "identical_assignments_to_lloyd": identical,
        "speedup_vs_gpu_lloyd": None if lloyd_s is None else
        round(lloyd_s / (elapsed / steps), 3),
        "gpu_lloyd": None if lloyd_s is None else {
            "variant": base_v, "iters_per_s": round(st_l.iterations / lloyd_s, 3),
            "ms_per_fit": round(lloyd_s * 1e3, 3),
            "sims_per_s": round(st_l.sims_point_center / lloyd_s, 1)},
        "sims_per_s_raw": round(sims / elapsed, 1),
        "sims_per_s_lloyd_equiv": round(lloyd_equiv_sims / elapsed, 1),
        "sims_fraction": round(sims / lloyd_equiv_sims, 4),
        "sims_fraction_per_iter": sims_frac,
        "sims_fraction_per_iter_tests_every_step": sims_frac_tested,
        "rechecks_per_fit": st.rechecks,
        "variants": variants,
        "roofline": kernel_roofline(P, st_prof, variant),
    }


def cpu_baseline_sparse(P, variant, gpu_iters, budget_s=12.0):
    """The FP64 oracle on a bounded sample: the first rows of the workload
    (same initial centres), the variant's first steps; scaled to all rows by
    the row count (a step's work is linear in the rows)."""
    import oracle
    base, _ = split(variant, False)
    steps = min(2, gpu_iters)
    rows = min(P.n, 20000)
    Xs = P.X.take_rows(np.arange(rows))
    t = time.perf_counter()
    r = oracle.fit(Xs, P.C0, base, steps)
    cpu_s = time.perf_counter() - t
    if cpu_s < budget_s / 4 and rows < P.n:  # too short to time well: take more rows
        rows = min(P.n, int(rows * budget_s / max(cpu_s, 1e-3) / 2))
        Xs = P.X.take_rows(np.arange(rows))
        t = time.perf_counter()
        r = oracle.fit(Xs, P.C0, base, steps)
        cpu_s = time.perf_counter() - t
    full_s = cpu_s * P.n / rows
    return {"value": round(r.iterations / full_s, 5), "unit": "iters/s",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": "FP64 oracle %s on the first %d of %d rows, %d assignment steps (%.1f s), "
                      "scaled to all rows" % (base, rows, P.n, r.iterations, cpu_s)}


def cpu_baseline_dense(P):
    """The FP64 oracle's assignment step on evenly spaced rows (about 10 s on
    16 host cores), scaled to all rows."""
    import datagen
    import oracle
    m = min(P.n, 320000)
    sub = np.arange(0, P.n, P.n // m)[:m]
    Xs = P.Xh[sub]
    rp = np.arange(0, Xs.size + 1, Xs.shape[1], dtype=np.int64)
    Xc = datagen.CSR(Xs.shape[0], Xs.shape[1], rp,
                     np.tile(np.arange(Xs.shape[1], dtype=np.int32), Xs.shape[0]), Xs.ravel())
    t = time.perf_counter()
    oracle.assign(Xc, P.C0.astype(np.float64))
    cpu_s = time.perf_counter() - t
    step_s = cpu_s * P.n / len(sub)
    return {"value": round(1.0 / step_s, 5), "unit": "iters/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": "FP64 oracle assignment step on %d of %d rows (%.1f s), scaled to all "
                      "rows" % (len(sub), P.n, cpu_s)}


def run_batched(dev, variant, steps, warmup, workers_arg, skip_baseline, no_cpu, max_iter=0):
    """256 independent sparse problems (n_b log-normal in [1e3, 5e4], k_b =
    8 * U{1..32}, d = 20,000, ~80 stored entries per row, 30 steps at most),
    solved by one skm_fit_batched call, against the plain GPU Lloyd fit of
    each problem one after another."""
    import torch
    import datagen
    from paper_2107_04074_amd import skm
    t0 = time.time()
    insts = datagen.batched_instances()
    probs = []
    for p in insts:
        Xd = skm.DeviceCSR.from_host(p.X, dev)
        C0 = torch.from_numpy(datagen.init_centers_csr(p.X, p.init)).to(dev)
        probs.append((Xd, p.k, C0, max_iter or p.max_iter))
    n_tot = sum(p.X.n for p in insts)
    nnz_tot = sum(p.X.nnz for p in insts)
    log("generated c5: %d problems, %d rows, %d stored entries in %.1fs" % (
        len(insts), n_tot, nnz_tot, time.time() - t0))

    def total_steps(res):
        return sum(r[2].iterations for r in res)

    base_res = base_s = None
    if not skip_baseline:
        ws_size = max(skm.workspace_size(X, k, "lloyd") for X, k, _, _ in probs)
        ws = torch.empty(ws_size, dtype=torch.uint8, device=dev)

        def sequential():
            return [skm.fit(X, k, C0, "lloyd", it, workspace=ws, want_centers=False,
                            per_iter=False)[0::3] for X, k, C0, it in probs]
        sequential()
        base_s, base_res = timed(sequential, 1)
        base_res = [(a, None, st) for a, st in base_res]
        log("c5 sequential lloyd: %d steps, %.1f ms" % (total_steps(base_res), base_s * 1e3))

    sweep = {}
    workers = workers_arg
    if workers == 0:
        for w in (1, 2, 4, 8):
            skm.fit_batched(probs, variant, workers=w, want_centers=False)
            sweep[w] = round(timed(lambda: skm.fit_batched(probs, variant, workers=w,
                                                           want_centers=False), 1)[0] * 1e3, 3)
            log("c5 batched %s workers=%d: %.1f ms" % (variant, w, sweep[w]))
        workers = min(sweep, key=sweep.get)
    bws = torch.empty(skm.batched_workspace_size(probs, variant, workers=workers),
                      dtype=torch.uint8, device=dev)
    for _ in range(warmup):
        skm.fit_batched(probs, variant, workers=workers, workspace=bws, want_centers=False)
    torch.cuda.synchronize()
    runs = []
    t_start = time.perf_counter()
    for _ in range(steps):
        runs.append(skm.fit_batched(probs, variant, workers=workers, workspace=bws,
                                    want_centers=False))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    res = runs[-1]
    nsteps = total_steps(res)
    identical = None
    if base_res is not None:
        identical = all(torch.equal(a, b[0]) and s.iterations == b[2].iterations
                        for (a, _, s), b in zip(res, base_res))
    sims = sum(r[2].sims_point_center for run in runs for r in run)
    lloyd_sims = sum(X.n * k * r[2].iterations for run in runs
                     for (X, k, _, _), r in zip(probs, run))
    out = {
        "value": round(nsteps * steps / elapsed, 3),
        "unit": "iters/s",
        "ms_per_step": round(elapsed / steps * 1e3, 4),
        "dtype": "f32",
        "config": {"workload": "c5: %d batched spherical k-means problems (%s), n_b log-normal "
                               "in [1e3, 5e4] (sum %d), k_b in 8..256, d=20000, nnz %d, at most "
                               "%d steps each, one skm_fit_batched call per step" % (
                                   len(probs), variant, n_tot, nnz_tot, probs[0][3]),
                   "variant": variant, "problems": len(probs), "rows": n_tot, "nnz": nnz_tot,
                   "workers": workers, "parallelism": "single GPU",
                   "driver": "host threads, one HIP stream per worker, each running the "
                             "single-problem fit"},
        "assignment_steps_per_call": nsteps,
        "identical_assignments_to_lloyd": identical,
        "speedup_vs_sequential_gpu_lloyd": None if base_s is None else
        round(base_s / (elapsed / steps), 3),
        "sequential_gpu_lloyd": None if base_s is None else {
            "ms": round(base_s * 1e3, 3), "iters_per_s": round(total_steps(base_res) / base_s, 3)},
        "worker_sweep_ms": sweep,
        "walk_layouts": walk_layout_choices(probs),
        "sims_per_s_raw": round(sims / elapsed, 1),
        "sims_per_s_lloyd_equiv": round(lloyd_sims / elapsed, 1),
        "sims_fraction": round(sims / max(lloyd_sims, 1), 4),
    }
    if not no_cpu:
        import oracle
        # bounded sample: problems in index order until ~8 s of oracle work,
        # each fitted to its GPU step count; scaled to the whole batch by
        # stored entries x k x steps
        work = [X.nnz * k * r[2].iterations for (X, k, _, _), r in zip(probs, res)]
        t = time.perf_counter()
        done, w_done = 0, 0.0
        for b, p in enumerate(insts):
            oracle.fit(p.X, datagen.init_centers_csr(p.X, p.init), variant, res[b][2].iterations)
            done += 1
            w_done += work[b]
            if time.perf_counter() - t > 8.0:
                break
        cpu_s = time.perf_counter() - t
        est_all = cpu_s * sum(work) / max(w_done, 1.0)
        out["cpu_baseline"] = {
            "value": round(nsteps / est_all, 4), "unit": "iters/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": "FP64 oracle %s on the first %d of %d problems (%.1f s), scaled to the "
                      "batch by stored entries x k x steps" % (variant, done, len(insts), cpu_s)}
    return out


# Dimensionality experiment (Section 6, the run times on the DBLP
# author-conference matrix and on its transpose): the same number of stored
# entries as many short rows over few columns, or as few long rows over many
# columns; beside them the shape of RCV-1 (Table 1), on which Table 3 shows the
# largest speed-ups of the bounded variants.  Seeded synthetic stand-ins with
# the shapes and densities of Table 1.
DIMS_SHAPES = (("rows_1842986_x_cols_5236", 1_842_986, 5_236, 2.9, 0),
               ("rows_5236_x_cols_1842986", 5_236, 1_842_986, 1032.0, 0),
               ("rows_804414_x_cols_47236", 804_414, 47_236, 75.6, 0),
               # the RCV-1 shape again with topic structure (100 topics), so that
               # the centres settle as they do on real text
               ("rows_804414_x_cols_47236_topics", 804_414, 47_236, 75.6, 100))
DIMS_K = (10, 50, 200, 500)
DIMS_VARIANTS = ("lloyd", "simp_hamerly", "hamerly", "simp_elkan", "elkan", "yinyang")


def run_dims(dev, max_iter):
    """Every variant at every k on both shapes: ms per fit (best of two after
    a warm-up), the row walks' time in it (HIP events, one more fit), steps,
    similarities computed (fraction of Lloyd's), rows re-decided in FP64 per
    step and the centre-centre inner products the full variants evaluated;
    assignments are checked identical to the Lloyd fit's."""
    import torch
    import datagen
    from paper_2107_04074_amd import skm
    rows = []
    for si, (name, n, d, mean, topics) in enumerate(DIMS_SHAPES):
        t0 = time.time()
        Xh = datagen.sparse_tfidf(n, d, mean, datagen.BASE_SEED + 60 + si, topics=topics)
        X = skm.DeviceCSR.from_host(Xh, dev)
        log("generated %s: n=%d d=%d nnz=%d in %.1fs" % (name, Xh.n, Xh.d, Xh.nnz,
                                                        time.time() - t0))
        for k in DIMS_K:
            init = datagen.init_rows(Xh.n, k, datagen.BASE_SEED + 70 + k)
            C0 = torch.from_numpy(datagen.init_centers_csr(Xh, init)).to(dev)
            ref = None
            for v in DIMS_VARIANTS:
                ws = torch.empty(skm.workspace_size(X, k, v), dtype=torch.uint8, device=dev)

                def fit():
                    return skm.fit(X, k, C0, v, max_iter, workspace=ws, want_centers=False,
                                   per_iter=False)
                fit()
                best, (a, _, _, st) = timed(fit, 2)
                # the row walks' share, from one more fit with events around them
                st_p = skm.fit(X, k, C0, v, max_iter, workspace=ws, want_centers=False,
                               per_iter=False, profile=1)[3]
                if ref is None:
                    ref = (a, st.iterations, best)
                row = {"shape": name, "k": k, "variant": v, "ms_per_fit": round(best * 1e3, 3),
                       "steps": st.iterations,
                       "speedup_vs_gpu_lloyd": round(ref[2] / best, 3),
                       "sims_fraction": round(st.sims_point_center /
                                              (Xh.n * k * st.iterations), 4),
                       "centre_centre_products": st.sims_center_center,
                       "fp64_redecided_rows_per_step": round(st.rechecks / st.iterations, 1),
                       "row_walk_ms_per_fit": round(st_p.sim_kernel_ms, 3),
                       "identical": bool(torch.equal(a, ref[0])) and st.iterations == ref[1]}
                rows.append(row)
                log("%s k=%d %-13s %9.3f ms/fit  walks %8.3f ms  steps %d  sims %.3f  cc %d  "
                    "redecided/step %d  identical %s" % (
                        name, k, v, best * 1e3, st_p.sim_kernel_ms, st.iterations,
                        row["sims_fraction"], st.sims_center_center,
                        st.rechecks // max(st.iterations, 1), row["identical"]))
                del ws
        del X
        torch.cuda.empty_cache()
    return {"config": {"workload": "dims: shapes of the DBLP author-conference matrix and its "
                                   "transpose (1842986 x 5236, 2.9 entries per row; 5236 x "
                                   "1842986, 1032 per row) and of RCV-1 (804414 x 47236, 75.6 "
                                   "per row; plain, and with 100 topics), k in %s, at most %d "
                                   "steps, FP32 copy" % (
                                       list(DIMS_K), max_iter),
                       "parallelism": "single GPU"},
            "dtype": "f32", "table": rows,
            "all_identical": all(r["identical"] for r in rows)}


SPARSE_TABLE = {
    "c2": ["lloyd", "simp_hamerly", "hamerly", "simp_elkan", "elkan", "yinyang",
           "lloyd_fp16", "hamerly_fp16", "yinyang_fp16"],
    "c3": ["lloyd_fp16", "hamerly_fp16", "yinyang", "yinyang_fp16", "simp_elkan",
           "simp_elkan_fp16"],
    "c1": ["lloyd", "hamerly", "elkan", "yinyang"],
}
DENSE_TABLE = ["lloyd_bf16", "simp_hamerly_bf16", "hamerly_fp32"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed fits of the headline")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--variant", default="hamerly")
    ap.add_argument("--workload", default="all",
                    choices=["all", "c1", "c2", "c3", "c4", "c5", "dims"],
                    help="all (default): c3 headline, then c4, c5, c2 and the dimensionality "
                         "experiment (dims) as secondary records")
    ap.add_argument("--workers", type=int, default=0,
                    help="c5: concurrent streams of the batched fit (0 = sweep 1, 2, 4, 8 "
                         "untimed and keep the fastest)")
    ap.add_argument("--max-iter", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--quick", action="store_true", help="skip the per-variant tables")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    ap.add_argument("--skip-baseline", action="store_true",
                    help="time only the chosen variant (for counter runs: every launch of "
                         "the similarity kernel then belongs to the timed fits)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2107_04074_amd import skm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    skm.load()
    t_run = time.time()

    if args.calib_copy_mib:
        nbytes = args.calib_copy_mib << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read + written per launch" % nbytes)

    head = "c3" if args.workload == "all" else args.workload
    common = {"metric": METRIC, "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "data": "synthetic"}

    if head == "dims":
        out = dict(common)
        out.update(run_dims(dev, args.max_iter or 20))
        print(json.dumps(out), flush=True)
        return

    if head == "c5":
        rec = run_batched(dev, args.variant, args.steps, args.warmup, args.workers,
                          args.skip_baseline, args.no_cpu, args.max_iter)
        out = dict(common)
        out.update(rec)
        print(json.dumps(out), flush=True)
        return

    P = Problem(head, dev)
    if args.max_iter:
        P.max_iter = args.max_iter
    variant = args.variant
    if P.dense and split(variant, True)[1] == 1 and not variant.endswith("_bf16"):
        variant = variant + "_bf16"
    table = [] if (args.quick or args.skip_baseline) else (
        DENSE_TABLE if P.dense else SPARSE_TABLE[head])
    rec = run_single(P, variant, args.steps, args.warmup, table, args.skip_baseline)
    out = dict(common)
    out.update(rec)
    if not args.no_cpu:
        out["cpu_baseline"] = (cpu_baseline_dense(P) if P.dense else
                               cpu_baseline_sparse(P, variant, rec["iterations_per_fit"]))
    P.release()
    del P
    torch.cuda.empty_cache()

    if args.workload == "all":
        # secondary records: each workload's own line of figures, same
        # timing rules, fewer timed fits
        workloads = {}
        for name in ("c4", "c5", "c2", "dims"):
            t0 = time.time()
            if name == "dims":
                r = run_dims(dev, 20)
            elif name == "c5":
                r = run_batched(dev, "hamerly", 2, 1, 0, False, args.no_cpu)
            else:
                Q = Problem(name, dev)
                v = "hamerly_bf16" if Q.dense else "hamerly"
                r = run_single(Q, v, 3 if name == "c4" else 5, 1,
                               [] if args.quick else (DENSE_TABLE if Q.dense
                                                      else SPARSE_TABLE[name]), False)
                if not args.no_cpu:
                    r["cpu_baseline"] = (cpu_baseline_dense(Q) if Q.dense else
                                         cpu_baseline_sparse(Q, v, r["iterations_per_fit"]))
                Q.release()
                del Q
                torch.cuda.empty_cache()
            r["wall_s"] = round(time.time() - t0, 1)
            workloads[name] = r
            log("%s done in %.1fs" % (name, r["wall_s"]))
        out["workloads"] = workloads
    out["bench_wall_s"] = round(time.time() - t_run, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
