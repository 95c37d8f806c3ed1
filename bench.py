#!/usr/bin/env python3
"""Benchmark: Lloyd-equivalent iterations/s of accelerated spherical k-means
on one MI355X, against the plain GPU FP32 Lloyd fit at identical assignments.

Workload (default): n = 100,000 synthetic tf-idf documents, d = 50,000
terms, ~100 stored entries per row (log-normal lengths, Zipf(1.1) terms,
tf-idf weights, unit rows), k = 100 centres initialised from 100 seeded
random documents, run until no assignment changes.  Inputs are generated on
the host and copied to the GPU before any timing starts.

A step is one complete fit (every assignment step, centre update, movement,
bound update and test, until convergence).  W untimed warm-up fits, then K
timed fits between synchronisations; value = assignment steps executed / fit
time ("Lloyd-equivalent" because every variant performs exactly the
assignment steps of Lloyd with identical results).  The plain Lloyd fit is
timed the same way for the speedup.

Prints one JSON line (see the project design notes for the fields).
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
    """HBM bytes per launch of `kernel` from the committed counter summary
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--variant", default="hamerly")
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--workers", type=int, default=0,
                    help="c5: concurrent streams of the batched fit (0 = sweep 1, 2, 4, 8 "
                         "untimed and keep the fastest)")
    ap.add_argument("--max-iter", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-iters", type=int, default=0,
                    help="oracle sample: first N assignment steps (0 = auto)")
    ap.add_argument("--quick", action="store_true",
                    help="skip the per-variant comparison table")
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
    import datagen
    from paper_2107_04074_amd import skm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    skm.load()

    if args.workload == "c5":
        return run_batched(args, torch, dev, datagen, skm)

    t0 = time.time()
    dense = args.workload == "c4"
    if dense:
        c4 = datagen.C4
        Xh = datagen.dense_vmf(c4["n"], c4["d"], c4["n_means"], c4["seed"])
        init = datagen.init_rows(Xh.shape[0], c4["k"], c4["seed"])
        C0 = Xh[init].copy()
        Xd = skm.DeviceDense.from_host(Xh, dev)
        k, max_iter = c4["k"], args.max_iter or 20
        n_rows, d_cols, nnz = Xh.shape[0], Xh.shape[1], Xh.size
        name = "c4"
        X = None
    else:
        X, init, cfg = datagen.sparse_workload(args.workload)
        C0 = datagen.init_centers_csr(X, init)
        Xd = skm.DeviceCSR.from_host(X, dev)
        k, max_iter = cfg.k, args.max_iter or cfg.max_iter
        n_rows, d_cols, nnz = X.n, X.d, X.nnz
        name = cfg.name
    log("generated %s: n=%d d=%d nnz=%d k=%d in %.1fs" % (name, n_rows, d_cols, nnz, k,
                                                         time.time() - t0))
    C0d = torch.from_numpy(C0).to(dev)

    ws = {}

    def split(v):
        # "<variant>", or with a precision suffix: "_fp32" (FP32 similarities),
        # "_bf16" (dense: BF16 matrix cores), "_fp16" (CSR: FP16 centre copy
        # for the row walk); every precision gives the same exact assignments
        if v.endswith("_fp32"):
            return v[:-5], 0
        if v.endswith("_bf16"):
            return v[:-5], 1
        if v.endswith("_fp16"):
            return v[:-5], 2
        return v, (1 if dense else 0)

    def workspace(v):
        if v not in ws:
            base, prec = split(v)
            ws[v] = torch.empty(skm.workspace_size(Xd, k, base, precision=prec),
                                dtype=torch.uint8, device=dev)
        return ws[v]

    def one_fit(v, profile=0):
        base, prec = split(v)
        return skm.fit(Xd, k, C0d, base, max_iter, workspace=workspace(v), want_centers=False,
                       per_iter=False, profile=profile, precision=prec)

    if args.calib_copy_mib:
        nbytes = args.calib_copy_mib << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read + written per launch" % nbytes)

    # plain GPU FP32 Lloyd: the reference the speedup and the assignment
    # check use
    base_v = "lloyd_fp32" if dense else "lloyd"
    if args.variant == "hamerly" and dense:
        args.variant = "hamerly_bf16"
    if args.skip_baseline:
        a_ref = st_ref = st_l = None
        lloyd_s = None
    else:
        a_ref, _, _, st_ref = one_fit(base_v)
        torch.cuda.synchronize()
        lloyd_times = []
        for _ in range(2):
            torch.cuda.synchronize()
            t = time.perf_counter()
            a_l, _, _, st_l = one_fit(base_v)
            torch.cuda.synchronize()
            lloyd_times.append(time.perf_counter() - t)
        lloyd_s = min(lloyd_times)
        log("lloyd: %d steps, %.3f ms/fit" % (st_l.iterations, lloyd_s * 1e3))

    # timed variant
    for _ in range(args.warmup):
        one_fit(args.variant, profile=1)
    torch.cuda.synchronize()
    stats = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        a_v, _, _, st = one_fit(args.variant, profile=1)
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start

    identical = None if a_ref is None else (
        bool(torch.equal(a_v, a_ref)) and all(s.iterations == st_ref.iterations for s in stats))

    # every variant, timed the same way (best of 2), for the comparison table
    variants = {}
    table = (["lloyd_fp32", "lloyd_bf16", "simp_hamerly_bf16", "hamerly_bf16",
              "hamerly_fp32"] if dense else
             ["lloyd", "simp_hamerly", "hamerly", "simp_elkan", "elkan", "yinyang",
              "lloyd_fp16", "simp_hamerly_fp16", "hamerly_fp16", "yinyang_fp16"])
    for v in ([] if (args.quick or args.skip_baseline) else table):
        one_fit(v)
        best = None
        for _ in range(2):
            torch.cuda.synchronize()
            t = time.perf_counter()
            a_x, _, _, st_x = one_fit(v)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            best = dt if best is None else min(best, dt)
        variants[v] = {"ms_per_fit": round(best * 1e3, 4),
                       "iters_per_s": round(st_x.iterations / best, 3),
                       "speedup_vs_gpu_lloyd": round(lloyd_s / best, 3),
                       "sims_fraction": round(st_x.sims_point_center /
                                              (n_rows * k * st_x.iterations), 4),
                       "identical": bool(torch.equal(a_x, a_ref)) and
                       st_x.iterations == st_ref.iterations}
        log("%-13s %8.3f ms/fit  sims %.3f  identical %s" % (
            v, best * 1e3, variants[v]["sims_fraction"], variants[v]["identical"]))
    # pruned fraction of the similarities per assignment step (one more,
    # untimed fit of the timed variant with per-step statistics)
    vb, vp = split(args.variant)
    _, _, _, st_pi = skm.fit(Xd, k, C0d, vb, max_iter, workspace=workspace(args.variant),
                             want_centers=False, per_iter=True, precision=vp)
    torch.cuda.synchronize()
    pruned_per_iter = [round(1.0 - float(x) / (n_rows * k), 4)
                       for x in st_pi.sims_per_iter[:st_pi.iterations]]
    # the same with the bound tests at every step (schedule 1, as the paper
    # runs them); the default schedule switches tests off while they prune
    # little, and such steps prune nothing
    pruned_tested = None
    if vb != "lloyd":
        _, _, _, st_ps = skm.fit(Xd, k, C0d, vb, max_iter, workspace=workspace(args.variant),
                                 want_centers=False, per_iter=True, precision=vp, schedule=1)
        torch.cuda.synchronize()
        pruned_tested = [round(1.0 - float(x) / (n_rows * k), 4)
                         for x in st_ps.sims_per_iter[:st_ps.iterations]]
    iters = sum(s.iterations for s in stats)
    ms_per_step = elapsed / args.steps * 1e3
    value = iters / elapsed
    sims = sum(s.sims_point_center for s in stats)
    lloyd_equiv_sims = n_rows * k * iters
    st = stats[-1]

    # dominant kernel: the similarity kernel, timed with HIP events on the
    # fit's stream inside the library
    launches = sum(s.sim_kernel_launches for s in stats)
    kern_ms = sum(s.sim_kernel_ms for s in stats)
    kern_nnz = sum(s.sim_kernel_nnz for s in stats)
    kern_rows = sum(s.sim_kernel_rows for s in stats)
    avg_launch_s = kern_ms / 1e3 / max(launches, 1)
    flops_per_launch = 2.0 * k * kern_nnz / max(launches, 1)
    achieved_tflops = flops_per_launch / avg_launch_s / 1e12 if avg_launch_s > 0 else 0.0
    operand_bytes_per_launch = (4.0 * k * kern_nnz + 8.0 * kern_nnz + 20.0 * kern_rows) / max(
        launches, 1)
    if dense:
        # MFMA-bound contraction: the peak of the precision it runs in
        vbase, vprec = split(args.variant)
        roof = {"kernel": "k_dense_sim", "bound": "mfma",
                "peak": 2500.0 if vprec == 1 else 157.3,
                "dtype": "bf16" if vprec == 1 else "f32"}
    else:
        roof = {"kernel": "k_assign_csr", "bound": "alu", "peak": PEAK_FP32_TFLOPS}
    traffic = measured_traffic(roof["kernel"], name, args.variant)

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {0: "f32", 1: "bf16", 2: "f32"}[split(args.variant)[1]],
        "data": "synthetic",
        "config": {"workload": "%s: spherical k-means %s, n=%d d=%d nnz=%d k=%d, seeded "
                               "random-row init, %s" % (
                                   name, args.variant, n_rows, d_cols, nnz, k,
                                   "run to no-change" if not dense else
                                   "%d assignment steps" % max_iter),
                   "variant": args.variant, "n": n_rows, "d": d_cols, "nnz": nnz, "k": k,
                   "max_iter": max_iter, "parallelism": "single GPU",
                   "centre_copy": {0: "fp32", 1: "bf16", 2: "fp16"}[split(args.variant)[1]]},
        "iterations_per_fit": st.iterations,
        "converged": st.converged,
        "identical_assignments_to_lloyd": identical,
        "speedup_vs_gpu_lloyd": None if lloyd_s is None else
        round(lloyd_s / (elapsed / args.steps), 3),
        "gpu_lloyd": None if lloyd_s is None else {
            "iters_per_s": round(st_l.iterations / lloyd_s, 3),
            "ms_per_fit": round(lloyd_s * 1e3, 4),
            "sims_per_s": round(st_l.sims_point_center / lloyd_s, 1)},
        "sims_per_s_raw": round(sims / elapsed, 1),
        "sims_per_s_lloyd_equiv": round(lloyd_equiv_sims / elapsed, 1),
        "pruned_fraction": round(1.0 - sims / lloyd_equiv_sims, 4),
        "pruned_per_iter": pruned_per_iter,
        "pruned_per_iter_tests_every_step": pruned_tested,
        "rechecks_per_fit": st.rechecks,
        "variants": variants,
        "roofline": {
            "kernel": roof["kernel"],
            "bound": roof["bound"],
            "achieved": round(achieved_tflops, 3),
            "peak": roof["peak"],
            "unit": "TFLOP/s",
            "frac": round(achieved_tflops / roof["peak"], 4),
            "traffic": traffic["bytes_per_launch"] if traffic else None,
            "traffic_source": traffic["file"] if traffic else None,
            "avg_launch_us": round(avg_launch_s * 1e6, 3),
            "launches": launches,
            "flops_per_launch": flops_per_launch,
            "operand_bytes_per_launch": operand_bytes_per_launch,
            "operand_GBps": round(operand_bytes_per_launch / avg_launch_s / 1e9, 1)
            if avg_launch_s > 0 else 0.0,
            # measured L2-to-fabric bytes (Infinity Cache or HBM) per launch over
            # this run's average launch time, against the 8 TB/s HBM peak
            "traffic_GBps": round(traffic["bytes_per_launch"] / avg_launch_s / 1e9, 1)
            if traffic and avg_launch_s > 0 else None,
            "traffic_frac_of_hbm_peak": round(traffic["bytes_per_launch"] / avg_launch_s /
                                              8.0e12, 4)
            if traffic and avg_launch_s > 0 else None,
        },
    }

    if not args.no_cpu and not dense:
        import oracle
        n_it = args.cpu_iters or max(1, min(st.iterations, 10))
        t = time.perf_counter()
        r = oracle.fit(X, C0, split(args.variant)[0], n_it)
        cpu_s = time.perf_counter() - t
        out["cpu_baseline"] = {
            "value": round(r.iterations / cpu_s, 4),
            "unit": "iters/s",
            "cores": oracle.threads(),
            "kind": "oracle",
            "sample": "FP64 oracle %s on the same %s input, first %d assignment steps "
                      "(%.1f s)" % (args.variant, name, r.iterations, cpu_s),
        }
    elif not args.no_cpu and dense:
        import oracle
        # about 10 s of oracle work on 16 host cores: 320,000 evenly spaced rows
        m = min(n_rows, 320000)
        sub = np.arange(0, n_rows, n_rows // m)[:m]
        Xs = Xh[sub]
        rp = np.arange(0, Xs.size + 1, Xs.shape[1], dtype=np.int64)
        Xc = datagen.CSR(Xs.shape[0], Xs.shape[1], rp,
                         np.tile(np.arange(Xs.shape[1], dtype=np.int32), Xs.shape[0]),
                         Xs.ravel())
        t = time.perf_counter()
        oracle.assign(Xc, C0.astype(np.float64))
        cpu_s = time.perf_counter() - t
        step_s = cpu_s * n_rows / len(sub)
        out["cpu_baseline"] = {
            "value": round(1.0 / step_s, 5),
            "unit": "iters/s",
            "cores": oracle.threads(),
            "kind": "oracle",
            "sample": "FP64 oracle assignment step on %d of %d rows (%.1f s), scaled to all "
                      "rows" % (len(sub), n_rows, cpu_s),
        }
    print(json.dumps(out), flush=True)


def run_batched(args, torch, dev, datagen, skm):
    """c5: 256 independent sparse problems (n_b log-normal in [1e3, 5e4],
    k_b = 8 * U{1..32}, d = 20,000, ~80 stored entries per row, 30 steps at
    most), solved by one skm_fit_batched call against the plain GPU Lloyd fit
    of each problem one after another."""
    t0 = time.time()
    insts = datagen.batched_instances()
    probs = []
    for p in insts:
        Xd = skm.DeviceCSR.from_host(p.X, dev)
        C0 = torch.from_numpy(datagen.init_centers_csr(p.X, p.init)).to(dev)
        probs.append((Xd, p.k, C0, args.max_iter or p.max_iter))
    n_tot = sum(p.X.n for p in insts)
    nnz_tot = sum(p.X.nnz for p in insts)
    log("generated c5: %d problems, %d rows, %d stored entries in %.1fs" % (
        len(insts), n_tot, nnz_tot, time.time() - t0))
    variant = args.variant

    def total_steps(res):
        return sum(r[2].iterations for r in res)

    # plain GPU FP32 Lloyd, one problem after another on the current stream
    base_res = None
    base_s = None
    if not args.skip_baseline:
        ws_size = max(skm.workspace_size(X, k, "lloyd") for X, k, _, _ in probs)
        ws = torch.empty(ws_size, dtype=torch.uint8, device=dev)

        def sequential():
            out = []
            for X, k, C0, it in probs:
                a, C, _, st = skm.fit(X, k, C0, "lloyd", it, workspace=ws, want_centers=False,
                                      per_iter=False)
                out.append((a, C, st))
            return out
        sequential()
        torch.cuda.synchronize()
        t = time.perf_counter()
        base_res = sequential()
        torch.cuda.synchronize()
        base_s = time.perf_counter() - t
        log("sequential lloyd: %d steps, %.1f ms" % (total_steps(base_res), base_s * 1e3))

    # worker count: the requested one, or the fastest of a short sweep
    sweep = {}
    workers = args.workers
    if workers == 0:
        for w in (1, 2, 4, 8):
            skm.fit_batched(probs, variant, workers=w, want_centers=False)
            torch.cuda.synchronize()
            t = time.perf_counter()
            skm.fit_batched(probs, variant, workers=w, want_centers=False)
            torch.cuda.synchronize()
            sweep[w] = round((time.perf_counter() - t) * 1e3, 3)
            log("batched %s workers=%d: %.1f ms" % (variant, w, sweep[w]))
        workers = min(sweep, key=sweep.get)
    bws = torch.empty(skm.batched_workspace_size(probs, variant, workers=workers),
                      dtype=torch.uint8, device=dev)
    for _ in range(args.warmup):
        skm.fit_batched(probs, variant, workers=workers, workspace=bws, want_centers=False,
                        profile=1)
    torch.cuda.synchronize()
    runs = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        runs.append(skm.fit_batched(probs, variant, workers=workers, workspace=bws,
                                    want_centers=False, profile=1))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    res = runs[-1]
    steps = total_steps(res)
    identical = None
    if base_res is not None:
        identical = all(torch.equal(a, b[0]) and s.iterations == b[2].iterations
                        for (a, _, s), b in zip(res, base_res))
    value = steps * args.steps / elapsed
    sims = sum(r[2].sims_point_center for run in runs for r in run)
    lloyd_sims = sum(X.n * k * r[2].iterations for run in runs
                     for (X, k, _, _), r in zip(probs, run))
    launches = sum(r[2].sim_kernel_launches for run in runs for r in run)
    kern_ms = sum(r[2].sim_kernel_ms for run in runs for r in run)
    flops = sum(2.0 * k * r[2].sim_kernel_nnz for run in runs
                for (X, k, _, _), r in zip(probs, run))
    avg_launch_s = kern_ms / 1e3 / max(launches, 1)
    achieved = flops / max(launches, 1) / avg_launch_s / 1e12 if avg_launch_s > 0 else 0.0
    traffic = measured_traffic("k_assign_csr", "c5", variant)
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c5: %d batched spherical k-means problems (%s), n_b log-normal "
                               "in [1e3, 5e4] (sum %d), k_b in 8..256, d=20000, nnz %d, at most "
                               "%d steps each, one skm_fit_batched call per step" % (
                                   len(probs), variant, n_tot, nnz_tot, probs[0][3]),
                   "variant": variant, "problems": len(probs), "rows": n_tot, "nnz": nnz_tot,
                   "workers": workers, "parallelism": "single GPU"},
        "assignment_steps_per_call": steps,
        "identical_assignments_to_lloyd": identical,
        "speedup_vs_sequential_gpu_lloyd": None if base_s is None else
        round(base_s / (elapsed / args.steps), 3),
        "sequential_gpu_lloyd": None if base_s is None else {
            "ms": round(base_s * 1e3, 3), "iters_per_s": round(total_steps(base_res) / base_s, 3)},
        "worker_sweep_ms": sweep,
        "sims_per_s_raw": round(sims / elapsed, 1),
        "sims_per_s_lloyd_equiv": round(lloyd_sims / elapsed, 1),
        "pruned_fraction": round(1.0 - sims / max(lloyd_sims, 1), 4),
        "roofline": {
            "kernel": "k_assign_csr", "bound": "alu", "achieved": round(achieved, 3),
            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "traffic": traffic["bytes_per_launch"] if traffic else None,
            "traffic_source": traffic["file"] if traffic else None,
            "avg_launch_us": round(avg_launch_s * 1e6, 3), "launches": launches,
        },
    }
    if not args.no_cpu:
        import oracle
        # bounded sample: the first problems in index order until ~10 s of
        # oracle work, each fitted to the same step count as on the GPU;
        # scaled to the whole batch by stored entries x k x steps
        work = [X.nnz * k * r[2].iterations for (X, k, _, _), r in zip(probs, res)]
        t = time.perf_counter()
        done = 0
        w_done = 0.0
        for b, p in enumerate(insts):
            C0 = datagen.init_centers_csr(p.X, p.init)
            oracle.fit(p.X, C0, variant, res[b][2].iterations)
            done += 1
            w_done += work[b]
            if time.perf_counter() - t > 10.0:
                break
        cpu_s = time.perf_counter() - t
        est_all = cpu_s * sum(work) / max(w_done, 1.0)
        out["cpu_baseline"] = {
            "value": round(steps / est_all, 4),
            "unit": "iters/s",
            "cores": oracle.threads(),
            "kind": "oracle",
            "sample": "FP64 oracle %s on the first %d of %d problems (%.1f s), scaled to the "
                      "batch by stored entries x k x steps" % (variant, done, len(insts), cpu_s),
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
