"""Row-walk layout tuner (needs a GPU): times (HIP events around every
assignment step's walk) both layouts of the FP32 centre copy's row walk
(skm_options.walk_layout 1 = default, 2 = alternative) on seeded
synthetic tf-idf rows for every padded width
kp = 32, 64, 128, 256 and both row-length classes of the table (short:
24 stored entries per row on average, long: 80), and writes
csrc/walk_tuning.h with the faster layout of each cell.  The alternative is
taken only when it is at least 2% faster.  Both layouts must give identical
assignments (the exact argmax does not depend on the FP32 summation order);
the tuner stops with an error if they do not.

    python -m paper_2107_04074_amd.tune_walk [--out PATH] [--reps 5]

Rebuild the library afterwards (python -m paper_2107_04074_amd.build).
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROW_CLASSES = ((0, 24.0), (1, 80.0))   # (class, mean stored entries per row)
WIDTHS = (32, 64, 128, 256)             # kp; kp = 16 has only the default layout
N_ROWS, D_COLS, STEPS, SEED = 20_000, 20_000, 15, 20_240_611


def _time_fits(skm, torch, X, k, C0, layout, ws, reps):
    """Best row-walk time (HIP events around every step's walk, profile = 1)
    over `reps` of a Lloyd fit and of a Hamerly fit, in seconds, and the
    assignments."""
    best = [1e30, 1e30]
    out = []
    for _ in range(reps):
        out = []
        for i, var in enumerate(("lloyd", "hamerly")):
            a, _, _, st = skm.fit(X, k, C0, var, STEPS, workspace=ws, want_centers=False,
                                  per_iter=False, walk_layout=layout, profile=1)
            torch.cuda.synchronize()
            best[i] = min(best[i], st.sim_kernel_ms * 1e-3)
            out.append(a)
    return best, out


def tune(out_path: str, reps: int = 5) -> list:
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    import datagen
    from paper_2107_04074_amd import skm

    dev = torch.device("cuda:0")
    table = [[0] * 5 for _ in ROW_CLASSES]
    notes = []
    for rc, mean in ROW_CLASSES:
        Xh = datagen.sparse_tfidf(N_ROWS, D_COLS, mean, SEED + rc)
        X = skm.DeviceCSR.from_host(Xh, dev)
        for kp in WIDTHS:
            k = 3 * kp // 4
            init = datagen.init_rows(Xh.n, k, SEED + kp)
            C0 = torch.from_numpy(datagen.init_centers_csr(Xh, init)).to(dev)
            ws = torch.empty(skm.workspace_size(X, k, "hamerly"), dtype=torch.uint8, device=dev)
            _time_fits(skm, torch, X, k, C0, 1, ws, 1)  # warm-up of both kernels
            _time_fits(skm, torch, X, k, C0, 2, ws, 1)
            t0, a0 = _time_fits(skm, torch, X, k, C0, 1, ws, reps)
            t1, a1 = _time_fits(skm, torch, X, k, C0, 2, ws, reps)
            for x, y in zip(a0, a1):
                if not torch.equal(x, y):
                    raise RuntimeError("layouts disagree at kp=%d, mean row %g" % (kp, mean))
            s0, s1 = sum(t0), sum(t1)
            pick = 1 if s1 < 0.98 * s0 else 0
            c = kp.bit_length() - 5
            table[rc][c] = pick
            note = ("kp %4d, mean row %2d: row walks %.3f ms (default), %.3f ms (alternative) "
                    "-> %d" % (kp, int(mean), s0 * 1e3, s1 * 1e3, pick))
            notes.append(note)
            print(note, flush=True)
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", "gpu").split(":")[0]
    _write(out_path, table, notes, "%s, %d compute units" % (arch, props.multi_processor_count))
    return table


def _write(path: str, table, notes, device: str) -> None:
    rows = ",\n".join("    {" + ", ".join(str(v) for v in r) + "}" for r in table)
    body = [
        "// Row-walk layout of the FP32 centre copy for Lloyd and Hamerly fits, per",
        "// padded width kp = 16, 32, 64, 128, 256 (index log2(kp) - 4) and row-length",
        "// class (0: under 48 stored entries per row on average, 1: 48 or more).",
        "// 0: the default layout (k <= 64: a group of kp/4 lanes per row, several rows",
        "// per wave; k in (64, 256]: one row per wave, one 16-byte unit per lane);",
        "// 1: the alternative (k in (16, 64]: one row per wave in sub-waves of kp/4",
        "// lanes, 64/(kp/4) stored entries per gather instruction; k in (64, 256]:",
        "// one row per wave, two 16-byte units per lane, sub-waves of kp/8 lanes).",
        "// Written by paper_2107_04074_amd/tune_walk.py on %s:" % device,
        "// %d x %d seeded tf-idf rows, k = 3 kp / 4, row-walk time of a Lloyd and" % (N_ROWS, D_COLS),
        "// a Hamerly fit of %d steps at most (HIP events), best of the repetitions:" % STEPS,
    ]
    body += ["//   " + n for n in notes]
    body += [
        "#pragma once",
        "",
        "namespace skm {",
        "constexpr int kWalkTuneWidths = 5;",
        "constexpr int kWalkTuneRowClasses = 2;",
        "constexpr int kWalkTuneShortRow = 48;  // mean stored entries per row below: class 0",
        "constexpr int kWalkTune[kWalkTuneRowClasses][kWalkTuneWidths] = {",
        rows,
        "};",
        "}  // namespace skm",
        "",
    ]
    with open(path, "w") as f:
        f.write("\n".join(body))


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=os.path.join(HERE, "csrc", "walk_tuning.h"))
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args(argv)
    table = tune(a.out, a.reps)
    print("wrote %s: %s" % (a.out, np.array(table).tolist()))


if __name__ == "__main__":
    main()
