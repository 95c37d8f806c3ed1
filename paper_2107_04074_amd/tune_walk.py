"""Row-walk tuner (needs a GPU).  Times (HIP events around every assignment
step's walk) the alternatives of the FP32 centre copy's row walk on seeded
synthetic tf-idf rows, for the three row-length classes of the table (6,
30 and 80 stored entries per row on average), and writes
csrc/walk_tuning.h:

  - layouts, padded widths kp = 32 ... 512 (20,000 columns; whole rows):
    skm_options.walk_layout 1 (default) against 2 (kp <= 64: one row per
    wave; above: four rows per wave); the alternative is taken when at
    least 2% faster;
  - slicing, kp = 512, 1024, 2048, 4096 (10,000 columns, so every copy stays
    below the 256 MB the library always slices above), per variant family
    (Lloyd and Hamerly; simplified and full Elkan; Yin-Yang): chunk_walk 1
    (256 centres per launch) against 2 (whole rows in one launch, at kp =
    512 in the layout just measured for Lloyd and Hamerly); whole rows are
    taken when at least 2% faster.

Each cell times one fit of every variant of its family (layouts: Lloyd and
Hamerly; k = 3 kp / 4, 15 steps at most), best of the repetitions.  Both
alternatives must give identical assignments (the exact argmax does not
depend on the FP32 summation order or the launch split); the tuner stops
with an error if they do not.

    python -m paper_2107_04074_amd.tune_walk [--out PATH] [--reps 5]

Rebuild the library afterwards (python -m paper_2107_04074_amd.build).

The tables hold the plan's first choice.  Where they pick whole rows, a fit
still times slices against them in its first steps when the rows' structure
rather than their shape decides (Elkan and Yin-Yang: packed slices for the
steps with tests; Lloyd and Hamerly: copies of 64 MB or more, larger than
the ones measured here) and keeps the faster.
"""
from __future__ import annotations

import argparse
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
# (class, mean stored entries per row of the tuning matrix); a matrix falls
# into the first class whose bound exceeds its mean
ROW_CLASSES = ((0, 6.0), (1, 30.0), (2, 80.0))
ROW_BOUNDS = (20, 48)
LAYOUT_WIDTHS = (32, 64, 128, 256, 512)  # kp = 16 has only the default layout
CHUNK_WIDTHS = (512, 1024, 2048, 4096)
N_ROWS, STEPS, SEED = 100_000, 15, 20_240_611
D_LAYOUT, D_CHUNK = 20_000, 10_000
FAMILIES = (("lloyd", "hamerly"), ("simp_elkan", "elkan"), ("yinyang",))


def _walk_times(skm, torch, X, k, C0, ws, reps, variants, **opt):
    """Best row-walk time (profile = 1) over `reps` of a fit of each variant,
    summed, in seconds, and the assignments."""
    best = [1e30] * len(variants)
    out = []
    for _ in range(reps):
        out = []
        for i, var in enumerate(variants):
            a, _, _, st = skm.fit(X, k, C0, var, STEPS, workspace=ws, want_centers=False,
                                  per_iter=False, profile=1, **opt)
            torch.cuda.synchronize()
            best[i] = min(best[i], st.sim_kernel_ms * 1e-3)
            out.append(a)
    return sum(best), out


def _compare(skm, torch, X, Xh, k, reps, variants, opt_a, opt_b, what, datagen, dev):
    init = datagen.init_rows(Xh.n, k, SEED + k)
    C0 = torch.from_numpy(datagen.init_centers_csr(Xh, init)).to(dev)
    size = max(skm.workspace_size(X, k, v, **o) for v in variants for o in (opt_a, opt_b))
    ws = torch.empty(size, dtype=torch.uint8, device=dev)
    _walk_times(skm, torch, X, k, C0, ws, 1, variants, **opt_a)  # warm-up of every kernel
    _walk_times(skm, torch, X, k, C0, ws, 1, variants, **opt_b)
    ta, aa = _walk_times(skm, torch, X, k, C0, ws, reps, variants, **opt_a)
    tb, ab = _walk_times(skm, torch, X, k, C0, ws, reps, variants, **opt_b)
    for x, y in zip(aa, ab):
        if not torch.equal(x, y):
            raise RuntimeError("%s: the alternatives disagree at k=%d" % (what, k))
    return ta, tb


def tune(out_path: str, reps: int = 5):
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    import datagen
    from paper_2107_04074_amd import skm

    dev = torch.device("cuda:0")
    layout = [[0] * 6 for _ in ROW_CLASSES]
    chunk = [[[1] * 4 for _ in ROW_CLASSES] for _ in FAMILIES]
    notes = []
    for rc, mean in ROW_CLASSES:
        for d, widths in ((D_LAYOUT, LAYOUT_WIDTHS), (D_CHUNK, CHUNK_WIDTHS)):
            if d == D_CHUNK:
                # whole rows at kp = 512 in the layout just measured
                whole512 = layout[rc][5] + 1
            Xh = datagen.sparse_tfidf(N_ROWS, d, mean, SEED + rc)
            X = skm.DeviceCSR.from_host(Xh, dev)
            for kp in widths:
                k = 3 * kp // 4
                if d == D_LAYOUT:
                    t0, t1 = _compare(skm, torch, X, Xh, k, reps, FAMILIES[0],
                                      {"walk_layout": 1, "chunk_walk": 2},
                                      {"walk_layout": 2, "chunk_walk": 2}, "layouts",
                                      datagen, dev)
                    pick = 1 if t1 < 0.98 * t0 else 0
                    layout[rc][kp.bit_length() - 5] = pick
                    note = ("layout kp %4d, mean row %2d, d %d: %.3f ms default, %.3f ms "
                            "alternative -> %d" % (kp, int(mean), d, t0 * 1e3, t1 * 1e3, pick))
                    notes.append(note)
                    print(note, flush=True)
                    continue
                for fam, variants in enumerate(FAMILIES):
                    whole = {"chunk_walk": 2}
                    if kp == 512 and fam == 0:
                        whole["walk_layout"] = whole512
                    t0, t1 = _compare(skm, torch, X, Xh, k, reps, variants, {"chunk_walk": 1},
                                      whole, "slicing", datagen, dev)
                    pick = 0 if t1 < 0.98 * t0 else 1
                    chunk[fam][rc][kp.bit_length() - 10] = pick
                    note = ("slices %-18s kp %4d, mean row %2d, d %d: %.3f ms sliced, %.3f ms "
                            "whole rows -> %d" % ("+".join(variants), kp, int(mean), d,
                                                  t0 * 1e3, t1 * 1e3, pick))
                    notes.append(note)
                    print(note, flush=True)
            del X
            torch.cuda.empty_cache()
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", "gpu").split(":")[0]
    _write(out_path, layout, chunk, notes,
           "%s, %d compute units" % (arch, props.multi_processor_count))
    return layout, chunk


def _rows(table):
    return ",\n".join("    {" + ", ".join(str(v) for v in r) + "}" for r in table)


def _write(path: str, layout, chunk, notes, device: str) -> None:
    body = [
        "// Row-walk choices of the FP32 centre copy, per row-length class (0: under",
        "// %d stored entries per row on average, 1: under %d, 2: more).  Written by" % ROW_BOUNDS,
        "// paper_2107_04074_amd/tune_walk.py on %s, %d seeded" % (device, N_ROWS),
        "// tf-idf rows, k = 3 kp / 4, summed row-walk time of one fit of every variant",
        "// of the family (%d steps at most, HIP events), best of the repetitions:" % STEPS,
    ]
    body += ["//   " + n for n in notes]
    body += [
        "#pragma once",
        "",
        "namespace skm {",
        "// Layout per padded width kp = 16, 32, ..., 512 (index log2(kp) - 4) of a",
        "// whole-row walk.  0: the default layout (k <= 64: a group of kp/4 lanes per",
        "// row, several rows per wave; k in (64, 512]: one row per wave, in two",
        "// sub-waves of 32 lanes at kp = 128, one 16-byte unit per lane at 256, two",
        "// at 512); 1: the alternative (k in (16, 64]: one row per wave in sub-waves",
        "// of kp/4 lanes, 64/(kp/4) stored entries per gather instruction; k in",
        "// (64, 512]: a group of 16 lanes per row, four rows per wave, kp/64 16-byte",
        "// units per lane).",
        "constexpr int kWalkTuneWidths = 6;",
        "constexpr int kWalkTuneRowClasses = 3;",
        "// mean stored entries per row below which a matrix is in class 0, 1",
        "constexpr int kWalkTuneRowBound[kWalkTuneRowClasses - 1] = {%d, %d};" % ROW_BOUNDS,
        "constexpr int kWalkTune[kWalkTuneRowClasses][kWalkTuneWidths] = {",
        _rows(layout),
        "};",
        "// Slicing per variant family (0: Lloyd and Hamerly, 1: Elkan, 2: Yin-Yang),",
        "// row-length class and padded width kp = 512, 1024, 2048, 4096 (index",
        "// log2(kp) - 9) while the copy fits the last-level cache: 1 = walk 256",
        "// centres per launch, 0 = whole rows in one launch.",
        "constexpr int kChunkTuneFamilies = 3;",
        "constexpr int kChunkTuneWidths = 4;",
        "constexpr int kChunkTune[kChunkTuneFamilies][kWalkTuneRowClasses][kChunkTuneWidths] = {",
        ",\n".join("    {" + ", ".join("{" + ", ".join(str(v) for v in r) + "}" for r in fam) + "}"
                   for fam in chunk),
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
    layout, chunk = tune(a.out, a.reps)
    print("wrote %s: layouts %s, slicing %s" % (a.out, layout, chunk))


if __name__ == "__main__":
    main()
