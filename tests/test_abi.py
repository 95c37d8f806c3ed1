"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid arguments before touching a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2107_04074_amd import skm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "skm.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(skm.LIB_PATH):
        from paper_2107_04074_amd import build
        build.build()
    return skm.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(skm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_binding_exports():
    assert declared_functions() == sorted(skm.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", skm.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (skm_[a-z0-9_]+)$", out, flags=re.M))
    for name in declared_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None


def test_header_compiles_as_c(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "skm.h"\nint main(void){skm_stats s; (void)s; '
                   'return skm_version() > 0 ? 0 : 1;}\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-I",
                    os.path.join(ROOT, "include"), str(src)], check=True)


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the structs have the header's sizes/offsets."""
    src = tmp_path / "l.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "skm.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(skm_matrix), '
                   'sizeof(skm_options), sizeof(skm_stats), offsetof(skm_stats, per_iter_len), '
                   'offsetof(skm_matrix, ld)); return 0;}\n')
    exe = tmp_path / "l"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals == [ctypes.sizeof(skm.SkmMatrix), ctypes.sizeof(skm.SkmOptions),
                    ctypes.sizeof(skm.SkmStats), skm.SkmStats.per_iter_len.offset,
                    skm.SkmMatrix.ld.offset]


def _fake_csr(n=10, d=20, nnz=30):
    # host pointers that are never dereferenced by the validation paths
    return skm.SkmMatrix(skm.CSR_F32, 0, n, d, nnz, 0x1000, 0x2000, 0x3000, None, 0)


def test_invalid_arguments_are_rejected(lib):
    m = _fake_csr()
    o = skm.SkmOptions()
    st = skm.SkmStats()
    # k out of range
    assert lib.skm_workspace_size(ctypes.byref(m), 0, 0, None) == 0
    assert b"k" in lib.skm_last_error()
    assert lib.skm_workspace_size(ctypes.byref(m), 11, 0, None) == 0
    # bad variant
    assert lib.skm_workspace_size(ctypes.byref(m), 3, 9, None) == 0
    assert b"variant" in lib.skm_last_error()
    # valid request has a positive size that grows with the variant's state
    lloyd = lib.skm_workspace_size(ctypes.byref(m), 3, skm.LLOYD, ctypes.byref(o))
    ham = lib.skm_workspace_size(ctypes.byref(m), 3, skm.HAMERLY, ctypes.byref(o))
    elk = lib.skm_workspace_size(ctypes.byref(m), 3, skm.ELKAN, ctypes.byref(o))
    assert 0 < lloyd < ham and lloyd < elk
    # fit: NULL init, max_iter 0, bad bound_form: rejected before any GPU call
    rc = lib.skm_fit(ctypes.byref(m), 3, None, 0, 5, None, None, 0, 0x4000, None, None,
                     ctypes.byref(st), None)
    assert rc == skm.ERR_INVALID_ARG
    rc = lib.skm_fit(ctypes.byref(m), 3, 0x5000, 0, 0, None, None, 0, 0x4000, None, None,
                     ctypes.byref(st), None)
    assert rc == skm.ERR_INVALID_ARG and b"max_iter" in lib.skm_last_error()
    bad = skm.SkmOptions(7, 0, 0, 0, 0.0)
    rc = lib.skm_fit(ctypes.byref(m), 3, 0x5000, 0, 5, ctypes.byref(bad), None, 0, 0x4000,
                     None, None, ctypes.byref(st), None)
    assert rc == skm.ERR_INVALID_ARG
    bad = skm.SkmOptions(0, 0, 0, 0, 0.0, None, None, None, 2)
    rc = lib.skm_fit(ctypes.byref(m), 3, 0x5000, 0, 5, ctypes.byref(bad), None, 0, 0x4000,
                     None, None, ctypes.byref(st), None)
    assert rc == skm.ERR_INVALID_ARG and b"schedule" in lib.skm_last_error()
    for layout, cw, what in ((3, 0, b"walk_layout"), (-1, 0, b"walk_layout"),
                             (0, 3, b"chunk_walk"), (1, -1, b"chunk_walk")):
        bad = skm.SkmOptions(0, 0, 0, 0, 0.0, None, None, None, 0, 0, layout, cw)
        rc = lib.skm_fit(ctypes.byref(m), 3, 0x5000, 0, 5, ctypes.byref(bad), None, 0, 0x4000,
                         None, None, ctypes.byref(st), None)
        assert rc == skm.ERR_INVALID_ARG and what in lib.skm_last_error()
    bad = skm.SkmOptions(0, 0, 0, 0, 0.0, None, None, None, 0, 0, 0, 4)
    assert lib.skm_workspace_size(ctypes.byref(m), 3, skm.HAMERLY, ctypes.byref(bad)) == 0
    assert b"chunk_walk" in lib.skm_last_error()
    # undersized caller workspace
    rc = lib.skm_fit(ctypes.byref(m), 3, 0x5000, 0, 5, None, 0x6000, 16, 0x4000, None, None,
                     ctypes.byref(st), None)
    assert rc == skm.ERR_OUT_OF_MEMORY
    # empty / unknown formats
    m0 = _fake_csr(n=0)
    assert lib.skm_workspace_size(ctypes.byref(m0), 1, 0, None) == 0
    md = skm.SkmMatrix(skm.DENSE_F32, 0, 10, 20, 0, None, None, None, 0x1000, 20)
    m9 = skm.SkmMatrix(9, 0, 10, 20, 0, None, None, None, None, 0)
    assert lib.skm_workspace_size(ctypes.byref(m9), 2, 0, None) == 0
    assert b"format" in lib.skm_last_error()
    del md
    # k beyond the largest supported geometry
    big = _fake_csr(n=10000)
    assert lib.skm_workspace_size(ctypes.byref(big), 5000, 0, None) == 0
    assert lib.skm_status_string(skm.ERR_UNSUPPORTED) == b"unsupported"


def test_batched_arguments_are_rejected(lib):
    """skm_fit_batched validates every problem before any GPU call; its
    workspace is one slot (the largest problem's need) per worker."""
    ms = (skm.SkmMatrix * 3)(_fake_csr(), _fake_csr(n=40), _fake_csr())
    ks = (ctypes.c_int32 * 3)(3, 5, 2)
    its = (ctypes.c_int32 * 3)(5, 5, 5)
    ptrs = (ctypes.c_void_p * 3)(0x5000, 0x6000, 0x7000)
    st = (skm.SkmStats * 3)()
    one = lib.skm_fit_batched_workspace_size(3, ms, ks, skm.HAMERLY, None, 1)
    three = lib.skm_fit_batched_workspace_size(3, ms, ks, skm.HAMERLY, None, 3)
    biggest = max(lib.skm_workspace_size(ctypes.byref(ms[b]), ks[b], skm.HAMERLY, None)
                  for b in range(3))
    assert one >= biggest and three == 3 * one
    # workers = 0 (lockstep): every problem keeps its own state, plus the
    # shared views, walk arguments, control blocks and work items
    lock = lib.skm_fit_batched_workspace_size(3, ms, ks, skm.HAMERLY, None, 0)
    singles = sum(lib.skm_workspace_size(ctypes.byref(ms[b]), ks[b], skm.HAMERLY, None)
                  for b in range(3))
    assert lock >= singles
    # variants without a lockstep form take the host-thread slots (at most
    # one worker per problem)
    assert (lib.skm_fit_batched_workspace_size(3, ms, ks, skm.ELKAN, None, 0) ==
            lib.skm_fit_batched_workspace_size(3, ms, ks, skm.ELKAN, None, 3))
    # a bad problem is named
    ks_bad = (ctypes.c_int32 * 3)(3, 0, 2)
    assert lib.skm_fit_batched_workspace_size(3, ms, ks_bad, skm.HAMERLY, None, 1) == 0
    assert b"problem 1" in lib.skm_last_error()
    assert lib.skm_fit_batched(0, ms, ks, ptrs, 0, its, None, 0, None, 0, ptrs, None, st,
                               None) == skm.ERR_INVALID_ARG
    its_bad = (ctypes.c_int32 * 3)(5, 0, 5)
    rc = lib.skm_fit_batched(3, ms, ks, ptrs, 0, its_bad, None, 0, None, 0, ptrs, None, st,
                             None)
    assert rc == skm.ERR_INVALID_ARG and b"problem 1" in lib.skm_last_error()
    rc = lib.skm_fit_batched(3, ms, ks, None, 0, its, None, 0, None, 0, ptrs, None, st, None)
    assert rc == skm.ERR_INVALID_ARG
    rc = lib.skm_fit_batched(3, ms, ks, ptrs, 0, its, None, -1, None, 0, ptrs, None, st, None)
    assert rc == skm.ERR_INVALID_ARG
    rc = lib.skm_fit_batched(3, ms, ks, ptrs, 0, its, None, 1, 0x8000, 16, ptrs, None, st, None)
    assert rc == skm.ERR_OUT_OF_MEMORY


def test_seeding_and_warm_start_arguments_are_rejected(lib):
    m = _fake_csr(n=10)
    u = (ctypes.c_double * 3)(0.1, 0.5, 0.9)
    assert lib.skm_seed_workspace_size(ctypes.byref(m), 3) > 0
    assert lib.skm_seed_workspace_size(ctypes.byref(m), 11) == 0  # k > n
    md = skm.SkmMatrix(skm.DENSE_F32, 0, 10, 20, 0, None, None, None, 0x1000, 20)
    assert lib.skm_seed_workspace_size(ctypes.byref(md), 3) > 0  # dense rows are accepted
    wide = skm.SkmMatrix(skm.DENSE_F32, 0, 10, 300, 0, None, None, None, 0x1000, 300)
    assert lib.skm_seed_workspace_size(ctypes.byref(wide), 3) == 0
    assert b"d <= 256" in lib.skm_last_error()
    call = lambda alpha, uu: lib.skm_seed_kmeanspp(ctypes.byref(m), 3, alpha, uu, 0x5000, None,
                                                   None, None, None, None, 0, None)
    assert call(0.5, u) == skm.ERR_INVALID_ARG and b"alpha" in lib.skm_last_error()
    bad = (ctypes.c_double * 3)(0.1, 1.0, 0.2)
    assert call(1.0, bad) == skm.ERR_INVALID_ARG and b"uniform 1" in lib.skm_last_error()
    neg = (ctypes.c_double * 3)(-0.1, 0.5, 0.2)
    assert call(1.0, neg) == skm.ERR_INVALID_ARG
    assert call(1.0, None) == skm.ERR_INVALID_ARG
    # warm start: all three arrays or none (CSR and dense alike)
    st = skm.SkmStats()
    o = skm.SkmOptions(0, 0, 0, 0, 0.0, 0x7000, None, None)
    for mm in (m, md):
        rc = lib.skm_fit(ctypes.byref(mm), 3, 0x5000, 0, 5, ctypes.byref(o), None, 0, 0x4000,
                         None, None, ctypes.byref(st), None)
        assert rc == skm.ERR_INVALID_ARG and b"warm" in lib.skm_last_error()


def test_afkmc2_arguments_are_rejected(lib):
    m = _fake_csr(n=10)
    assert lib.skm_seed_afkmc2_workspace_size(ctypes.byref(m), 3, 4) > 0
    assert lib.skm_seed_afkmc2_workspace_size(ctypes.byref(m), 3, 0) == 0
    assert b"chain" in lib.skm_last_error()
    assert lib.skm_seed_afkmc2_workspace_size(ctypes.byref(m), 11, 4) == 0
    good = (ctypes.c_double * 15)(*([0.5] * 15))  # 1 + 2 * (2 * 4 - 1)
    rc = lib.skm_seed_afkmc2(ctypes.byref(m), 3, 4, 0.9, good, 0x5000, None, None, 0, None)
    assert rc == skm.ERR_INVALID_ARG and b"alpha" in lib.skm_last_error()
    bad = (ctypes.c_double * 15)(*([0.5] * 14 + [1.0]))
    rc = lib.skm_seed_afkmc2(ctypes.byref(m), 3, 4, 1.0, bad, 0x5000, None, None, 0, None)
    assert rc == skm.ERR_INVALID_ARG and b"uniform 14" in lib.skm_last_error()
    rc = lib.skm_seed_afkmc2(ctypes.byref(m), 3, 4, 1.0, good, None, None, None, 0, None)
    assert rc == skm.ERR_INVALID_ARG


def test_product_path_refuses_without_library(monkeypatch, tmp_path):
    """The binding never falls back to CPU code: a missing library raises."""
    monkeypatch.setattr(skm, "_lib", None)
    with pytest.raises(RuntimeError):
        skm.load(str(tmp_path / "missing.so"))


def test_centre_copy_offsets_fit_32_bits(lib):
    """The row kernels address the centre-minor copy with 32-bit element
    offsets (column * k_padded + centre): shapes with d * k_padded >= 2^32 are
    refused on the host (SKM_ERR_UNSUPPORTED), never launched."""
    o = skm.SkmOptions()
    ok = _fake_csr(n=5000, d=(1 << 20) - 1)
    assert lib.skm_workspace_size(ctypes.byref(ok), 4096, skm.LLOYD, ctypes.byref(o)) > 0
    for d, k in (((1 << 20), 4096), ((1 << 21), 2048), ((1 << 22), 1000)):
        m = _fake_csr(n=5000, d=d)
        assert lib.skm_workspace_size(ctypes.byref(m), k, skm.LLOYD, ctypes.byref(o)) == 0
        assert b"2^32" in lib.skm_last_error()
        assert lib.skm_assign_workspace_size(ctypes.byref(m), k) == 0
        st = skm.SkmStats()
        rc = lib.skm_fit(ctypes.byref(m), k, 0x5000, skm.HAMERLY, 5, None, None, 0, 0x4000,
                         None, None, ctypes.byref(st), None)
        assert rc == skm.ERR_UNSUPPORTED
        rc = lib.skm_assign(ctypes.byref(m), k, 0x5000, 0x4000, None, None, None, 0, None)
        assert rc == skm.ERR_UNSUPPORTED


def test_walk_tuning_table_is_well_formed():
    """The compiled row-walk tables (written by tune_walk.py): layouts, one
    entry per row-length class (three) and padded width kp = 16 ... 512,
    each 0 or 1, kp = 16 (no alternative layout) always 0; slicing, one
    entry per variant family, class and kp = 512 ... 4096, each 0 or 1."""
    path = os.path.join(os.path.dirname(skm.__file__), "csrc", "walk_tuning.h")
    text = open(path).read()
    body = re.search(r"kWalkTune\[kWalkTuneRowClasses\]\[kWalkTuneWidths\]\s*=\s*\{(.*?)\};",
                     text, re.S).group(1)
    rows = [[int(v) for v in r.split(",")] for r in re.findall(r"\{([^{}]*)\}", body)]
    assert len(rows) == 3 and all(len(r) == 6 for r in rows)
    assert all(v in (0, 1) for r in rows for v in r)
    assert all(r[0] == 0 for r in rows)
    body = re.search(r"kChunkTune\[kChunkTuneFamilies\]\[kWalkTuneRowClasses\]"
                     r"\[kChunkTuneWidths\]\s*=\s*\{(.*?)\};", text, re.S).group(1)
    rows = [[int(v) for v in r.split(",")] for r in re.findall(r"\{([^{}]*)\}", body)]
    assert len(rows) == 3 * 3 and all(len(r) == 4 for r in rows)
    assert all(v in (0, 1) for r in rows for v in r)


def test_tuner_writes_a_table_the_library_compiles(tmp_path):
    """tune_walk.py's header writer: its output compiles with the names and
    shapes the library reads (checked by static_asserts in a host-only
    translation unit), so a re-measured table drops in without edits."""
    from paper_2107_04074_amd import tune_walk
    hdr = tmp_path / "walk_tuning.h"
    layout = [[0, 1, 0, 1, 0, 1], [0, 0, 1, 1, 0, 0], [0, 0, 0, 0, 0, 1]]
    chunk = [[[1, 0, 1, 0], [0, 1, 1, 1], [0, 0, 0, 1]], [[1, 1, 0, 0], [0, 0, 1, 1], [1, 0, 0, 0]],
             [[0, 0, 0, 0], [1, 1, 1, 1], [0, 1, 0, 1]]]
    tune_walk._write(str(hdr), layout, chunk, ["note"], "test device")
    src = tmp_path / "t.cc"
    src.write_text(
        '#include "walk_tuning.h"\n'
        "using namespace skm;\n"
        "static_assert(kWalkTuneWidths == 6 && kWalkTuneRowClasses == 3, \"\");\n"
        "static_assert(kChunkTuneFamilies == 3 && kChunkTuneWidths == 4, \"\");\n"
        "static_assert(kWalkTune[1][2] == 1 && kWalkTune[0][5] == 1, \"\");\n"
        "static_assert(kChunkTune[0][0][2] == 1 && kChunkTune[1][1][3] == 1, \"\");\n"
        "static_assert(kChunkTune[2][0][0] == 0 && kChunkTune[2][1][0] == 1, \"\");\n"
        "static_assert(kWalkTune[2][5] == 1 && kChunkTune[1][2][0] == 1, \"\");\n"
        "static_assert(kWalkTuneRowBound[0] < kWalkTuneRowBound[1], \"\");\n"
        "int main() { return 0; }\n")
    r = subprocess.run(["g++", "-std=c++17", "-fsyntax-only", "-I", str(tmp_path), str(src)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def _walk_table(name):
    text = open(os.path.join(os.path.dirname(skm.__file__), "csrc", "walk_tuning.h")).read()
    body = re.search(name + r"\[[^=]*=\s*\{(.*?)\};", text, re.S).group(1)
    return [[int(v) for v in r.split(",")] for r in re.findall(r"\{([^{}]*)\}", body)]


def test_slicing_decision_follows_the_table(lib):
    """Whether a fit slices the FP32 centre copy at k > 256 shows in its
    workspace (a 56-byte running record per row when sliced): chunk_walk 1
    and 2 force the two sizes; 0 follows the compiled table for the variant
    family and row-length class, and always slices above a 256 MB copy."""
    bounds = [int(v) for v in re.search(
        r"kWalkTuneRowBound\[[^\]]*\]\s*=\s*\{([^}]*)\}",
        open(os.path.join(os.path.dirname(skm.__file__), "csrc",
                          "walk_tuning.h")).read()).group(1).split(",")]
    table = _walk_table("kChunkTune")  # family-major rows of 4 widths
    n, k = 5000, 500  # k_p = 512: width index 0
    for fam, variant in ((0, skm.HAMERLY), (1, skm.ELKAN), (2, skm.YINYANG)):
        for rc, mean in enumerate((3, 30, 90)):
            assert mean < bounds[rc] if rc < len(bounds) else mean >= bounds[-1]
            for d, big in ((20000, False), (200000, True)):  # copy 41 MB / 410 MB
                m = _fake_csr(n=n, d=d, nnz=n * mean)
                size = {}
                for cw in (0, 1, 2):
                    o = skm.SkmOptions(0, 0, 0, 0, 0.0, None, None, None, 0, 0, 0, cw)
                    size[cw] = lib.skm_workspace_size(ctypes.byref(m), k, variant, ctypes.byref(o))
                assert size[1] > size[2] > 0
                sliced = big or table[3 * fam + rc][0] == 1
                # Elkan and Yin-Yang keep what slices need (running record,
                # Elkan's survival words): they may switch to them mid-fit
                # (not on rows under 20 stored entries: class 0)
                assert size[0] == (size[1] if sliced or (fam > 0 and rc > 0) else size[2]), \
                    (fam, rc, d)
    # Lloyd and Hamerly: a copy of 64 MB or more below 256 MB (here 102 MB,
    # k_p = 512, long rows) slices, or keeps the running record of the slices
    # its first steps time against the table's whole rows
    m = _fake_csr(n=n, d=50000, nnz=n * 90)
    size = {}
    for cw in (0, 1, 2):
        o = skm.SkmOptions(0, 0, 0, 0, 0.0, None, None, None, 0, 0, 0, cw)
        size[cw] = lib.skm_workspace_size(ctypes.byref(m), k, skm.HAMERLY, ctypes.byref(o))
    assert size[0] == size[1] > size[2] > 0
    # 128 < k <= 256: whole rows unless chunk_walk 1 asks Elkan or Yin-Yang
    # for their one packed slice (by default they may switch to it); Lloyd
    # and Hamerly never slice there
    m = _fake_csr(n=n, d=200000, nnz=n * 30)
    for variant, packs in ((skm.HAMERLY, False), (skm.ELKAN, True), (skm.YINYANG, True)):
        size = {}
        for cw in (0, 1, 2):
            o = skm.SkmOptions(0, 0, 0, 0, 0.0, None, None, None, 0, 0, 0, cw)
            size[cw] = lib.skm_workspace_size(ctypes.byref(m), 200, variant, ctypes.byref(o))
        assert size[2] > 0
        assert (size[1] > size[2]) if packs else (size[1] == size[2]), variant
        # the timed choice at this width: Yin-Yang only
        assert size[0] == (size[1] if variant == skm.YINYANG else size[2]), variant
