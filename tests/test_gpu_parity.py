"""GPU parity: libskm (through the C ABI) against the FP64 oracle.

Bar: assignments identical wherever the oracle's top-1/top-2 similarity gap
exceeds 1e-5 (the FP64 re-decision makes them identical far below that; the
number of points inside the band is reported), centres within 1e-6
(Euclidean, unit vectors), objective within 1e-6 relative.  Bounded variants
must reproduce the GPU Lloyd trajectory bit for bit."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

GAP = 1e-5


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


@pytest.fixture(scope="module")
def skm(torch_cuda):
    from paper_2107_04074_amd import skm as s
    s.load()
    return s


def say(*a):
    print(*a, flush=True)


def gap_of(S):
    if S.shape[1] == 1:
        return np.full(S.shape[0], np.inf)
    part = np.partition(S, -2, axis=1)
    return part[:, -1] - part[:, -2]


def check_assign(X, C32, a_gpu, best_gpu, label, terms=None):
    a_ref, s1, s2 = oracle.assign(X, C32.astype(np.float64))
    gap = s1 - s2 if C32.shape[0] > 1 else np.full(X.n, np.inf)
    clear = gap > GAP
    bad = np.flatnonzero(clear & (a_gpu != a_ref))
    say("%s: n=%d k=%d band=%d mismatches(clear)=%d mismatches(all)=%d" %
        (label, X.n, C32.shape[0], int((~clear).sum()), len(bad), int((a_gpu != a_ref).sum())))
    assert len(bad) == 0, bad[:10]
    # every assignment in the band still attains the FP64 maximum to 1e-12
    assert np.all(s1 - np.take_along_axis(
        oracle.sims(X, C32.astype(np.float64), np.arange(X.n)), a_gpu[:, None].astype(np.int64),
        1)[:, 0] <= 1e-12)
    m = X.row_lengths() if terms is None else terms
    err = np.abs(best_gpu.astype(np.float64) - s1)
    assert np.all(err <= (m + 3) * 2.0 ** -24 * 1.02 + 1e-12)
    return a_ref


# ----------------------------------------------------------------- assign

@pytest.mark.parametrize("k", [1, 3, 10, 17, 40, 100, 130, 300, 700, 1500, 2600])
def test_assign_matches_oracle(skm, torch_cuda, k):
    torch = torch_cuda
    say("case assign k=%d" % k)
    X = datagen.sparse_tfidf(2500, 3000, 30.0, 1000 + k)
    rng = np.random.default_rng(k)
    rows = rng.choice(X.n, size=k, replace=k > X.n)
    C = datagen.init_centers_csr(X, rows).astype(np.float64)
    C += 0.05 * np.abs(rng.normal(size=C.shape)) * (rng.random(C.shape) < 0.01)
    C /= np.linalg.norm(C, axis=1, keepdims=True)
    C32 = C.astype(np.float32)
    Xd = skm.DeviceCSR.from_host(X)
    a, best, second = skm.assign(Xd, torch.from_numpy(C32).cuda())
    torch.cuda.synchronize()
    check_assign(X, C32, a.cpu().numpy(), best.cpu().numpy(), "assign k=%d" % k)


def test_assign_ties_and_empty_rows(skm, torch_cuda):
    torch = torch_cuda
    say("case assign ties/empty rows")
    X = datagen.sparse_tfidf(600, 800, 12.0, 77)
    # insert empty rows 0, 5, 599 by rebuilding row_ptr
    lens = np.diff(X.row_ptr)
    lens[[0, 5, 599]] = 0
    keep = np.ones(X.nnz, bool)
    for r in [0, 5, 599]:
        keep[X.row_ptr[r]:X.row_ptr[r + 1]] = False
    rp = np.zeros(X.n + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    Y = datagen.CSR(X.n, X.d, rp, X.col[keep], X.val[keep])
    C = datagen.init_centers_csr(Y, np.array([10, 20, 10, 30, 20]))  # duplicates
    Yd = skm.DeviceCSR.from_host(Y)
    a, best, second = skm.assign(Yd, torch.from_numpy(C).cuda())
    a = a.cpu().numpy()
    a_ref = check_assign(Y, C, a, best.cpu().numpy(), "ties")
    assert np.array_equal(a, a_ref)  # exact ties resolve to the lowest index
    assert not np.any(np.isin(a, [2, 4]))
    assert a[0] == 0 and a[5] == 0 and a[599] == 0


# ----------------------------------------------------------------- fit

VARIANTS = ["lloyd", "hamerly", "elkan", "simp_hamerly", "simp_elkan", "yinyang"]


def run_fit(skm, torch, Xd, C0, k, variant, max_iter, **kw):
    a, C, C64, st = skm.fit(Xd, k, torch.from_numpy(C0).cuda(), variant, max_iter,
                            want_centers64=True, **kw)
    torch.cuda.synchronize()
    return a.cpu().numpy(), C.cpu().numpy(), C64.cpu().numpy(), st


def test_fit_c1_all_variants_match_oracle(skm, torch_cuda):
    torch = torch_cuda
    X, init, cfg = datagen.sparse_workload("c1")
    C0 = datagen.init_centers_csr(X, init)
    Xd = skm.DeviceCSR.from_host(X)
    ref = oracle.fit(X, C0, "lloyd", cfg.max_iter, trace=True)
    base = None
    for v in VARIANTS:
        for bf in ([0, 1] if "hamerly" in v else [0]):
            say("case fit c1 %s bound_form=%d" % (v, bf))
            a, C, C64, st = run_fit(skm, torch, Xd, C0, cfg.k, v, cfg.max_iter, bound_form=bf)
            assert st.iterations == ref.iterations and st.converged == ref.converged
            assert np.array_equal(st.changed_per_iter, ref.changed)
            assert np.array_equal(a, ref.a)
            assert np.abs(C64 - ref.C).max() < 1e-6
            assert np.linalg.norm(C.astype(np.float64) - ref.C, axis=1).max() < 1e-6
            obj_ref = float(ref.obj_update[~np.isnan(ref.obj_update)][-1])
            assert abs(st.objective - obj_ref) <= 1e-6 * obj_ref
            say("  iters=%d sims=%d (lloyd %d) rechecks=%d max|dC|=%.2e" %
                (st.iterations, st.sims_point_center, ref.sims.sum(), st.rechecks,
                 np.abs(C64 - ref.C).max()))
            if base is None:
                base = (a, C64)
            else:
                assert np.array_equal(a, base[0]) and np.array_equal(C64, base[1])
            if v != "lloyd":
                assert st.sims_point_center < ref.sims.sum()


def test_fit_c1_every_step(skm, torch_cuda):
    """Every step t: the GPU fit stopped after t steps against the oracle's
    own trajectory stopped after t steps (assignment, FP64 centres,
    objective), for Lloyd, Hamerly and Elkan."""
    torch = torch_cuda
    X, init, cfg = datagen.sparse_workload("c1")
    C0 = datagen.init_centers_csr(X, init)
    Xd = skm.DeviceCSR.from_host(X)
    for t in range(1, 8):
        ref = oracle.fit(X, C0, "lloyd", t)
        obj_ref = float(ref.obj_update[~np.isnan(ref.obj_update)][-1])
        for v in ["lloyd", "hamerly", "elkan"]:
            say("case c1 step %d %s" % (t, v))
            a, C, C64, st = run_fit(skm, torch, Xd, C0, cfg.k, v, t)
            assert st.iterations == ref.iterations and st.converged == ref.converged
            assert np.array_equal(a, ref.a)
            assert np.linalg.norm(C64 - ref.C, axis=1).max() < 1e-6
            assert abs(st.objective - obj_ref) <= 1e-6 * obj_ref
        if ref.converged:
            break


@pytest.mark.parametrize("bound_form", [0, 1])
def test_fit_reduced_c2(skm, torch_cuda, bound_form):
    torch = torch_cuda
    X, init, cfg = datagen.sparse_workload("c2", n=20000)
    C0 = datagen.init_centers_csr(X, init)
    Xd = skm.DeviceCSR.from_host(X)
    T = 25
    ref = oracle.fit(X, C0, "lloyd", T)
    base = None
    for v in VARIANTS:
        say("case fit reduced c2 %s bf=%d" % (v, bound_form))
        a, C, C64, st = run_fit(skm, torch, Xd, C0, cfg.k, v, T, bound_form=bound_form)
        say("  iters=%d sims=%d/%d rechecks=%d" % (st.iterations, st.sims_point_center,
                                                    ref.sims.sum(), st.rechecks))
        assert st.iterations == ref.iterations
        assert np.array_equal(st.changed_per_iter, ref.changed)
        assert np.array_equal(a, ref.a)
        assert np.linalg.norm(C64 - ref.C, axis=1).max() < 1e-6
        if base is None:
            base = (a, C64)
        else:
            assert np.array_equal(a, base[0]) and np.array_equal(C64, base[1])


def test_fit_large_clusters(skm, torch_cuda):
    """k = 8 on 20,000 rows: clusters of thousands of rows, whose member sums
    are rebuilt from several parts in the steps where many rows move; the
    whole trajectory matches the oracle's."""
    torch = torch_cuda
    X, init, cfg = datagen.sparse_workload("c2", n=20000)
    k = 8
    C0 = datagen.init_centers_csr(X, init[:k])
    Xd = skm.DeviceCSR.from_host(X)
    T = 30
    ref = oracle.fit(X, C0, "lloyd", T)
    for v in ["lloyd", "hamerly", "yinyang"]:
        say("case fit large clusters %s" % v)
        a, C, C64, st = run_fit(skm, torch, Xd, C0, k, v, T)
        say("  iters=%d sizes=%s" % (st.iterations, np.bincount(a, minlength=k).tolist()))
        assert st.iterations == ref.iterations
        assert np.array_equal(st.changed_per_iter, ref.changed)
        assert np.array_equal(a, ref.a)
        assert np.linalg.norm(C64 - ref.C, axis=1).max() < 1e-6
        assert abs(st.objective - ref.obj_update[~np.isnan(ref.obj_update)][-1]) <= \
            1e-6 * st.objective


def test_fit_partial_walks(skm, torch_cuda):
    """k = 300 with the FP32 copy (padded to 512 centres): Yin-Yang and Elkan
    walk only the groups / chunks their filters leave.  Started from the
    oracle's centres after 14 steps (where the centres move little and the
    filters prune), 8 more steps against the oracle's Lloyd trajectory."""
    torch = torch_cuda
    X, _, _ = datagen.sparse_workload("c2", n=50000)
    k, T = 300, 8
    C0 = datagen.init_centers_csr(X, np.random.default_rng(5).choice(X.n, k, replace=False))
    say("case partial walks: oracle warm-up")
    C14 = oracle.fit(X, C0, "lloyd", 14).C.astype(np.float32)
    say("case partial walks: oracle")
    ref = oracle.fit(X, C14, "lloyd", T)
    Xd = skm.DeviceCSR.from_host(X)
    for v, sched in [("lloyd", 0), ("yinyang", 0), ("yinyang", 1), ("elkan", 1),
                     ("simp_elkan", 1)]:
        say("case partial walks %s schedule=%d" % (v, sched))
        a, C, C64, st = run_fit(skm, torch, Xd, C14, k, v, T, schedule=sched)
        say("  iters=%d sims=%d of %d" % (st.iterations, st.sims_point_center, X.n * k * T))
        if sched == 1:
            # tests at every step: some walked rows skip groups / chunks and
            # count fewer than k similarities, so the total is no multiple of k
            assert st.sims_point_center < X.n * k * T and st.sims_point_center % k != 0
        assert st.iterations == ref.iterations and st.converged == ref.converged
        assert np.array_equal(st.changed_per_iter, ref.changed)
        assert np.array_equal(a, ref.a)
        assert np.linalg.norm(C64 - ref.C, axis=1).max() < 1e-6


@pytest.mark.parametrize("k", [800, 2049])
def test_fit_chunked_group_walks(skm, torch_cuda, k):
    """k = 800 with the FP32 copy (padded to 1024): the row walk takes the
    centres in four launches of 256 (the last one 32), carrying every row's
    running winner between launches; Yin-Yang walks only the groups its
    filters leave in each launch and Elkan only the 4-centre units holding a
    centre whose pair tests failed, so a launch may walk nothing of a row.
    k = 2049 (padded to 4096): nine launches, the last with one centre, and
    sixteen Elkan survival words per row.  Rows from a von Mises-Fisher
    mixture (60 components, d = 48, stored as CSR) keep the centres moving
    for several steps; every variant's whole trajectory must equal the
    oracle's Lloyd trajectory, with the tests at every step and with the
    default schedule."""
    torch = torch_cuda
    X = dense_csr(datagen.dense_vmf(12000, 48, 60, 4242))
    T = 60
    C0 = datagen.init_centers_csr(X, datagen.init_rows(X.n, k, 11))
    say("case chunked group walks: oracle")
    ref = oracle.fit(X, C0, "lloyd", T)
    Xd = skm.DeviceCSR.from_host(X)
    # (variant, schedule, precision): precision 2 walks the FP16 copy, whose
    # Yin-Yang and Elkan steps take 512 centres per launch
    for v, sched, prec in [("yinyang", 1, 0), ("yinyang", 0, 0), ("elkan", 1, 0),
                           ("simp_elkan", 0, 0), ("hamerly", 1, 0), ("lloyd", 0, 0),
                           ("yinyang", 1, 2), ("yinyang", 0, 2), ("elkan", 1, 2),
                           ("simp_elkan", 0, 2)]:
        say("case chunked group walks %s schedule=%d precision=%d" % (v, sched, prec))
        # chunk_walk = 1: Lloyd and Hamerly slice too (their choice is the
        # tuning table's otherwise; Elkan and Yin-Yang always slice)
        a, C, C64, st = run_fit(skm, torch, Xd, C0, k, v, T, schedule=sched, precision=prec,
                                chunk_walk=1)
        say("  iters=%d sims=%d of %d" % (st.iterations, st.sims_point_center,
                                          X.n * k * st.iterations))
        if v in ("yinyang", "elkan") and sched == 1:
            # walked rows skip groups / units: the count is no multiple of k
            assert st.sims_point_center < X.n * k * st.iterations
            assert st.sims_point_center % k != 0
        assert st.iterations == ref.iterations and st.converged == ref.converged
        assert np.array_equal(st.changed_per_iter, ref.changed)
        assert np.array_equal(a, ref.a)
        assert np.linalg.norm(C64 - ref.C, axis=1).max() < 1e-6


def test_fit_chunked_duplicate_centres(skm, torch_cuda):
    """Identical centres in different launches of a chunked walk (k = 600:
    FP32 slices of 256, FP16 slices of 512): every row with such a pair at
    its maximum is an exact FP64 tie across launches, which must go to the
    previous assignment if it attains the maximum, else to the lowest index,
    as in the oracle's Lloyd trajectory (the duplicate that loses keeps its
    centre, R3).  Every variant, both centre copies, tests at every step."""
    torch = torch_cuda
    X = dense_csr(datagen.dense_vmf(6000, 48, 40, 515))
    k, T = 600, 40
    rows = datagen.init_rows(X.n, k, 23)
    for src, dst in [(3, 260), (3, 520), (100, 356), (300, 599), (511, 512)]:
        rows[dst] = rows[src]
    C0 = datagen.init_centers_csr(X, rows)
    say("case chunked duplicate centres: oracle")
    ref = oracle.fit(X, C0, "lloyd", T)
    Xd = skm.DeviceCSR.from_host(X)
    for v in VARIANTS:
        for prec in (0, 2):
            say("case chunked duplicate centres %s precision=%d" % (v, prec))
            a, C, C64, st = run_fit(skm, torch, Xd, C0, k, v, T, schedule=1, precision=prec,
                                    chunk_walk=1)
            assert st.iterations == ref.iterations and st.converged == ref.converged
            assert np.array_equal(st.changed_per_iter, ref.changed)
            assert np.array_equal(a, ref.a)
            assert np.linalg.norm(C64 - ref.C, axis=1).max() < 1e-6


def test_fit_c2_full_size(skm, torch_cuda):
    """Full c2 workload (n=1e5, d=5e4, k=100) run to no-change: every
    variant identical to the oracle's full FP64 Lloyd trajectory."""
    torch = torch_cuda
    X, init, cfg = datagen.sparse_workload("c2")
    C0 = datagen.init_centers_csr(X, init)
    Xd = skm.DeviceCSR.from_host(X)
    say("case fit c2: oracle")
    ref = oracle.fit(X, C0, "lloyd", cfg.max_iter)
    say("  oracle: %d steps, converged %d" % (ref.iterations, ref.converged))
    for v in ["lloyd", "hamerly", "elkan", "simp_hamerly", "yinyang"]:
        say("case fit c2 %s" % v)
        a, C, C64, st = run_fit(skm, torch, Xd, C0, cfg.k, v, cfg.max_iter)
        say("  iters=%d converged=%d sims=%d rechecks=%d" % (st.iterations, st.converged,
                                                            st.sims_point_center, st.rechecks))
        assert st.iterations == ref.iterations and st.converged == ref.converged, v
        assert np.array_equal(st.changed_per_iter, ref.changed), v
        assert np.array_equal(a, ref.a), v
        assert np.linalg.norm(C64 - ref.C, axis=1).max() < 1e-6, v


# ----------------------------------------------------------------- dense (MFMA)

def dense_csr(D):
    n, d = D.shape
    rp = np.arange(0, n * d + 1, d, dtype=np.int64)
    return datagen.CSR(n, d, rp, np.tile(np.arange(d, dtype=np.int32), n),
                       np.ascontiguousarray(D, np.float32).ravel())


@pytest.mark.parametrize("d,k", [(64, 10), (200, 100), (256, 700), (37, 5)])
def test_dense_assign_matches_oracle(skm, torch_cuda, d, k):
    torch = torch_cuda
    say("case dense assign d=%d k=%d" % (d, k))
    X = datagen.dense_vmf(3000, d, 16, 500 + d)
    rng = np.random.default_rng(d + k)
    C = X[rng.choice(X.shape[0], k, replace=False)].astype(np.float64)
    C += 0.01 * rng.normal(size=C.shape)
    C = (C / np.linalg.norm(C, axis=1, keepdims=True)).astype(np.float32)
    Xd = skm.DeviceDense.from_host(X)
    a, best, second = skm.assign(Xd, torch.from_numpy(C).cuda())
    torch.cuda.synchronize()
    check_assign(dense_csr(X), C, a.cpu().numpy(), best.cpu().numpy(), "dense assign",
                 terms=max(32, 1 << (d - 1).bit_length()))


@pytest.mark.parametrize("precision", [0, 1])
def test_dense_fit_small_matches_oracle(skm, torch_cuda, precision):
    torch = torch_cuda
    X = datagen.dense_vmf(20000, 256, 64, 4242)
    init = datagen.init_rows(X.shape[0], 64, 4242)
    C0 = X[init].copy()
    Xd = skm.DeviceDense.from_host(X)
    Xc = dense_csr(X)
    ref = oracle.fit(Xc, C0, "lloyd", 40)
    base = None
    # schedule 1 runs the bound tests at every step; the default switches
    # them off while they prune little
    for v, sched in [("lloyd", 0), ("hamerly", 0), ("simp_hamerly", 0), ("hamerly", 1),
                     ("simp_hamerly", 1)]:
        say("case dense fit precision=%d %s schedule=%d" % (precision, v, sched))
        a, C, C64, st = run_fit(skm, torch, Xd, C0, 64, v, 40, precision=precision,
                                schedule=sched)
        say("  iters=%d sims=%d rechecks=%d (oracle iters %d)" % (
            st.iterations, st.sims_point_center, st.rechecks, ref.iterations))
        assert st.iterations == ref.iterations
        assert np.array_equal(a, ref.a)
        assert np.linalg.norm(C64 - ref.C, axis=1).max() < 1e-6
        if base is None:
            base = (a, C64)
        else:
            assert np.array_equal(a, base[0]) and np.array_equal(C64, base[1])


@pytest.mark.parametrize("d,k", [(37, 5), (100, 45), (200, 100), (64, 33), (20, 7), (64, 1)])
def test_dense_bf16_ragged_matches_oracle(skm, torch_cuda, d, k):
    """BF16 top-2 pass where the last centre tiles reach past k (k not a
    multiple of 32, down to a tile of padding only, and k = 1) at the padded
    widths dp = 32, 64, 128 and 256: whole trajectories equal the oracle's."""
    torch = torch_cuda
    X = datagen.dense_vmf(4000, d, max(4, k // 2), 900 + d)
    C0 = X[datagen.init_rows(X.shape[0], k, 77 + k)].copy()
    Xd = skm.DeviceDense.from_host(X)
    ref = oracle.fit(dense_csr(X), C0, "lloyd", 25)
    for v, sched in [("lloyd", 0), ("hamerly", 0), ("hamerly", 1)]:
        say("case dense bf16 ragged d=%d k=%d %s schedule=%d" % (d, k, v, sched))
        a, C, C64, st = run_fit(skm, torch, Xd, C0, k, v, 25, precision=1, schedule=sched)
        say("  iters=%d rechecks=%d (oracle iters %d)" % (st.iterations, st.rechecks,
                                                         ref.iterations))
        assert st.iterations == ref.iterations
        assert np.array_equal(a, ref.a)
        assert np.linalg.norm(C64 - ref.C, axis=1).max() < 1e-6


def adversarial_bf16_rows(n=4096, d=256, seed=5):
    """Rounding that defeats a plain BF16 argmax.  Centre c1's entries have
    the significand 1 + 2^-8 + 2^-10 (round to nearest even in BF16 takes
    them up to 1 + 2^-7), c2's have 1 + 2^-7 + 2^-8 - 2^-10 (taken down to
    the same value); each row copies 31 entries of each, so the BF16
    products overstate <x, c1> and understate <x, c2> by about 2.9e-3 each,
    and a filler coordinate shared with c1 sweeps the true gap through zero.
    Six distractor centres live on other coordinates."""
    rng = np.random.default_rng(seed)
    U = 1 + 2.0 ** -8 + 2.0 ** -10
    W = 1 + 2.0 ** -7 + 2.0 ** -8 - 2.0 ** -10
    sg = rng.choice([-1.0, 1.0], size=d)
    c1 = np.zeros(d)
    c2 = np.zeros(d)
    c1[0:63] = U / 8 * sg[0:63]
    c1[63] = np.sqrt(1 - (c1[0:63] ** 2).sum())
    c2[64:126] = W / 8 * sg[64:126]
    c2[126] = np.sqrt(1 - (c2[64:126] ** 2).sum())
    X = np.zeros((n, d))
    X[:, 0:31] = c1[0:31]
    X[:, 64:95] = c2[64:95]
    base = (X[0] ** 2).sum()
    fx = np.linspace(0.0, np.sqrt(1 - base) * 0.999, n)
    X[:, 63] = fx
    X[:, 200] = np.sqrt(1 - base - fx ** 2)
    C = [c1, c2]
    for _ in range(6):
        v = np.zeros(d)
        v[128:192] = rng.normal(size=64)
        C.append(v / np.linalg.norm(v))
    return X.astype(np.float32), np.array(C, dtype=np.float32)


def test_dense_bf16_adversarial_rounding(skm, torch_cuda):
    """Coherent BF16 rounding errors of opposite sign on the two leading
    centres: a plain BF16 argmax gets thousands of rows wrong, so every one of
    them has to fall inside the error band (built from the measured rounding
    norms of the row and centre copies) and be re-decided in FP64."""
    torch = torch_cuda
    X, C0 = adversarial_bf16_rows()
    Xc = dense_csr(X)
    S = oracle.sims(Xc, C0.astype(np.float64), np.arange(X.shape[0]))
    bf = lambda A: torch.from_numpy(np.ascontiguousarray(A)).to(torch.bfloat16).double().numpy()
    wrong = int((np.argmax(bf(X) @ bf(C0).T, 1) != np.argmax(S, 1)).sum())
    say("case dense bf16 adversarial: plain BF16 argmax wrong on %d of %d rows" %
        (wrong, X.shape[0]))
    assert wrong >= 1000
    Xd = skm.DeviceDense.from_host(X)
    ref1 = oracle.fit(Xc, C0, "lloyd", 1)
    gap = gap_of(S)
    a, C, C64, st = run_fit(skm, torch, Xd, C0, C0.shape[0], "lloyd", 1, precision=1)
    say("  step 1: rechecks=%d mismatches=%d" % (st.rechecks, int((a != ref1.a).sum())))
    assert st.rechecks >= wrong
    assert np.array_equal(a[gap > GAP], ref1.a[gap > GAP])
    assert np.all(S.max(1) - S[np.arange(len(a)), a] <= 1e-12)
    ref = oracle.fit(Xc, C0, "lloyd", 10)
    for v in ("lloyd", "hamerly", "simp_hamerly"):
        say("case dense bf16 adversarial %s 10 steps" % v)
        a, C, C64, st = run_fit(skm, torch, Xd, C0, C0.shape[0], v, 10, precision=1)
        assert st.iterations == ref.iterations
        assert np.array_equal(a, ref.a)
        assert np.linalg.norm(C64 - ref.C, axis=1).max() < 1e-6


def test_sparse_k_sweep_matches_oracle(skm, torch_cuda):
    """k on both sides of every centre-copy width the row walk specialises
    for (one 64-centre lane set, 128-byte lines of 32 FP32 or 64 FP16
    centres, the 2048 / 4096 ends), every variant, FP32 and FP16 copies:
    whole trajectories equal the oracle's on a small tf-idf matrix."""
    torch = torch_cuda
    X = datagen.sparse_tfidf(4200, 3000, 30.0, 9090)
    Xd = skm.DeviceCSR.from_host(X)
    for k in (1, 2, 63, 64, 65, 127, 128, 129, 255, 256, 257, 513, 1025, 2047, 2049, 4096):
        C0 = datagen.init_centers_csr(X, datagen.init_rows(X.n, k, 31 + k))
        ref = oracle.fit(X, C0, "lloyd", 8)
        for v in VARIANTS:
            for prec in (0, 2):
                # FP32 copy above 256 centres: 256-centre slices and whole
                # rows (the tuning table picks one of them); Elkan and
                # Yin-Yang at 128 < k <= 256: one packed slice on request
                sliceable = prec == 0 and k > 256
                packed = prec == 0 and 128 < k <= 256 and ("elkan" in v or v == "yinyang")
                cws = (1, 2) if sliceable else (0, 1) if packed else (0,)
                for cw in cws:
                    say("case sparse k sweep k=%d %s precision=%d chunk_walk=%d" % (k, v, prec, cw))
                    a, C, C64, st = run_fit(skm, torch, Xd, C0, k, v, 8, precision=prec,
                                            schedule=1, chunk_walk=cw)
                    assert st.iterations == ref.iterations
                    assert np.array_equal(a, ref.a)
                    assert np.linalg.norm(C64 - ref.C, axis=1).max() < 1e-6


@pytest.mark.parametrize("layout", [1, 2])
def test_walk_layouts_match_oracle(skm, torch_cuda, layout):
    """Both row-walk layouts of the FP32 copy that the tuning table chooses
    between (walk_layout 1: the default, 2: one row per wave at k <= 64, four
    rows per wave above), at k on both sides of every tuned width (16 < k <=
    512, whole-row walks), short and long rows, Lloyd, Hamerly, simplified
    Hamerly and Yin-Yang, tests adaptive and at every step: whole
    trajectories equal the oracle's."""
    torch = torch_cuda
    for mean, seed in ((12.0, 7070), (30.0, 7072), (60.0, 7071)):
        X = datagen.sparse_tfidf(3100, 2500, mean, seed)
        Xd = skm.DeviceCSR.from_host(X)
        for k in (17, 32, 33, 64, 65, 128, 129, 256, 257, 512):
            C0 = datagen.init_centers_csr(X, datagen.init_rows(X.n, k, 77 + k))
            ref = oracle.fit(X, C0, "lloyd", 10)
            # Yin-Yang: its plain steps take the fit walk, so the layout too
            for v in ("lloyd", "hamerly", "simp_hamerly", "yinyang"):
                for sched in (0, 1):
                    say("case walk layout %d mean row %g k=%d %s schedule=%d" %
                        (layout, mean, k, v, sched))
                    a, C, C64, st = run_fit(skm, torch, Xd, C0, k, v, 10, schedule=sched,
                                            walk_layout=layout, chunk_walk=2)
                    assert st.iterations == ref.iterations
                    assert np.array_equal(a, ref.a)
                    assert np.linalg.norm(C64 - ref.C, axis=1).max() < 1e-6


def test_short_rows_exact_ties_match_oracle(skm, torch_cuda):
    """Rows of about three stored entries (the density of the paper's DBLP
    author-conference matrix): many rows have exactly equal FP64
    similarities to several centres (their terms are absent from those
    centres), so the tie rule decides them.  At k = 100, 200 and 500 the
    tuning tables pick the grouped layout and whole-row walks; every variant
    (and the sliced walk, forced) must follow the oracle's Lloyd trajectory."""
    torch = torch_cuda
    X = datagen.sparse_tfidf(30000, 3000, 3.0, 8181)
    Xd = skm.DeviceCSR.from_host(X)
    for k in (100, 200, 500):
        C0 = datagen.init_centers_csr(X, datagen.init_rows(X.n, k, 17 + k))
        ref = oracle.fit(X, C0, "lloyd", 12)
        for v in VARIANTS:
            for cw in ((0, 1) if k > 256 else (0,)):
                say("case short rows k=%d %s chunk_walk=%d" % (k, v, cw))
                a, C, C64, st = run_fit(skm, torch, Xd, C0, k, v, 12, schedule=1, chunk_walk=cw)
                assert st.iterations == ref.iterations
                assert np.array_equal(a, ref.a)
                assert np.linalg.norm(C64 - ref.C, axis=1).max() < 1e-6
        say("  k=%d: %d of %d rows re-decided in FP64 in the last fit" % (k, st.rechecks, X.n))


def test_topical_rows_match_oracle(skm, torch_cuda):
    """Rows with topic structure (20 topics), where the centres settle and
    the bounds prune far more than on plain rows: every variant, tests at
    every step and adaptive, FP32 and FP16 copies, follows the oracle's
    Lloyd trajectory."""
    torch = torch_cuda
    X = datagen.sparse_tfidf(20000, 8000, 40.0, 5151, topics=20)
    Xd = skm.DeviceCSR.from_host(X)
    for k in (20, 100, 300):
        C0 = datagen.init_centers_csr(X, datagen.init_rows(X.n, k, 23 + k))
        ref = oracle.fit(X, C0, "lloyd", 20)
        for v in VARIANTS:
            # chunk_walk 1 at k = 100 and 300: 256-centre slices (at k = 100
            # one packed slice for Elkan and Yin-Yang, whole rows otherwise)
            for sched, prec, cw in ((1, 0, 0), (0, 0, 0), (1, 2, 0), (0, 0, 1)):
                if prec == 2 and k < 65 or cw == 1 and k < 65:
                    continue
                say("case topical rows k=%d %s schedule=%d precision=%d chunk_walk=%d" %
                    (k, v, sched, prec, cw))
                a, C, C64, st = run_fit(skm, torch, Xd, C0, k, v, 20, schedule=sched,
                                        precision=prec, chunk_walk=cw)
                assert st.iterations == ref.iterations
                assert np.array_equal(a, ref.a)
                assert np.linalg.norm(C64 - ref.C, axis=1).max() < 1e-6
                say("  sims %.3f of Lloyd's" % (st.sims_point_center / (X.n * k * st.iterations)))


@pytest.mark.parametrize("variant", ["yinyang", "elkan", "simp_elkan"])
def test_timed_walk_choice_matches_oracle(skm, torch_cuda, variant):
    """Yin-Yang (k_p >= 256) and Elkan (k_p >= 512) with whole-row walks time
    their steps with tests both ways in the first chunk of steps (whole rows
    at steps 2 and 5, packed 256-centre slices at 3 and 4) and keep the
    faster: steps of the two walks alternate in both directions, and every
    fit follows the oracle's Lloyd trajectory whichever walk it keeps, on
    topic-structured and plain rows, tests adaptive and at every step,
    against whole rows and packed slices throughout."""
    torch = torch_cuda
    for topics, seed in ((20, 5353), (0, 5354)):
        X = datagen.sparse_tfidf(20000, 8000, 40.0, seed, topics=topics)
        Xd = skm.DeviceCSR.from_host(X)
        for k in (129, 200, 256, 300, 600):
            C0 = datagen.init_centers_csr(X, datagen.init_rows(X.n, k, 41 + k))
            ref = oracle.fit(X, C0, "lloyd", 30)
            sims = {}
            for sched in (0, 1):
                for cw in (0, 1, 2):
                    say("case timed walk %s topics=%d k=%d schedule=%d chunk_walk=%d" %
                        (variant, topics, k, sched, cw))
                    a, C, C64, st = run_fit(skm, torch, Xd, C0, k, variant, 30, schedule=sched,
                                            chunk_walk=cw)
                    assert st.iterations == ref.iterations
                    assert np.array_equal(a, ref.a)
                    assert np.linalg.norm(C64 - ref.C, axis=1).max() < 1e-6
                    sims[sched, cw] = st.sims_point_center
            say("  similarities: timed choice %d, packed %d, whole rows %d" %
                (sims[1, 0], sims[1, 1], sims[1, 2]))


def test_timed_slices_large_copy_matches_oracle(skm, torch_cuda):
    """Lloyd and the Hamerly variants with an FP32 copy of 64 MB or more
    (40,000 columns, k_p = 512) where the table picks whole rows time
    256-centre slices against whole rows in their first steps (slices at
    steps 3 and 4) and keep the faster: every fit follows the oracle's Lloyd
    trajectory, on topic-structured and plain rows, tests adaptive and at
    every step."""
    torch = torch_cuda
    for topics, seed in ((20, 5355), (0, 5356)):
        X = datagen.sparse_tfidf(8000, 40000, 30.0, seed, topics=topics)
        Xd = skm.DeviceCSR.from_host(X)
        for k in (257, 400):
            C0 = datagen.init_centers_csr(X, datagen.init_rows(X.n, k, 43 + k))
            ref = oracle.fit(X, C0, "lloyd", 20)
            for v in ("lloyd", "hamerly", "simp_hamerly"):
                for sched in (0, 1):
                    say("case timed slices %s topics=%d k=%d schedule=%d" % (v, topics, k, sched))
                    a, C, C64, st = run_fit(skm, torch, Xd, C0, k, v, 20, schedule=sched)
                    assert st.iterations == ref.iterations
                    assert np.array_equal(a, ref.a)
                    assert np.linalg.norm(C64 - ref.C, axis=1).max() < 1e-6


def test_dense_shape_sweep_matches_oracle(skm, torch_cuda):
    """Seeded sweep of small dense shapes (row counts that leave partial
    waves and blocks, widths on both sides of every padded width, k on both
    sides of the 32-centre tiles and 64-centre chunks), FP32 and BF16, Lloyd
    and Hamerly: whole trajectories equal the oracle's."""
    torch = torch_cuda
    rng = np.random.default_rng(20260)
    shapes = [(1, 3, 1), (70, 17, 2), (300, 31, 31), (513, 33, 32), (600, 64, 33),
              (777, 65, 63), (1000, 100, 64), (1029, 129, 65), (640, 200, 100),
              (900, 256, 129)]
    for n, d, k in shapes:
        X = datagen.dense_vmf(n, d, max(2, k // 2), int(rng.integers(1 << 30)))
        C0 = X[datagen.init_rows(n, k, int(rng.integers(1 << 30)))].copy()
        ref = oracle.fit(dense_csr(X), C0, "lloyd", 15)
        Xd = skm.DeviceDense.from_host(X)
        for prec in (0, 1):
            for v in ("lloyd", "hamerly"):
                say("case dense sweep n=%d d=%d k=%d precision=%d %s" % (n, d, k, prec, v))
                a, C, C64, st = run_fit(skm, torch, Xd, C0, k, v, 15, precision=prec,
                                        schedule=1)
                assert st.iterations == ref.iterations
                assert np.array_equal(a, ref.a)
                assert np.linalg.norm(C64 - ref.C, axis=1).max() < 1e-6


# ------------------------------------------------- FP16 centre copy (CSR)

@pytest.mark.parametrize("k", [100, 200, 300, 700, 1500])
def test_fp16_centre_copy_matches_fp32(skm, torch_cuda, k):
    """precision = 2 walks the rows against an FP16 copy of the centres with
    a wider (value-relative on non-negative data) error band; the fit must
    be identical to the FP32 one, and equal to the oracle's."""
    torch = torch_cuda
    X = datagen.sparse_tfidf(6000, 8000, 40.0, 77 + k)
    C0 = datagen.init_centers_csr(X, datagen.init_rows(X.n, k, 5 + k))
    Xd = skm.DeviceCSR.from_host(X)
    ref = None
    for v in ["lloyd", "hamerly", "simp_hamerly", "yinyang"]:
        say("case fp16 centre copy k=%d %s" % (k, v))
        a32, C32, _, st32 = run_fit(skm, torch, Xd, C0, k, v, 30)
        a16, C16, _, st16 = run_fit(skm, torch, Xd, C0, k, v, 30, precision=2)
        assert np.array_equal(a32, a16) and np.array_equal(C32, C16)
        assert st32.iterations == st16.iterations
        say("  iterations %d rechecks fp32 %d fp16 %d" % (st16.iterations, st32.rechecks,
                                                          st16.rechecks))
        if ref is None:
            ref = oracle.fit(X, C0, "lloyd", 30)
        assert st16.iterations == ref.iterations and np.array_equal(a16, ref.a)


def test_fp16_centre_copy_mixed_signs(skm, torch_cuda):
    """Rows with negative entries take the absolute error bound."""
    torch = torch_cuda
    rng = np.random.default_rng(31)
    D = rng.normal(size=(3000, 48))
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    X = dense_csr(D.astype(np.float32))
    k = 150
    C0 = datagen.init_centers_csr(X, datagen.init_rows(X.n, k, 9))
    Xd = skm.DeviceCSR.from_host(X)
    ref = oracle.fit(X, C0, "lloyd", 25)
    for v in ["lloyd", "hamerly", "yinyang"]:
        say("case fp16 mixed signs %s" % v)
        a16, C16, _, st16 = run_fit(skm, torch, Xd, C0, k, v, 25, precision=2)
        assert st16.iterations == ref.iterations and np.array_equal(a16, ref.a)
