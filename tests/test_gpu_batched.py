"""GPU checks of skm_fit_batched (through the C ABI): every problem of a
batch gets exactly what skm_fit gives it alone (assignments, FP32 centres,
iteration counts: bit for bit), and small problems match the FP64 oracle's
Lloyd trajectory."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


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


@pytest.fixture(scope="module")
def problems():
    # the batched workload's generator at 4% of its row counts: 12 problems
    # of 40..2000 rows, k from 8 to 256 (capped at the row count)
    return datagen.batched_instances(n_inst=12, scale=0.04)


def say(*a):
    print(*a, flush=True)


def device_problems(skm, torch, insts, max_iter=None):
    out = []
    for p in insts:
        Xd = skm.DeviceCSR.from_host(p.X)
        C0 = torch.from_numpy(datagen.init_centers_csr(p.X, p.init)).cuda()
        out.append((Xd, p.k, C0, max_iter or p.max_iter))
    return out


@pytest.mark.parametrize("variant,workers", [("lloyd", 3), ("hamerly", 4), ("elkan", 2),
                                             ("simp_hamerly", 1), ("yinyang", 3)])
def test_batched_equals_individual_fits(skm, torch_cuda, problems, variant, workers):
    torch = torch_cuda
    say("case batched %s workers=%d" % (variant, workers))
    dp = device_problems(skm, torch, problems)
    res = skm.fit_batched(dp, variant, workers=workers)
    torch.cuda.synchronize()
    for b, ((Xd, k, C0, it), (a, C, st)) in enumerate(zip(dp, res)):
        a1, C1, _, st1 = skm.fit(Xd, k, C0, variant, it, per_iter=False)
        torch.cuda.synchronize()
        assert torch.equal(a, a1), b
        assert torch.equal(C, C1), b
        assert st.iterations == st1.iterations and st.converged == st1.converged, b
        # Elkan and Yin-Yang time their walk choice at wide k (whole rows or
        # packed slices), so two runs may count different similarities; the
        # results may not differ
        if variant not in ("elkan", "simp_elkan", "yinyang"):
            assert st.sims_point_center == st1.sims_point_center, b
    say("  %d problems, iterations %s" % (len(res), [r[2].iterations for r in res]))


def test_batched_matches_oracle(skm, torch_cuda, problems):
    torch = torch_cuda
    small = sorted(problems, key=lambda p: p.X.nnz * p.k)[:4]
    dp = device_problems(skm, torch, small)
    res = skm.fit_batched(dp, "hamerly", workers=2)
    torch.cuda.synchronize()
    for p, (Xd, k, C0, it), (a, C, st) in zip(small, dp, res):
        say("case batched oracle n=%d k=%d" % (p.X.n, k))
        ref = oracle.fit(p.X, datagen.init_centers_csr(p.X, p.init), "lloyd", it)
        assert st.iterations == ref.iterations and st.converged == ref.converged
        assert np.array_equal(a.cpu().numpy(), ref.a)
        assert np.linalg.norm(C.cpu().numpy().astype(np.float64) - ref.C, axis=1).max() < 1e-6


@pytest.mark.parametrize("variant,precision", [("hamerly", 0), ("yinyang", 0), ("elkan", 0),
                                               ("yinyang", 2)])
def test_batched_chunked_problems(skm, torch_cuda, variant, precision):
    """Problems wide enough for the chunked row walk (k = 300, 600, 1100)
    next to a small one, run by the batched driver on a shared workspace:
    each equals its own fit and the oracle's Lloyd trajectory."""
    torch = torch_cuda
    specs = [(3000, 300, 1), (4000, 600, 2), (2500, 1100, 3), (1500, 40, 4)]
    probs, refs = [], []
    for n, k, seed in specs:
        X = datagen.sparse_tfidf(n, 6000, 40.0, 700 + seed)
        C0 = datagen.init_centers_csr(X, datagen.init_rows(X.n, k, seed))
        Xd = skm.DeviceCSR.from_host(X)
        probs.append((Xd, k, torch.from_numpy(C0).cuda(), 12))
        refs.append((X, C0))
    say("case batched chunked %s precision=%d" % (variant, precision))
    res = skm.fit_batched(probs, variant, workers=3, precision=precision, chunk_walk=1)
    torch.cuda.synchronize()
    for (Xd, k, C0, it), (a, C, st), (X, C0h) in zip(probs, res, refs):
        a1, C1, _, st1 = skm.fit(Xd, k, C0, variant, it, per_iter=False, precision=precision,
                                 chunk_walk=1)
        torch.cuda.synchronize()
        assert torch.equal(a, a1) and torch.equal(C, C1), k
        assert st.iterations == st1.iterations, k
        ref = oracle.fit(X, C0h, "lloyd", it)
        assert st.iterations == ref.iterations and np.array_equal(a.cpu().numpy(), ref.a), k


def test_batched_matches_oracle_uneven(skm, torch_cuda):
    """The host-thread driver on an uneven subset of the batched workload at
    20% of its row counts -- the problems with the most rows and the most
    centres among them -- against the FP64 oracle's Lloyd trajectory."""
    torch = torch_cuda
    insts = datagen.batched_instances(scale=0.2)
    by_n = sorted(range(len(insts)), key=lambda b: insts[b].X.n)
    by_k = sorted(range(len(insts)), key=lambda b: insts[b].k)
    pick = sorted(set([by_n[-1], by_k[-1], by_n[0], by_k[0], by_n[len(by_n) // 2], 7]))
    sub = [insts[b] for b in pick]
    dp = device_problems(skm, torch, sub)
    res = skm.fit_batched(dp, "hamerly", workers=4)
    torch.cuda.synchronize()
    for p, (Xd, k, C0, it), (a, C, st) in zip(sub, dp, res):
        say("case batched oracle uneven n=%d k=%d" % (p.X.n, k))
        ref = oracle.fit(p.X, datagen.init_centers_csr(p.X, p.init), "lloyd", it)
        assert st.iterations == ref.iterations and st.converged == ref.converged
        assert np.array_equal(a.cpu().numpy(), ref.a)
        assert np.linalg.norm(C.cpu().numpy().astype(np.float64) - ref.C, axis=1).max() < 1e-6


def test_batched_twice_with_fewer_problems(skm, torch_cuda, problems):
    """Two calls in a row on one workspace, the second with fewer and
    smaller problems: no state leaks from the first call."""
    torch = torch_cuda
    dp = device_problems(skm, torch, problems, max_iter=6)
    ws = torch.empty(skm.batched_workspace_size(dp, "hamerly", workers=3), dtype=torch.uint8,
                     device="cuda")
    first = skm.fit_batched(dp, "hamerly", workers=3, workspace=ws)
    sub = dp[5:8]
    second = skm.fit_batched(sub, "hamerly", workers=3, workspace=ws)
    torch.cuda.synchronize()
    for (Xd, k, C0, it), (a, C, st) in zip(sub, second):
        a1, C1, _, _ = skm.fit(Xd, k, C0, "hamerly", it, per_iter=False)
        torch.cuda.synchronize()
        assert torch.equal(a, a1) and torch.equal(C, C1)
    for (a, C, st), (a2, C2, _) in zip(first[5:8], second):
        assert torch.equal(a, a2) and torch.equal(C, C2)


# ----------------------------------------------------- lockstep (workers = 0)
# The lockstep path is switched off in the library (its first GPU run did not
# finish and the cause is not yet found); these tests stay, skipped, until it
# is back on.
LOCKSTEP_OFF = pytest.mark.skip(reason="lockstep batched path switched off: its first GPU run "
                                       "did not finish, cause not yet found")

def _compare_with_single(skm, torch, dp, res, variant):
    for b, ((Xd, k, C0, it), (a, C, st)) in enumerate(zip(dp, res)):
        a1, C1, _, st1 = skm.fit(Xd, k, C0, variant, it, per_iter=False)
        torch.cuda.synchronize()
        assert torch.equal(a, a1), b
        assert torch.equal(C, C1), b
        assert st.iterations == st1.iterations and st.converged == st1.converged, b
        assert st.sims_point_center == st1.sims_point_center, b
        assert st.sims_center_center == st1.sims_center_center, b
        assert st.objective == st1.objective, b


@LOCKSTEP_OFF
@pytest.mark.parametrize("variant", ["lloyd", "hamerly", "simp_hamerly"])
@pytest.mark.parametrize("tile", [0, 64])
def test_lockstep_equals_individual_fits(skm, torch_cuda, problems, variant, tile):
    """One lockstep call (persistent batched walk, graph-replayed steps) gives
    every problem exactly its own skm_fit: assignments, centres, iteration
    count, similarity counts and objective, also with uneven step limits
    (problems stopping at their max_iter mid-chunk)."""
    torch = torch_cuda
    say("case lockstep %s tile=%d" % (variant, tile))
    dp = device_problems(skm, torch, problems)
    dp = [(X, k, C0, [30, 3, 9, 1, 17, 30][b % 6]) for b, (X, k, C0, _) in enumerate(dp)]
    res = skm.fit_batched(dp, variant, workers=0, batch_tile_rows=tile)
    torch.cuda.synchronize()
    _compare_with_single(skm, torch, dp, res, variant)
    say("  iterations %s" % [r[2].iterations for r in res])


@LOCKSTEP_OFF
def test_lockstep_matches_oracle_uneven(skm, torch_cuda):
    """Lockstep Hamerly on an uneven subset of the batched workload at 20% of
    its row counts -- the problems with the most rows and the most centres
    among them -- against the FP64 oracle's Lloyd trajectory."""
    torch = torch_cuda
    insts = datagen.batched_instances(scale=0.2)
    by_n = sorted(range(len(insts)), key=lambda b: insts[b].X.n)
    by_k = sorted(range(len(insts)), key=lambda b: insts[b].k)
    pick = sorted(set([by_n[-1], by_k[-1], by_n[0], by_k[0], by_n[len(by_n) // 2], 7]))
    sub = [insts[b] for b in pick]
    dp = device_problems(skm, torch, sub)
    res = skm.fit_batched(dp, "hamerly", workers=0)
    torch.cuda.synchronize()
    for p, (Xd, k, C0, it), (a, C, st) in zip(sub, dp, res):
        say("case lockstep oracle n=%d k=%d" % (p.X.n, k))
        ref = oracle.fit(p.X, datagen.init_centers_csr(p.X, p.init), "lloyd", it)
        assert st.iterations == ref.iterations and st.converged == ref.converged
        assert np.array_equal(a.cpu().numpy(), ref.a)
        assert np.linalg.norm(C.cpu().numpy().astype(np.float64) - ref.C, axis=1).max() < 1e-6


@LOCKSTEP_OFF
def test_lockstep_twice_with_fewer_problems(skm, torch_cuda, problems):
    torch = torch_cuda
    dp = device_problems(skm, torch, problems, max_iter=6)
    ws = torch.empty(skm.batched_workspace_size(dp, "hamerly", workers=0), dtype=torch.uint8,
                     device="cuda")
    first = skm.fit_batched(dp, "hamerly", workers=0, workspace=ws)
    sub = dp[5:8]
    second = skm.fit_batched(sub, "hamerly", workers=0, workspace=ws)
    torch.cuda.synchronize()
    _compare_with_single(skm, torch, sub, second, "hamerly")
    for (a, C, st), (a2, C2, _) in zip(first[5:8], second):
        assert torch.equal(a, a2) and torch.equal(C, C2)


@LOCKSTEP_OFF
def test_lockstep_full_batched_workload(skm, torch_cuda):
    """The whole batched workload (256 problems, 2.7 million rows): lockstep
    Hamerly equals every problem's own fit."""
    torch = torch_cuda
    say("case lockstep full batched workload")
    dp = device_problems(skm, torch, datagen.batched_instances())
    res = skm.fit_batched(dp, "hamerly", workers=0, want_centers=True)
    torch.cuda.synchronize()
    _compare_with_single(skm, torch, dp, res, "hamerly")
    say("  steps %d" % sum(r[2].iterations for r in res))
