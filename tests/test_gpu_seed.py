"""GPU checks of spherical k-means++ seeding and the warm start (through the
C ABI) against the FP64 oracle: the same uniforms give the same chosen rows;
the cached assignment step matches the oracle's; a fit started from the
cache reaches exactly the result of a cold fit from the same centres while
computing fewer similarities."""
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


def say(*a):
    print(*a, flush=True)


CASES = [("c1", None, 10, 1.0), ("c1", None, 10, 1.5), ("c2", 20000, 100, 1.0),
         ("c2", 3000, 3000, 1.0)]


@pytest.mark.parametrize("name,n,k,alpha", CASES)
def test_seeding_matches_oracle(skm, torch_cuda, name, n, k, alpha):
    torch = torch_cuda
    say("case seed %s n=%s k=%d alpha=%g" % (name, n, k, alpha))
    X, _, _ = datagen.sparse_workload(name, n)
    u = np.random.default_rng(k + int(10 * alpha)).random(k)
    ch_ref, a_ref, s1_ref, s2_ref = oracle.kmeanspp(X, k, alpha, u)
    Xd = skm.DeviceCSR.from_host(X)
    ch, C, a, s1, s2 = skm.seed_kmeanspp(Xd, k, u, alpha)
    torch.cuda.synchronize()
    assert np.array_equal(ch.cpu().numpy(), ch_ref)
    assert np.array_equal(C.cpu().numpy(), datagen.init_centers_csr(X, ch_ref))
    assert np.array_equal(a.cpu().numpy(), a_ref)
    assert np.abs(s1.cpu().numpy() - s1_ref).max() < 1e-12
    fin = np.isfinite(s2_ref)
    assert np.array_equal(np.isfinite(s2.cpu().numpy()), fin)
    assert np.abs(s2.cpu().numpy()[fin] - s2_ref[fin]).max(initial=0.0) < 1e-12


# k = 600 takes the chunked row walk (three launches of up to 256 FP32 or
# two of up to 512 FP16 centres per step) with bounds set from the seeding's
# cache
@pytest.mark.parametrize("variant,k,precision", [
    ("lloyd", 100, 0), ("hamerly", 100, 0), ("elkan", 100, 0), ("simp_hamerly", 100, 0),
    ("yinyang", 100, 0), ("hamerly", 600, 0), ("elkan", 600, 0), ("yinyang", 600, 0),
    ("elkan", 600, 2), ("yinyang", 600, 2)])
def test_warm_start_equals_cold_fit(skm, torch_cuda, variant, k, precision):
    torch = torch_cuda
    X, _, cfg = datagen.sparse_workload("c2", 20000)
    u = np.random.default_rng(11).random(k)
    Xd = skm.DeviceCSR.from_host(X)
    ch, C, a, s1, s2 = skm.seed_kmeanspp(Xd, k, u)
    say("case warm start %s k=%d precision=%d" % (variant, k, precision))
    ac, Cc, _, stc = skm.fit(Xd, k, C, variant, 60, precision=precision, chunk_walk=1)
    aw, Cw, _, stw = skm.fit(Xd, k, C, variant, 60, warm=(a, s1, s2), precision=precision,
                             chunk_walk=1)
    torch.cuda.synchronize()
    assert torch.equal(ac, aw) and torch.equal(Cc, Cw)
    assert stc.iterations == stw.iterations and stc.converged == stw.converged
    assert np.array_equal(stc.changed_per_iter, stw.changed_per_iter)
    # step 1 is free (Lloyd: exactly n k fewer similarities); the bounded
    # variants prune from step 2 on with bounds set from the FP64 cache
    if variant == "lloyd":
        assert stw.sims_point_center == stc.sims_point_center - X.n * k
    else:
        assert stw.sims_point_center < stc.sims_point_center
    say("  iterations %d, sims cold %d warm %d" % (stc.iterations, stc.sims_point_center,
                                                  stw.sims_point_center))
    # and the result is the oracle's Lloyd fit from the oracle's own seeding
    # with the same uniforms
    if variant == "hamerly":
        ch_ref, _, _, _ = oracle.kmeanspp(X, k, 1.0, u)
        assert np.array_equal(ch.cpu().numpy(), ch_ref)
        ref = oracle.fit(X, datagen.init_centers_csr(X, ch_ref), "lloyd", 60)
        assert ref.iterations == stw.iterations
        assert np.array_equal(aw.cpu().numpy(), ref.a)


@pytest.mark.parametrize("variant,k", [("yinyang", 200), ("yinyang", 300), ("elkan", 300),
                                       ("hamerly", 300)])
def test_warm_start_timed_walk_equals_cold_fit(skm, torch_cuda, variant, k):
    """Topic-structured rows, walk choice left to the fit (Elkan and Yin-Yang
    time whole rows against packed slices; Hamerly, with a copy of 64 MB or
    more, against slices): a warm start times its steps from step 1 on and
    ends where the cold fit does, and both follow the oracle's Lloyd
    trajectory from the seeded centres."""
    torch = torch_cuda
    d = 40000 if variant == "hamerly" else 8000
    X = datagen.sparse_tfidf(12000, d, 40.0, 6161, topics=20)
    u = np.random.default_rng(13).random(k)
    Xd = skm.DeviceCSR.from_host(X)
    ch, C, a, s1, s2 = skm.seed_kmeanspp(Xd, k, u)
    say("case warm start timed walk %s k=%d" % (variant, k))
    ac, Cc, _, stc = skm.fit(Xd, k, C, variant, 25)
    aw, Cw, _, stw = skm.fit(Xd, k, C, variant, 25, warm=(a, s1, s2))
    torch.cuda.synchronize()
    assert torch.equal(ac, aw) and torch.equal(Cc, Cw)
    assert stc.iterations == stw.iterations and stc.converged == stw.converged
    ref = oracle.fit(X, C.cpu().numpy(), "lloyd", 25)
    assert stc.iterations == ref.iterations
    assert np.array_equal(ac.cpu().numpy(), ref.a)
    say("  iterations %d, sims cold %d warm %d" % (stc.iterations, stc.sims_point_center,
                                                  stw.sims_point_center))


@pytest.mark.parametrize("name,n,k,chain,alpha", [("c1", None, 10, 20, 1.0),
                                                  ("c1", None, 10, 5, 1.5),
                                                  ("c2", 20000, 100, 50, 1.0),
                                                  ("c2", 3000, 300, 1, 1.0)])
def test_afkmc2_matches_oracle(skm, torch_cuda, name, n, k, chain, alpha):
    torch = torch_cuda
    say("case afkmc2 %s n=%s k=%d chain=%d alpha=%g" % (name, n, k, chain, alpha))
    X, _, _ = datagen.sparse_workload(name, n)
    u = np.random.default_rng(k + chain).random(1 + (k - 1) * (2 * chain - 1))
    ref = oracle.afkmc2(X, k, chain, alpha, u)
    Xd = skm.DeviceCSR.from_host(X)
    ch, C = skm.seed_afkmc2(Xd, k, chain, u, alpha)
    torch.cuda.synchronize()
    assert np.array_equal(ch.cpu().numpy(), ref)
    assert np.array_equal(C.cpu().numpy(), datagen.init_centers_csr(X, ref))


# ------------------------------------------------------------ dense rows
def dense_csr(D):
    """A dense matrix as the CSR matrix that stores every column (what the
    oracle reads)."""
    n, d = D.shape
    rp = np.arange(0, n * d + 1, d, dtype=np.int64)
    return datagen.CSR(n, d, rp, np.tile(np.arange(d, dtype=np.int32), n),
                       np.ascontiguousarray(D, np.float32).ravel())


@pytest.mark.parametrize("n,d,k,alpha", [(3000, 64, 20, 1.0), (5000, 200, 150, 1.5),
                                         (2000, 37, 7, 1.0)])
def test_seeding_dense_matches_oracle(skm, torch_cuda, n, d, k, alpha):
    torch = torch_cuda
    say("case seed dense n=%d d=%d k=%d alpha=%g" % (n, d, k, alpha))
    X = datagen.dense_vmf(n, d, max(4, k // 3), 700 + d)
    u = np.random.default_rng(k + d).random(k)
    ch_ref, a_ref, s1_ref, s2_ref = oracle.kmeanspp(dense_csr(X), k, alpha, u)
    Xd = skm.DeviceDense.from_host(X)
    ch, C, a, s1, s2 = skm.seed_kmeanspp(Xd, k, u, alpha)
    torch.cuda.synchronize()
    assert np.array_equal(ch.cpu().numpy(), ch_ref)
    assert np.array_equal(C.cpu().numpy(), X[ch_ref].astype(np.float32))
    assert np.array_equal(a.cpu().numpy(), a_ref)
    assert np.abs(s1.cpu().numpy() - s1_ref).max() < 1e-12
    fin = np.isfinite(s2_ref)
    assert np.array_equal(np.isfinite(s2.cpu().numpy()), fin)
    assert np.abs(s2.cpu().numpy()[fin] - s2_ref[fin]).max(initial=0.0) < 1e-12


@pytest.mark.parametrize("n,d,k,chain", [(3000, 64, 20, 20), (2000, 37, 9, 1)])
def test_afkmc2_dense_matches_oracle(skm, torch_cuda, n, d, k, chain):
    torch = torch_cuda
    say("case afkmc2 dense n=%d d=%d k=%d chain=%d" % (n, d, k, chain))
    X = datagen.dense_vmf(n, d, max(4, k // 3), 800 + d)
    u = np.random.default_rng(k + chain).random(1 + (k - 1) * (2 * chain - 1))
    ref = oracle.afkmc2(dense_csr(X), k, chain, 1.0, u)
    Xd = skm.DeviceDense.from_host(X)
    ch, C = skm.seed_afkmc2(Xd, k, chain, u, 1.0)
    torch.cuda.synchronize()
    assert np.array_equal(ch.cpu().numpy(), ref)
    assert np.array_equal(C.cpu().numpy(), X[ref].astype(np.float32))


@pytest.mark.parametrize("variant,precision", [("lloyd", 0), ("hamerly", 0), ("hamerly", 1),
                                               ("simp_hamerly", 1)])
def test_warm_start_dense_equals_cold_fit(skm, torch_cuda, variant, precision):
    """Dense rows: a fit started from the seeding's cached first step ends
    exactly where the cold fit from the same centres does (tests at every
    step, so the warm bounds are used from step 2 on)."""
    torch = torch_cuda
    X = datagen.dense_vmf(20000, 128, 40, 4343)
    k = 64
    u = np.random.default_rng(5).random(k)
    Xd = skm.DeviceDense.from_host(X)
    ch, C, a, s1, s2 = skm.seed_kmeanspp(Xd, k, u)
    say("case warm start dense %s precision=%d" % (variant, precision))
    ac, Cc, _, stc = skm.fit(Xd, k, C, variant, 40, precision=precision, schedule=1)
    aw, Cw, _, stw = skm.fit(Xd, k, C, variant, 40, precision=precision, schedule=1,
                             warm=(a, s1, s2))
    torch.cuda.synchronize()
    assert torch.equal(ac, aw) and torch.equal(Cc, Cw)
    assert stc.iterations == stw.iterations and stc.converged == stw.converged
    assert np.array_equal(stc.changed_per_iter, stw.changed_per_iter)
    assert stw.sims_point_center < stc.sims_point_center
    say("  iterations %d, sims cold %d warm %d" % (stc.iterations, stc.sims_point_center,
                                                  stw.sims_point_center))
    if variant == "hamerly" and precision == 1:
        ref = oracle.fit(dense_csr(X), X[ch.cpu().numpy()].astype(np.float32), "lloyd", 40)
        assert ref.iterations == stw.iterations
        assert np.array_equal(aw.cpu().numpy(), ref.a)
