"""GPU fits of the two workloads too large for the oracle to run inside a
test, against the oracle's own FP64 Lloyd trajectories stored by
tests/golden/make_full_size.py (the oracle and the input generator only; no
value comes from the GPU):

  c3  sparse tf-idf, n = 1,000,000, d = 100,000, k = 1,000: checkpoints after
      assignment steps 1, 2, 10, 25 and 50
  c4  dense von Mises-Fisher rows, n = 2,000,000, d = 256, k = 4,096, BF16
      matrix cores: every step 1 ... 20

A fit stopped after step t must reproduce the oracle's state after step t:
the whole assignment (SHA-256 of the int32 array) -- or, failing that, the
sampled rows everywhere outside the 1e-5 top-2 band, with the trajectory
reported as diverged from there on --, the changed-row counts of every step,
the objective sum_j |S(j)| within 1e-6 relative, and the FP64 centres at the
stored coordinates within 1e-6.  The input generator is pinned by a SHA-256
of the generated matrix."""
import hashlib
import os

import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, flush=True)


def sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2107_04074_amd import skm
    skm.load()
    return torch, skm


def check_checkpoint(G, i, t, a, C64, st, label):
    """Compares one fit (stopped after step t) with checkpoint i of G.
    Returns False once the trajectory has left the oracle's (a row inside
    the band decided the other way)."""
    rows = G["sample_rows"]
    inband = np.unpackbits(G["inband"][i])[:len(rows)].astype(bool)
    ref = G["a_sample"][i].astype(np.int32)
    mism = a[rows] != ref
    same = sha(a.astype(np.int32)) == str(G["assign_sha"][i])
    say("%s step %d: whole assignment %s; sampled rows %d, in the 1e-5 band %d, mismatches %d "
        "(outside the band %d); sims %d rechecks %d" % (
            label, t, "identical" if same else "DIFFERS", len(rows), int(inband.sum()),
            int(mism.sum()), int((mism & ~inband).sum()), st.sims_point_center, st.rechecks))
    assert not np.any(mism & ~inband), np.flatnonzero(mism & ~inband)[:10]
    assert st.iterations == t
    if not same:
        say("%s: trajectory diverged at step %d inside the band; later checkpoints not "
            "comparable" % (label, t))
        return False
    assert np.array_equal(st.changed_per_iter[:t], G["changed"][:t])
    obj = float(G["objective"][i])
    if not np.isnan(obj):
        assert abs(st.objective - obj) <= 1e-6 * obj, (st.objective, obj)
    cl = G["clusters"]
    if "centre_cols" in G.files:
        got = np.take_along_axis(C64[cl], G["centre_cols"][i].astype(np.int64), axis=1)
    else:
        got = C64[cl]
    err = np.abs(got - G["centre_vals"][i]).max()
    say("%s step %d: objective %.9g (oracle %.9g), centre coordinates max error %.2e" % (
        label, t, st.objective, obj, err))
    assert err <= 1e-6
    return True


def run(torch, skm, Xd, k, C0, variant, t, precision):
    a, _, C64, st = skm.fit(Xd, k, torch.from_numpy(C0).cuda(), variant, t,
                            want_centers=False, want_centers64=True, precision=precision)
    torch.cuda.synchronize()
    return a.cpu().numpy(), C64.cpu().numpy(), st


@pytest.mark.parametrize("variant,precision", [("hamerly", 0), ("yinyang", 0), ("simp_elkan", 0),
                                               ("yinyang", 2)])
def test_c3_trajectory_against_oracle(env, variant, precision):
    torch, skm = env
    G = np.load(os.path.join(GOLDEN, "c3_lloyd_trajectory.npz"))
    say("case c3 generate")
    X, init, cfg = datagen.sparse_workload("c3")
    assert sha(np.array([X.n, X.d], np.int64), X.row_ptr, X.col, X.val) == str(G["input_sha"])
    assert np.array_equal(init, G["init_rows"])
    C0 = datagen.init_centers_csr(X, init)
    Xd = skm.DeviceCSR.from_host(X)
    label = "c3 %s precision %d" % (variant, precision)
    for i, t in enumerate(G["step"]):
        say("case %s max_iter=%d" % (label, t))
        a, C64, st = run(torch, skm, Xd, cfg.k, C0, variant, int(t), precision)
        if not check_checkpoint(G, i, int(t), a, C64, st, label):
            break


@pytest.mark.parametrize("variant", ["hamerly", "lloyd"])
def test_c4_trajectory_against_oracle(env, variant):
    torch, skm = env
    G = np.load(os.path.join(GOLDEN, "c4_lloyd_trajectory.npz"))
    cfg = datagen.C4
    say("case c4 generate")
    X = datagen.dense_vmf(cfg["n"], cfg["d"], cfg["n_means"], cfg["seed"])
    assert sha(np.array(X.shape, np.int64), X) == str(G["input_sha"])
    init = datagen.init_rows(X.shape[0], cfg["k"], cfg["seed"])
    assert np.array_equal(init, G["init_rows"])
    C0 = X[init].copy()
    Xd = skm.DeviceDense.from_host(X)
    label = "c4 bf16 %s" % variant
    steps = list(G["step"]) if variant == "hamerly" else [1, 5, 20]
    for t in steps:
        i = int(t) - 1
        say("case %s max_iter=%d" % (label, t))
        a, C64, st = run(torch, skm, Xd, cfg["k"], C0, variant, int(t), 1)
        if not check_checkpoint(G, i, int(t), a, C64, st, label):
            break
