"""GPU tests of the input checks of skm_fit (options.validate).

validate = 1 rejects initial centres that are not unit vectors
(SKM_ERR_NOT_NORMALIZED); validate = 2 also rejects data rows that are not
unit vectors, and malformed inputs with SKM_ERR_INVALID_ARG before any kernel
walks the rows: row_ptr not starting at 0, decreasing, or not ending at nnz;
column ids outside [0, d) or not strictly ascending within a row (sparse
vectors are sorted (index, value) pairs, Section 2 of the paper); NaN or
infinite values.  Every malformed case is built on the host from a valid
matrix by one edit, and only reaches the library with validate = 2."""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2107_04074_amd import skm
    skm.load()
    X = datagen.sparse_tfidf(300, 400, 12.0, 4242)
    init = datagen.init_rows(X.n, 5, 4242)
    C0 = datagen.init_centers_csr(X, init)
    return torch, skm, X, C0


def say(*a):
    print(*a, flush=True)


def device_csr(torch, skm, rp, col, val, n, d):
    return skm.DeviceCSR(n, d, torch.from_numpy(np.asarray(rp, np.int64)).cuda(),
                         torch.from_numpy(np.asarray(col, np.int32)).cuda(),
                         torch.from_numpy(np.asarray(val, np.float32)).cuda())


def fit_status(torch, skm, Xd, C0, validate, k=5, variant="hamerly"):
    try:
        skm.fit(Xd, k, torch.from_numpy(np.ascontiguousarray(C0, np.float32)).cuda(), variant,
                10, validate=validate)
        torch.cuda.synchronize()
        return skm.OK, ""
    except skm.SkmError as e:
        return e.status, str(e)


def test_valid_input_passes_every_level(env):
    torch, skm, X, C0 = env
    Xd = skm.DeviceCSR.from_host(X, "cuda:0")
    outs = []
    for v in (0, 1, 2):
        a, _, _, st = skm.fit(Xd, 5, torch.from_numpy(C0).cuda(), "hamerly", 10, validate=v)
        outs.append((a.cpu().numpy(), st.iterations))
    assert all(np.array_equal(outs[0][0], o[0]) and outs[0][1] == o[1] for o in outs)


def test_non_unit_initial_centre(env):
    torch, skm, X, C0 = env
    Xd = skm.DeviceCSR.from_host(X, "cuda:0")
    C = C0.copy()
    C[3] *= 1.01
    assert fit_status(torch, skm, Xd, C, 0)[0] == skm.OK  # rescaled without checks
    st, msg = fit_status(torch, skm, Xd, C, 1)
    say("validate=1, centre 3 scaled by 1.01:", msg)
    assert st == skm.ERR_NOT_NORMALIZED and "centre 3" in msg


def test_non_unit_row(env):
    torch, skm, X, C0 = env
    val = X.val.copy()
    val[X.row_ptr[7]:X.row_ptr[8]] *= 1.5
    Xd = device_csr(torch, skm, X.row_ptr, X.col, val, X.n, X.d)
    assert fit_status(torch, skm, Xd, C0, 1)[0] == skm.OK
    st, msg = fit_status(torch, skm, Xd, C0, 2)
    say("validate=2, row 7 scaled by 1.5:", msg)
    assert st == skm.ERR_NOT_NORMALIZED


def _malformed(X):
    """(label, row_ptr, col, val, n, d, nnz_override, row named in the error)"""
    rp, col, val = X.row_ptr, X.col, X.val
    lens = X.row_lengths()
    r = 11 + int(np.flatnonzero(lens[11:] >= 3)[0])
    b, e = int(rp[r]), int(rp[r + 1])
    cases = []
    rp1 = rp.copy(); rp1[0] = 1
    cases.append(("row_ptr[0] != 0", rp1, col, val, 0))
    rp2 = rp.copy(); rp2[r + 1] = rp2[r] - 1
    cases.append(("decreasing row_ptr", rp2, col, val, r))
    rp3 = rp.copy(); rp3[-1] = rp3[-1] - 1
    cases.append(("row_ptr[n] != nnz", rp3, col, val, X.n))
    c4 = col.copy(); c4[b + 1] = X.d
    cases.append(("column = d", rp, c4, val, r))
    c5 = col.copy(); c5[b] = -1
    cases.append(("negative column", rp, c5, val, r))
    c6 = col.copy(); c6[b + 1] = c6[b]
    cases.append(("repeated column", rp, c6, val, r))
    c7 = col.copy(); c7[b], c7[b + 1] = col[b + 1], col[b]
    cases.append(("descending columns", rp, c7, val, r))
    v8 = val.copy(); v8[b + 2] = np.nan
    cases.append(("NaN value", rp, col, v8, r))
    v9 = val.copy(); v9[e - 1] = np.inf
    cases.append(("infinite value", rp, col, v9, r))
    return cases


@pytest.mark.parametrize("case", range(9))
def test_malformed_csr_rejected(env, case):
    torch, skm, X, C0 = env
    label, rp, col, val, row = _malformed(X)[case]
    Xd = device_csr(torch, skm, rp, col, val, X.n, X.d)
    st, msg = fit_status(torch, skm, Xd, C0, 2)
    say("validate=2, %s: status %d, %s" % (label, st, msg))
    assert st == skm.ERR_INVALID_ARG
    assert ("%d" % row) in msg


def test_dense_checks(env):
    torch, skm, _, _ = env
    Xh = datagen.dense_vmf(600, 48, 8, 99)
    init = datagen.init_rows(Xh.shape[0], 6, 99)
    C0 = Xh[init].copy()
    good = skm.DeviceDense.from_host(Xh, "cuda:0")
    assert fit_status(torch, skm, good, C0, 2, k=6)[0] == skm.OK
    C = C0.copy()
    C[2] *= 0.9
    st, msg = fit_status(torch, skm, good, C, 1, k=6)
    assert st == skm.ERR_NOT_NORMALIZED and "centre 2" in msg
    Xn = Xh.copy()
    Xn[123, 5] = np.nan
    st, msg = fit_status(torch, skm, skm.DeviceDense.from_host(Xn, "cuda:0"), C0, 2, k=6)
    say("dense NaN:", msg)
    assert st == skm.ERR_INVALID_ARG and "123" in msg
    Xs = Xh.copy()
    Xs[50] *= 1.2
    st, msg = fit_status(torch, skm, skm.DeviceDense.from_host(Xs, "cuda:0"), C0, 2, k=6)
    assert st == skm.ERR_NOT_NORMALIZED
