"""skm_assign_noalloc (library-owned scratch, no allocation inside the call)
against skm_assign through the C ABI: identical outputs, bit for bit, on two
calls in a row (the second smaller, so it runs on the first call's leftover
scratch contents), for both row mappings (k <= 64 and k > 64); and a
problem beyond the buffer is refused before anything is enqueued."""
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
    return torch, skm


def one(torch, skm, n, d, mean, k, seed):
    X = datagen.sparse_tfidf(n, d, mean, seed)
    C = datagen.init_centers_csr(X, datagen.init_rows(X.n, k, seed))
    Xd = skm.DeviceCSR.from_host(X, "cuda:0")
    Cd = torch.from_numpy(C).cuda()
    print("case noalloc n=%d d=%d k=%d" % (X.n, d, k), flush=True)
    a0, b0, s0 = skm.assign(Xd, Cd)
    sec = torch.empty(X.n, dtype=torch.float32, device="cuda:0")
    a1, b1, s1 = skm.assign_noalloc(Xd, Cd, second=sec)
    torch.cuda.synchronize()
    assert torch.equal(a0, a1)
    assert torch.equal(b0, b1)
    assert torch.equal(s0, s1)
    return a1


@pytest.mark.parametrize("first,second", [((12000, 8000, 40.0, 300), (5000, 3000, 30.0, 37)),
                                          ((6000, 4000, 30.0, 60), (3000, 2000, 20.0, 700))])
def test_noalloc_matches_assign_twice(env, first, second):
    torch, skm = env
    one(torch, skm, *first, seed=11)
    one(torch, skm, *second, seed=12)


def test_noalloc_refuses_oversized(env):
    torch, skm = env
    X = datagen.sparse_tfidf(2000, 60000, 20.0, 13)
    k = 200  # 60000 * 256 * 4 + 200 * 60000 * 8 bytes > 64 MiB
    C = torch.from_numpy(datagen.init_centers_csr(X, datagen.init_rows(X.n, k, 13))).cuda()
    Xd = skm.DeviceCSR.from_host(X, "cuda:0")
    with pytest.raises(skm.SkmError) as e:
        skm.assign_noalloc(Xd, C)
    assert e.value.status == skm.ERR_UNSUPPORTED
    assert "no-allocation buffer" in str(e.value)
    torch.cuda.synchronize()
