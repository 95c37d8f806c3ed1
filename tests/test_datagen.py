"""Input generator checks: determinism, unit rows, CSR structure, statistics."""
import numpy as np

import datagen


def test_sparse_deterministic_and_thread_independent():
    a = datagen.sparse_tfidf(3000, 4000, 40.0, 123)
    b = datagen.sparse_tfidf(3000, 4000, 40.0, 123)
    c = datagen.sparse_tfidf(3000, 4000, 40.0, 124)
    assert np.array_equal(a.row_ptr, b.row_ptr)
    assert np.array_equal(a.col, b.col)
    assert np.array_equal(a.val.view(np.uint32), b.val.view(np.uint32))
    assert not (a.nnz == c.nnz and np.array_equal(a.col, c.col))


def test_sparse_structure():
    X, init, cfg = datagen.sparse_workload("c1")
    rp = X.row_ptr
    assert rp[0] == 0 and np.all(np.diff(rp) >= 1)
    assert X.col.min() >= 0 and X.col.max() < X.d
    for i in range(X.n):
        seg = X.col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(seg) > 0)  # ascending, no repeats
    assert np.all(X.val > 0)  # no explicit zeros
    norms = np.sqrt(np.add.reduceat(X.val.astype(np.float64) ** 2, rp[:-1]))
    assert np.abs(norms - 1.0).max() < 1e-6
    assert len(np.unique(init)) == cfg.k and init.min() >= 0 and init.max() < X.n


def test_sparse_statistics():
    # mean row length close to the requested mean (the always-present top
    # term has idf 0 and is dropped, so slightly fewer entries survive)
    X = datagen.sparse_tfidf(20000, 50000, 100.0, 7)
    m = X.row_lengths()
    assert 90.0 < m.mean() < 101.0
    # Zipf popularity: the most frequent surviving column appears in a large
    # share of rows, the median column in few
    df = np.bincount(X.col, minlength=X.d)
    assert df.max() > 0.3 * X.n
    assert np.median(df) < 0.01 * X.n


def test_sparse_topics_structure_and_default():
    """topics = 0 is the plain generator; with topics the rows keep the CSR
    contract (ascending distinct columns, unit norm) and form clusters: a
    seeded FP64 Lloyd fit with k = topics converges in far fewer steps than
    on plain rows and finds clusters of nearly equal size (the topics)."""
    import oracle
    a = datagen.sparse_tfidf(4000, 3000, 40.0, 99)
    b = datagen.sparse_tfidf(4000, 3000, 40.0, 99, topics=0)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.val, b.val)
    t = datagen.sparse_tfidf(4000, 3000, 40.0, 99, topics=10)
    assert not (t.nnz == a.nnz and np.array_equal(t.col, a.col))
    rp = t.row_ptr
    for i in range(t.n):
        assert np.all(np.diff(t.col[rp[i]:rp[i + 1]]) > 0)
    norms = np.sqrt(np.add.reduceat(t.val.astype(np.float64) ** 2, rp[:-1]))
    assert np.abs(norms - 1.0).max() < 1e-6
    fits = [oracle.fit(X, datagen.init_centers_csr(X, datagen.init_rows(X.n, 10, 5)), "lloyd", 30)
            for X in (a, t)]
    assert fits[1].iterations + 4 <= fits[0].iterations
    sizes = np.bincount(fits[1].a, minlength=10)
    assert np.all(np.abs(sizes - t.n / 10) < 0.25 * t.n / 10)


def test_vmf_rows_unit_and_concentrated():
    X, comp = datagen.dense_vmf(4000, 64, 8, 11, return_components=True)
    nr = np.linalg.norm(X.astype(np.float64), axis=1)
    assert np.abs(nr - 1).max() < 1e-6
    # points of one component are more similar to each other than to others
    same = X[comp == comp[0]]
    other = X[comp != comp[0]]
    mean_same = (same @ same.mean(0)).mean()
    mean_other = (other @ same.mean(0)).mean()
    assert mean_same > mean_other + 0.1


def test_batched_instance_list():
    inst = datagen.batched_instances(n_inst=4, scale=0.05)
    assert len(inst) == 4
    for b in inst:
        assert b.k % 8 == 0 or b.k == b.X.n
        assert len(np.unique(b.init)) == b.k
