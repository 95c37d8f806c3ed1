"""Pins for the FP64 oracle.  Each test ties the oracle to something other
than itself: an identity of the paper's Section 2-5 mathematics, explicit
angles, an exhaustive search, numpy's independent dense arithmetic, or a
special case with a closed-form answer."""
import math

import numpy as np
import pytest

import datagen
import oracle


def dense_csr(D):
    n, d = D.shape
    rp = np.arange(0, n * d + 1, d, dtype=np.int64)
    col = np.tile(np.arange(d, dtype=np.int32), n)
    return datagen.CSR(n, d, rp, col, np.ascontiguousarray(D, dtype=np.float32).ravel())


def unit_rows(rng, n, d):
    D = rng.normal(size=(n, d))
    return D / np.linalg.norm(D, axis=1, keepdims=True)


def numpy_argmax_rule(S, prev=None):
    """Independent tie rule: keep prev when it attains the row max, else the
    lowest index among the maxima."""
    mx = S.max(axis=1)
    a = np.argmax(S == mx[:, None], axis=1)
    if prev is not None:
        keep = (prev >= 0) & (S[np.arange(len(S)), np.maximum(prev, 0)] == mx)
        a = np.where(keep, prev, a)
    return a


# ---------------------------------------------------------------- Section 2

def test_sim_matches_euclidean_identity():
    """Eq. (1)-(2): <x,c> = (|x|^2 + |c|^2 - |x-c|^2)/2 = 1 - d^2/2 on unit
    vectors."""
    X = datagen.sparse_tfidf(300, 2000, 30.0, 5)
    rng = np.random.default_rng(0)
    C = unit_rows(rng, 7, X.d)
    S = oracle.sims(X, C, np.arange(X.n))
    Xd = X.to_dense().astype(np.float64)
    d2 = ((Xd[:, None, :] - C[None, :, :]) ** 2).sum(-1)
    xn = (Xd ** 2).sum(1)[:, None]
    expand = (xn + 1.0 - d2) / 2.0
    assert np.abs(S - expand).max() < 1e-13
    # stored rows are unit to float rounding: Eq. (2) holds to that level
    assert np.abs(S - (1.0 - d2 / 2.0)).max() < 1e-6


# ---------------------------------------------------------------- Section 3

@pytest.mark.parametrize("d", [2, 3, 10, 300])
def test_cosine_triangle_inequalities(d):
    """Eq. (4) <= sim(x,y) <= Eq. (5) for exact similarities, and Eq. (3)'s
    arc-length form equals Eq. (4)."""
    rng = np.random.default_rng(d)
    for _ in range(2000):
        x, y, z = unit_rows(rng, 3, d)
        sxz, szy, sxy = float(x @ z), float(z @ y), float(x @ y)
        lo = oracle.lower_unguarded(sxz, szy)
        hi = oracle.upper_unguarded(sxz, szy)
        assert lo <= sxy + 1e-12 and sxy <= hi + 1e-12
        arc = math.cos(math.acos(max(-1, min(1, sxz))) + math.acos(max(-1, min(1, szy))))
        assert abs(arc - lo) < 1e-9


# ------------------------------------------------------ Section 4 bounds

def test_guarded_bounds_cover_exact_worst_case():
    """Guarded Eq. (6)/(7) never cut into the region reachable after a move
    by angle acos(p) (triangle inequality on arc length), and equal the
    exact worst case; the printed forms without guards do cut in."""
    rng = np.random.default_rng(1)
    bad_u = bad_l = 0
    for _ in range(50000):
        tu, tp = rng.uniform(0, math.pi), rng.uniform(0, math.pi)
        u, p = math.cos(tu), math.cos(tp)
        g = oracle.upper_update(u, p)
        exact = oracle.angle_upper(u, p)
        assert g >= exact - 1e-12
        assert abs(g - exact) < 1e-7
        if oracle.upper_unguarded(u, p) < exact - 1e-9:
            bad_u += 1
        gl = oracle.lower_update(u, p)
        exact_l = oracle.angle_lower(u, p)
        assert gl <= exact_l + 1e-12
        assert abs(gl - exact_l) < 1e-7
        if oracle.lower_unguarded(u, p) > exact_l + 1e-9:
            bad_l += 1
    assert bad_u > 1000 and bad_l > 1000


def test_unguarded_upper_bound_counterexample():
    """A point at angle 0.3 from a centre that moves 0.1 sideways and then
    0.3 towards the point: the printed Eq. (7) applied twice bounds the
    similarity by cos(0.1), yet the centre ends almost on the point."""
    x = np.array([1.0, 0.0, 0.0])
    c0 = np.array([math.cos(0.3), math.sin(0.3), 0.0])
    # move 0.1 perpendicular to the x-c0 plane
    c1 = math.cos(0.1) * c0 + math.sin(0.1) * np.array([0.0, 0.0, 1.0])
    p1 = float(c0 @ c1)
    # move from c1 towards x along the great circle by 0.3
    th1 = math.acos(float(x @ c1))
    w = x - (x @ c1) * c1
    w /= np.linalg.norm(w)
    c2 = math.cos(0.3) * c1 + math.sin(0.3) * w
    p2 = float(c1 @ c2)
    true_sim = float(x @ c2)
    u0 = float(x @ c0)
    raw = oracle.upper_unguarded(oracle.upper_unguarded(u0, p1), p2)
    guarded = oracle.upper_update(oracle.upper_update(u0, p1), p2)
    assert th1 > 0.3 and true_sim > raw + 1e-3  # printed form is violated
    assert guarded >= true_sim


def test_half_angle_and_cc_algebra():
    """Section 5.2: cos(acos(x)/2) = sqrt((x+1)/2), and the proof's step
    l(2l^2-1) + sqrt((1-l^2)(1-(2l^2-1)^2)) = l on [0,1]."""
    for g in np.linspace(-1, 1, 2001):
        assert abs(oracle.cc(g) - math.cos(0.5 * math.acos(g))) < 1e-12
    for l in np.linspace(0, 1, 2001):
        assert abs(oracle.upper_unguarded(l, 2 * l * l - 1) - l) < 2e-7
        assert abs(oracle.upper_unguarded(l, 2 * l * l - 1) - l) < 1e-12 or l > 0.999


def test_hamerly_bound_forms():
    """Section 5.3: on [0,1]^2 the guarded Eq. (7) with the largest movement
    is never looser than min(1, Eq. (9)); both cover the exact worst case;
    Eq. (9) is invalid once cosines may be negative."""
    rng = np.random.default_rng(2)
    for _ in range(20000):
        u, p = rng.uniform(0, 1), rng.uniform(0, 1)
        tight = oracle.upper_update(u, p)
        eq9 = min(1.0, u + math.sqrt((1 - u * u) * (1 - p * p)))
        assert tight <= eq9 + 1e-12
        assert abs(oracle.upper_eq9(u, p) - eq9) < 1e-12
        exact = oracle.angle_upper(u, p)
        assert tight >= exact - 1e-12 and eq9 >= exact - 1e-12
    # negative u: Eq. (9) as printed falls below the exact worst case
    u, p = -0.9, 0.2
    assert min(1.0, u + math.sqrt((1 - u * u) * (1 - p * p))) < oracle.angle_upper(u, p)
    assert oracle.upper_eq9(u, p) >= oracle.angle_upper(u, p) - 1e-12


# ------------------------------------------------------ Section 5 steps

def test_assignment_is_exhaustive_argmax_with_tie_rule():
    X = datagen.sparse_tfidf(500, 1500, 25.0, 9)
    rng = np.random.default_rng(3)
    C = unit_rows(rng, 12, X.d)
    C[5] = C[2]  # exact duplicate: ties resolved to the lower index
    a, s1, s2 = oracle.assign(X, C)
    S = X.to_dense().astype(np.float64) @ C.T
    srt = np.sort(S, axis=1)
    gap = srt[:, -1] - srt[:, -2]
    ref = numpy_argmax_rule(S)
    clear = gap > 1e-12
    assert np.array_equal(a[clear], ref[clear])
    assert np.all(a != 5)
    assert np.allclose(s1, S.max(1), atol=1e-14)
    # previous assignment kept when it attains the maximum
    prev = np.where(a == 2, 5, a).astype(np.int32)
    a2, _, _ = oracle.assign(X, C, prev)
    assert np.array_equal(a2, prev)


def test_transposed_assignment_identical_and_exhaustive():
    """The transposed-centre assignment step (used for the full-size
    trajectories) computes the same sequential sums: identical to the plain
    step bit for bit, and the exhaustive argmax of numpy's dense product."""
    X = datagen.sparse_tfidf(700, 2000, 30.0, 19)
    rng = np.random.default_rng(8)
    C = unit_rows(rng, 37, X.d)
    C[11] = C[4]
    a, s1, s2 = oracle.assign(X, C)
    at, s1t, s2t = oracle.assign(X, C, transposed=True)
    assert np.array_equal(a, at) and np.array_equal(s1, s1t) and np.array_equal(s2, s2t)
    S = X.to_dense().astype(np.float64) @ C.T
    srt = np.sort(S, axis=1)
    clear = (srt[:, -1] - srt[:, -2]) > 1e-12
    assert np.array_equal(at[clear], numpy_argmax_rule(S)[clear])
    assert np.all(at != 11)
    prev = np.where(at == 4, 11, at).astype(np.int32)
    a2, _, _ = oracle.assign(X, C, prev, transposed=True)
    assert np.array_equal(a2, prev)


@pytest.mark.parametrize("which", ["c1", "c2"])
def test_lloyd_trajectory_equals_fit(which):
    """The step-by-step Lloyd driver (checkpoints of the full-size
    trajectories) reproduces the oracle's own Lloyd fit exactly: every
    assignment, the centres, the changed counts and objectives."""
    X, init, cfg = datagen.sparse_workload(which, n=None if which == "c1" else 3000)
    C0 = datagen.init_centers_csr(X, init)
    ref = oracle.fit(X, C0, "lloyd", 30, trace=True)
    seen = []

    def on_step(t, a, C, s1, s2, changed, obj):
        assert np.array_equal(a, ref.a_trace[:, t - 1])
        assert changed == ref.changed[t - 1]
        assert np.all(s1 >= s2)
        if obj is None:
            assert np.isnan(ref.obj_update[t - 1])
        else:
            assert obj == ref.obj_update[t - 1]
        seen.append(t)

    a, C, it, conv = oracle.lloyd_trajectory(X, C0, 30, on_step)
    assert it == ref.iterations and conv == ref.converged
    assert seen == list(range(1, it + 1))
    assert np.array_equal(a, ref.a) and np.array_equal(C, ref.C)


def test_update_unit_centres_and_objective():
    X = datagen.sparse_tfidf(800, 3000, 30.0, 10)
    k = 9
    rng = np.random.default_rng(4)
    a = rng.integers(0, k - 1, size=X.n).astype(np.int32)  # cluster k-1 empty
    Cp = unit_rows(rng, k, X.d)
    C, norms, obj = oracle.update(X, a, Cp)
    Xd = X.to_dense().astype(np.float64)
    S = np.zeros((k, X.d))
    np.add.at(S, a, Xd)
    assert np.allclose(norms, np.linalg.norm(S, axis=1), rtol=1e-13)
    for j in range(k - 1):
        assert abs(np.linalg.norm(C[j]) - 1.0) < 1e-14
        assert np.abs(C[j] - S[j] / np.linalg.norm(S[j])).max() < 1e-14
    assert np.array_equal(C[k - 1], Cp[k - 1])  # empty cluster keeps its centre
    # Cauchy-Schwarz: the new centres realise sum_i <x_i, c_a(i)> = sum_j |S_j|
    assert abs(obj - float((Xd * C[a]).sum())) < 1e-9 * obj


def test_objective_monotone_c1():
    X, init, cfg = datagen.sparse_workload("c1")
    C0 = datagen.init_centers_csr(X, init)
    r = oracle.fit(X, C0, "lloyd", 100)
    assert r.converged
    seq = []
    for t in range(r.iterations):
        seq.append(r.obj_assign[t])
        if not np.isnan(r.obj_update[t]):
            seq.append(r.obj_update[t])
    seq = np.array(seq)
    assert np.all(np.diff(seq) >= -1e-12 * seq[1:])


def _check_variants_equal(X, C0, max_iter, check=True):
    ref = oracle.fit(X, C0, "lloyd", max_iter, trace=True)
    for v in ["elkan", "hamerly", "simp_elkan", "simp_hamerly", "yinyang"]:
        for bf in (0, 1):
            if bf == 1 and ("elkan" in v or v == "yinyang"):
                continue
            r = oracle.fit(X, C0, v, max_iter, bound_form=bf, trace=True, check_bounds=check)
            assert r.iterations == ref.iterations, (v, bf)
            assert np.array_equal(r.a_trace, ref.a_trace), (v, bf)
            assert np.array_equal(r.C, ref.C), (v, bf)
            assert r.violations == 0, (v, bf)
            assert r.sims.sum() <= ref.sims.sum()
    return ref


def test_variants_equal_lloyd_c1():
    X, init, cfg = datagen.sparse_workload("c1")
    ref = _check_variants_equal(X, datagen.init_centers_csr(X, init), 100)
    assert ref.converged


def test_variants_equal_lloyd_reduced_c2():
    X, init, cfg = datagen.sparse_workload("c2", n=4000)
    _check_variants_equal(X, datagen.init_centers_csr(X, init), 25, check=False)


@pytest.mark.parametrize("seed", range(12))
def test_variants_equal_lloyd_adversarial_low_dim(seed):
    """Mixed-sign data in d = 2, 3: negative cosines and large centre moves
    exercise every guard."""
    rng = np.random.default_rng(seed)
    d = 2 + seed % 2
    n = 60 + 11 * seed
    k = 2 + seed % 6
    D = unit_rows(rng, n, d)
    X = dense_csr(D)
    C0 = D[rng.choice(n, k, replace=False)].astype(np.float32)
    _check_variants_equal(X, C0, 200)


@pytest.mark.parametrize("seed", range(4))
def test_yinyang_several_groups_low_dim(seed):
    """Yin-Yang with 2-3 groups of 32 centres on mixed-sign d = 3 data: the
    group filter, the old centre joining its group's bound and every guard
    in play; same trajectory as Lloyd, no bound violation, fewer sims."""
    rng = np.random.default_rng(50 + seed)
    D = unit_rows(rng, 500, 3)
    X = dense_csr(D)
    k = 40 + 13 * seed
    C0 = D[rng.choice(500, k, replace=False)].astype(np.float32)
    ref = oracle.fit(X, C0, "lloyd", 200, trace=True)
    r = oracle.fit(X, C0, "yinyang", 200, trace=True, check_bounds=True)
    assert r.iterations == ref.iterations
    assert np.array_equal(r.a_trace, ref.a_trace) and np.array_equal(r.C, ref.C)
    assert r.violations == 0
    assert r.sims.sum() < ref.sims.sum()


def test_guards_are_necessary():
    """Planted mistake in the oracle only: the printed Eq. (6)/(7) without
    guards (bound_form=2) prunes a centre that Lloyd picks on this case
    (found by a search over small mixed-sign problems); the guarded
    Hamerly matches Lloyd."""
    rng = np.random.default_rng(1)
    d = int(rng.choice([2, 3]))
    n = int(rng.integers(20, 200))
    k = int(rng.integers(2, 8))
    D = unit_rows(rng, n, d)
    X = dense_csr(D)
    C0 = D[rng.choice(n, k, replace=False)].astype(np.float32)
    ref = oracle.fit(X, C0, "lloyd", 200, trace=True)
    good = oracle.fit(X, C0, "hamerly", 200, trace=True, check_bounds=True)
    bad = oracle.fit(X, C0, "hamerly", 200, bound_form=2, trace=True, check_bounds=True)
    assert good.violations == 0 and np.array_equal(good.a_trace, ref.a_trace)
    assert bad.violations > 0
    assert bad.iterations != ref.iterations or not np.array_equal(bad.a_trace, ref.a_trace)


# ------------------------------------------------------ exhaustive search

@pytest.mark.parametrize("seed", range(6))
def test_brute_force_tiny(seed):
    rng = np.random.default_rng(100 + seed)
    n, k, d = 7, 2 + seed % 2, 2 + seed % 3
    D = np.abs(unit_rows(rng, n, d)) if seed % 2 else unit_rows(rng, n, d)
    D = D.astype(np.float32).astype(np.float64)
    best, lab = oracle.brute_force_best_partition(D, k)
    X = dense_csr(D)
    r = oracle.fit(X, D[rng.choice(n, k, replace=False)], "lloyd", 100)
    assert r.obj_update[~np.isnan(r.obj_update)].max() <= best + 1e-12
    # the optimal partition's centres are a fixed point of Lloyd
    S = np.zeros((k, d))
    np.add.at(S, lab, D)
    used = np.linalg.norm(S, axis=1) > 0
    if used.all():
        Copt = S / np.linalg.norm(S, axis=1, keepdims=True)
        r2 = oracle.fit(X, Copt, "lloyd", 10)
        assert r2.iterations == 2 and r2.changed[1] == 0
        assert abs(r2.obj_update[0] - best) < 1e-12


# ------------------------------------------------------ special cases

def test_k_equals_one():
    X = datagen.sparse_tfidf(300, 800, 20.0, 12)
    C0 = datagen.init_centers_csr(X, np.array([4]))
    r = oracle.fit(X, C0, "hamerly", 10)
    assert r.iterations == 2 and r.converged and np.all(r.a == 0)
    s = X.to_dense().astype(np.float64).sum(0)
    assert np.abs(r.C[0] - s / np.linalg.norm(s)).max() < 1e-14


def test_k_equals_n_distinct():
    rng = np.random.default_rng(5)
    D = np.abs(unit_rows(rng, 25, 6))
    X = dense_csr(D)
    r = oracle.fit(X, D.astype(np.float32), "elkan", 10)
    assert r.iterations == 2 and r.converged
    assert np.array_equal(r.a, np.arange(25))
    assert abs(r.obj_update[0] - 25.0) < 1e-5


def test_duplicate_init_rows_keep_empty_cluster():
    X = datagen.sparse_tfidf(400, 1000, 20.0, 13)
    init = np.array([3, 3, 10, 20])
    C0 = datagen.init_centers_csr(X, init)
    ref = oracle.fit(X, C0, "lloyd", 50, trace=True)
    assert not np.any(ref.a_trace[:, 0] == 1)  # step 1: ties go to index 0
    one = oracle.fit(X, C0, "lloyd", 1)
    c1 = C0[1].astype(np.float64)
    # cluster 1 was empty after step 1 and keeps its (unit) centre
    assert np.abs(one.C[1] - c1 / np.linalg.norm(c1)).max() < 1e-15
    for v in ["elkan", "hamerly"]:
        r = oracle.fit(X, C0, v, 50, trace=True)
        assert np.array_equal(r.a_trace, ref.a_trace)


def test_init_at_fixed_point_converges_at_step_two():
    X, init, cfg = datagen.sparse_workload("c1")
    r = oracle.fit(X, datagen.init_centers_csr(X, init), "lloyd", 100)
    r2 = oracle.fit(X, r.C, "hamerly", 100)
    assert r2.iterations == 2 and r2.changed[1] == 0
    assert np.array_equal(r2.a, r.a)


def test_d2_arcs_by_hand():
    """On the unit circle the assignment is the nearest centre in angle."""
    ang = np.linspace(0.05, 2 * math.pi - 0.05, 40)
    D = np.stack([np.cos(ang), np.sin(ang)], 1)
    cang = np.array([0.5, 2.0, 4.0])
    C = np.stack([np.cos(cang), np.sin(cang)], 1)
    a, _, _ = oracle.assign(dense_csr(D), C)
    diff = np.abs((ang[:, None] - cang[None, :] + math.pi) % (2 * math.pi) - math.pi)
    assert np.array_equal(a, np.argmin(diff, axis=1))


# ---------------------------------------------- Section 5.6, spherical k-means++

def _circle(deg):
    """Unit vectors at the given angles; multiples of 90 degrees are exact."""
    a = np.radians(np.asarray(deg, dtype=np.float64))
    P = np.stack([np.cos(a), np.sin(a)], 1)
    exact = np.asarray(deg) % 90 == 0
    P[exact] = np.rint(P[exact])
    return dense_csr(P)


def test_kmeanspp_by_hand():
    """Points at 0, 10, 90, 180 and 270 degrees, alpha = 1.  u0 = 0.1 picks
    row floor(0.5) = 0.  Weights 1 - cos(angle to 0 deg) are then
    (0, 0.01519, 1, 2, 1), total 4.01519, so u1 = 0.6 (target 2.40911) is
    first exceeded at the 180 degree row (running sums 0, 0.0152, 1.0152,
    3.0152).  With centres at 0 and 180 the weights are (0, 0.01519, 1, 0,
    1), total 2.01519: u2 = 0.5 (target 1.00760) stops at the 90 degree row
    (running sum 1.01519) and u2 = 0.51 (target 1.02775) passes it and stops
    at 270 degrees."""
    X = _circle([0, 10, 90, 180, 270])
    ch, a, s1, s2 = oracle.kmeanspp(X, 3, 1.0, np.array([0.1, 0.6, 0.5]))
    assert list(ch) == [0, 3, 2]
    # the cached step: 10 deg -> centre 0 (cos 10 vs cos 80); 270 deg is at
    # 90 deg from centres 0 and 1 alike: the lower index wins
    assert list(a) == [0, 0, 2, 1, 0]
    c10, c80 = math.cos(math.radians(10)), math.cos(math.radians(80))
    assert np.allclose(s1, [1, c10, 1, 1, 0], atol=1e-6)
    assert np.allclose(s2, [0, c80, 0, 0, 0], atol=1e-6)
    ch, _, _, _ = oracle.kmeanspp(X, 3, 1.0, np.array([0.1, 0.6, 0.51]))
    assert list(ch) == [0, 3, 4]


def test_kmeanspp_alpha_and_edge_draws():
    """alpha = 1 gives a duplicate of a chosen row weight 0; the metric form
    alpha = 1.5 gives it 0.5, so u = 0 (first row of positive weight) picks
    it.  u just below 1 picks the last row of positive weight."""
    X = _circle([0, 0, 90, 200])
    ch, _, _, _ = oracle.kmeanspp(X, 2, 1.0, np.array([0.0, 0.0]))
    assert list(ch) == [0, 2]
    ch, _, _, _ = oracle.kmeanspp(X, 2, 1.5, np.array([0.0, 0.0]))
    assert list(ch) == [0, 1]
    ch, _, _, _ = oracle.kmeanspp(X, 2, 1.0, np.array([0.0, 1.0 - 1e-12]))
    assert list(ch) == [0, 3]


def test_kmeanspp_all_weights_zero():
    """Identical, exactly unit rows: after the first draw every weight is 0
    (alpha = 1), so the lowest-index rows not yet chosen follow."""
    X = _circle([90, 90, 90, 90])
    ch, a, _, _ = oracle.kmeanspp(X, 3, 1.0, np.array([0.9, 0.5, 0.5]))
    assert list(ch) == [3, 0, 1]
    assert np.all(a == 0)  # equal similarities: the lowest centre index


def test_kmeanspp_cache_equals_assignment_step():
    """The running maximum cached during seeding equals the exhaustive
    assignment step against the chosen rows (unit length), and no row is
    drawn twice."""
    X, _, _ = datagen.sparse_workload("c1")
    u = np.random.default_rng(5).random(10)
    for alpha in (1.0, 1.5):
        ch, a, s1, s2 = oracle.kmeanspp(X, 10, alpha, u)
        assert len(set(ch.tolist())) == 10
        C = datagen.init_centers_csr(X, ch).astype(np.float64)
        C /= np.linalg.norm(C, axis=1, keepdims=True)
        a2, t1, t2 = oracle.assign(X, C)
        assert np.array_equal(a, a2)
        assert np.max(np.abs(s1 - t1)) < 1e-13 and np.max(np.abs(s2 - t2)) < 1e-13


def test_afkmc2_by_hand():
    """Four exact points at 0, 90, 180, 270 degrees, alpha = 1, u0 = 0.1:
    centre 0 is row 0, weights 1 - <x, c0> = (0, 1, 2, 1), W = 4, so
    q = w / 8 + 1 / 8 = (0.125, 0.25, 0.375, 0.25), running sums 0.125,
    0.375, 0.75, 1.  Chain of two proposals (draws up0, up1; acceptance
    draw ua): y2 replaces y1 when d(y2) q(y1) > ua d(y1) q(y2)."""
    X = _circle([0, 90, 180, 270])
    # y1 = row 1 (0.2), y2 = row 2 (0.5): 2 * 0.25 > ua * 1 * 0.375 always
    assert list(oracle.afkmc2(X, 2, 2, 1.0, np.array([0.1, 0.2, 0.5, 0.99]))) == [0, 2]
    # y1 = row 2, y2 = row 1: 1 * 0.375 > ua * 2 * 0.25 iff ua < 0.75
    assert list(oracle.afkmc2(X, 2, 2, 1.0, np.array([0.1, 0.5, 0.3, 0.7]))) == [0, 1]
    assert list(oracle.afkmc2(X, 2, 2, 1.0, np.array([0.1, 0.5, 0.3, 0.8]))) == [0, 2]
    # chain length 1: the proposal itself (inverse transform on q)
    assert list(oracle.afkmc2(X, 2, 1, 1.0, np.array([0.1, 0.74]))) == [0, 2]
    assert list(oracle.afkmc2(X, 2, 1, 1.0, np.array([0.1, 0.76]))) == [0, 3]
    # both proposals on the centre itself: d = 0 twice, the chain stays
    assert list(oracle.afkmc2(X, 2, 2, 1.0, np.array([0.1, 0.05, 0.1, 0.5]))) == [0, 0]
    # third centre with centres at 0 and 180 degrees: d = (0, 1, 0, 1);
    # y1 = row 2 (d 0), y2 = row 3 (d 1): 1 * 0.375 > 0 always
    u = np.array([0.1, 0.2, 0.5, 0.99, 0.5, 0.9, 0.3])
    assert list(oracle.afkmc2(X, 3, 2, 1.0, u)) == [0, 2, 3]


def test_afkmc2_long_chain_prefers_far_rows():
    """With a long chain the draw concentrates where alpha - max <x, c> is
    large: on two well separated clusters the second centre lands in the
    other cluster far more often than the uniform share."""
    rng = np.random.default_rng(3)
    a = np.array([1.0, 0.0, 0.0])
    b = np.array([0.0, 0.0, 1.0])
    P = np.concatenate([a + 0.05 * rng.normal(size=(90, 3)), b + 0.05 * rng.normal(size=(10, 3))])
    P /= np.linalg.norm(P, axis=1, keepdims=True)
    X = dense_csr(P)
    hits = 0
    for s in range(60):
        u = np.random.default_rng(100 + s).random(1 + 2 * 20 - 1)
        u[0] = 0.05  # centre 0 in the large cluster
        ch = oracle.afkmc2(X, 2, 20, 1.0, u)
        hits += ch[1] >= 90
    assert hits >= 50  # the small cluster holds 10% of the rows


# ------------------------------------------- dense FP64 oracle (numpy product)

def test_dense_oracle_matches_csr_oracle():
    """The numpy dense Lloyd used for the full-size dense trajectory equals
    the CSR oracle on the same rows stored densely: identical trajectory,
    centres and objectives to rounding (1e-13)."""
    from oracle import dense as od
    X = datagen.dense_vmf(3000, 40, 12, 321)
    init = datagen.init_rows(X.shape[0], 12, 321)
    C0 = X[init].copy()
    ref = oracle.fit(dense_csr(X), C0, "lloyd", 40, trace=True)
    got = []

    def on_step(t, a, C, s1, s2, changed, obj):
        assert np.array_equal(a, ref.a_trace[:, t - 1])
        assert changed == ref.changed[t - 1]
        if obj is not None:
            assert abs(obj - ref.obj_update[t - 1]) < 1e-12 * obj
        got.append(t)

    a, C, it, conv = od.lloyd_trajectory(X, C0, 40, on_step)
    assert it == ref.iterations and conv == ref.converged and len(got) == it
    assert np.abs(C - ref.C).max() < 1e-13


def test_dense_oracle_assign_rules():
    """Tie rule and second best on a hand-made case: duplicate centres, a
    previous assignment that attains the maximum, k = 1."""
    from oracle import dense as od
    X = np.array([[1, 0, 0], [0, 1, 0], [0.6, 0.8, 0]], np.float32)
    C = np.array([[0, 1, 0], [1, 0, 0], [0, 1, 0]], np.float64)
    a, s1, s2 = od.assign(X, C)
    assert list(a) == [1, 0, 0]  # row 1 ties centres 0 and 2: lowest index
    assert np.allclose(s1, [1, 1, 0.8]) and np.allclose(s2, [0, 1, 0.8])
    a2, _, _ = od.assign(X, C, np.array([1, 2, 2], np.int32))
    assert list(a2) == [1, 2, 2]  # previous centre kept where it attains the max
    a1, s1, s2 = od.assign(X, C[:1])
    assert list(a1) == [0, 0, 0] and np.all(np.isneginf(s2))
    Cn, norms, obj = od.update(X, np.array([1, 0, 0], np.int32), np.eye(3)[:3])
    s0 = X[1].astype(np.float64) + X[2].astype(np.float64)  # float32 rows, exact sum
    assert np.allclose(Cn[0], s0 / np.linalg.norm(s0), rtol=0, atol=1e-15)
    assert np.array_equal(Cn[2], np.eye(3)[2])  # empty cluster keeps its centre
    assert abs(obj - (np.linalg.norm(s0) + 1.0)) < 1e-15
