"""FP64 CPU oracle for accelerated spherical k-means (arXiv 2107.04074).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The GPU library never imports, links or
calls anything here, and this package imports nothing from it.

The arithmetic lives in ``skm_oracle.c`` (plain double loops, built with gcc
into ``liboracle.so``); this module is its ctypes wrapper plus two pure-Python
helpers for tiny inputs (exhaustive partition search and the bound formulas
written with explicit angles).

Variants follow the numbering LLOYD=0, ELKAN=1, HAMERLY=2, SIMP_ELKAN=3,
SIMP_HAMERLY=4, YINYANG=5 (Sections 5, 5.2, 5.3, 5.1, 5.4 and 5.5 of the
paper; Yin-Yang with groups of 32 consecutive centres).
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "skm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

LLOYD, ELKAN, HAMERLY, SIMP_ELKAN, SIMP_HAMERLY, YINYANG = 0, 1, 2, 3, 4, 5
VARIANTS = {"lloyd": LLOYD, "elkan": ELKAN, "hamerly": HAMERLY,
            "simp_elkan": SIMP_ELKAN, "simp_hamerly": SIMP_HAMERLY, "yinyang": YINYANG}


def build(force: bool = True) -> str:
    """Compile skm_oracle.c with gcc (-O2, OpenMP, no FMA contraction so the
    sums are plain sequential double additions)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, i32, dbl, p = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
        lib.oracle_assign.restype = None
        lib.oracle_assign.argtypes = [i64, i64, p, p, p, i32, p, p, p, p, p]
        lib.oracle_assign_ct.restype = None
        lib.oracle_assign_ct.argtypes = [i64, i64, p, p, p, i32, p, p, p, p, p]
        lib.oracle_init_centres.restype = None
        lib.oracle_init_centres.argtypes = [i32, i64, p]
        lib.oracle_sims.restype = None
        lib.oracle_sims.argtypes = [i64, i64, p, p, p, i32, p, p, i64, p]
        lib.oracle_update.restype = dbl
        lib.oracle_update.argtypes = [i64, i64, p, p, p, i32, p, p, p, p]
        for name in ("oracle_lower_update", "oracle_upper_update", "oracle_upper_eq9"):
            getattr(lib, name).restype = dbl
            getattr(lib, name).argtypes = [dbl, dbl, dbl]
        for name in ("oracle_lower_unguarded", "oracle_upper_unguarded"):
            getattr(lib, name).restype = dbl
            getattr(lib, name).argtypes = [dbl, dbl]
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_threads.argtypes = []
        lib.oracle_cc.restype = dbl
        lib.oracle_cc.argtypes = [dbl]
        lib.oracle_fit.restype = i32
        lib.oracle_fit.argtypes = [i64, i64, p, p, p, i32, p, i32, i32, i32, i32, p, p,
                                   p, p, p, p, p, p, p, p]
        lib.oracle_afkmc2.restype = None
        lib.oracle_afkmc2.argtypes = [i64, i64, p, p, p, i32, i32, dbl, p, p]
        lib.oracle_kmeanspp.restype = None
        lib.oracle_kmeanspp.argtypes = [i64, i64, p, p, p, i32, dbl, p, p, p, p, p]
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _csr_args(X):
    rp = np.ascontiguousarray(X.row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(X.col, dtype=np.int32)
    v = np.ascontiguousarray(X.val, dtype=np.float32)
    return rp, ci, v


def assign(X, C: np.ndarray, a_prev: Optional[np.ndarray] = None,
           transposed: bool = False):
    """Exhaustive assignment step: (a, best, second) with the tie rule
    'keep the previous centre if it attains the maximum, else the lowest
    index'.  C is k x d (float64; float32 is promoted exactly).
    ``transposed`` reads the centres from a d x k copy (same sums in the same
    order, identical results; faster for large k and d)."""
    lib = _load()
    rp, ci, v = _csr_args(X)
    C = np.ascontiguousarray(C, dtype=np.float64)
    k = C.shape[0]
    a = np.empty(X.n, dtype=np.int32)
    s1 = np.empty(X.n)
    s2 = np.empty(X.n)
    ap = None if a_prev is None else np.ascontiguousarray(a_prev, dtype=np.int32)
    if transposed:
        CT = np.ascontiguousarray(C.T)
        lib.oracle_assign_ct(X.n, X.d, _p(rp), _p(ci), _p(v), k, _p(CT), _p(ap), _p(a),
                             _p(s1), _p(s2))
    else:
        lib.oracle_assign(X.n, X.d, _p(rp), _p(ci), _p(v), k, _p(C), _p(ap), _p(a), _p(s1),
                          _p(s2))
    return a, s1, s2


def lloyd_trajectory(X, C_init: np.ndarray, max_iter: int, on_step=None):
    """Plain spherical Lloyd (Section 5) step by step, as oracle ``fit`` runs
    it (INIT, ARGMAX, STOP and EMPTY readings), with the centres read from a
    transposed copy.  After assignment step t (1-based) ``on_step(t, a, C,
    best, second, changed, objective)`` sees the step's assignment, its top-2
    similarities (against the centres before the step), the centres after the
    update that follows it (unchanged when nothing changed) and sum_j |S(j)|
    of those centres (None when nothing changed).  Returns (a, C, iterations,
    converged)."""
    lib = _load()
    C = np.array(C_init, dtype=np.float64, order="C", copy=True)
    k = C.shape[0]
    lib.oracle_init_centres(k, X.d, _p(C))
    a = None
    it, conv = 0, False
    for t in range(1, max_iter + 1):
        a_new, s1, s2 = assign(X, C, a, transposed=True)
        changed = X.n if a is None else int(np.count_nonzero(a_new != a))
        a = a_new
        it = t
        obj = None
        if changed == 0:
            conv = True
        else:
            C, _, obj = update(X, a, C)
        if on_step is not None:
            on_step(t, a, C, s1, s2, changed, obj)
        if conv:
            break
    return a, C, it, conv


def kmeanspp(X, k: int, alpha: float, u: np.ndarray):
    """Spherical k-means++ seeding with the given uniforms u[0..k) in [0, 1):
    (chosen rows, assign, best, second), the last three being the assignment
    step against the chosen rows rescaled to unit length."""
    lib = _load()
    rp, ci, v = _csr_args(X)
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert u.shape == (k,)
    chosen = np.empty(k, dtype=np.int32)
    a = np.empty(X.n, dtype=np.int32)
    s1 = np.empty(X.n)
    s2 = np.empty(X.n)
    lib.oracle_kmeanspp(X.n, X.d, _p(rp), _p(ci), _p(v), k, float(alpha), _p(u), _p(chosen),
                        _p(a), _p(s1), _p(s2))
    return chosen, a, s1, s2


def afkmc2(X, k: int, m: int, alpha: float, u: np.ndarray) -> np.ndarray:
    """AFK-MC2 seeding (spherical form) with chain length m and the given
    uniforms: u[0], then per centre t >= 1 the m proposal draws and the
    m - 1 acceptance draws (1 + (k - 1)(2m - 1) values in [0, 1)).
    Returns the chosen row indices."""
    lib = _load()
    rp, ci, v = _csr_args(X)
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert u.shape == (1 + (k - 1) * (2 * m - 1),)
    chosen = np.empty(k, dtype=np.int32)
    lib.oracle_afkmc2(X.n, X.d, _p(rp), _p(ci), _p(v), k, m, float(alpha), _p(u), _p(chosen))
    return chosen


def sims(X, C: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """All similarities of the listed rows to the k centres (len(rows) x k)."""
    lib = _load()
    rp, ci, v = _csr_args(X)
    C = np.ascontiguousarray(C, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((len(rows), C.shape[0]))
    lib.oracle_sims(X.n, X.d, _p(rp), _p(ci), _p(v), C.shape[0], _p(C), _p(rows), len(rows),
                    _p(out))
    return out


def update(X, a: np.ndarray, C_prev: np.ndarray):
    """Centre step: (C, norms, objective) with c(j) = S(j)/|S(j)|; empty
    clusters keep C_prev(j); objective = sum_j |S(j)|."""
    lib = _load()
    rp, ci, v = _csr_args(X)
    C_prev = np.ascontiguousarray(C_prev, dtype=np.float64)
    k = C_prev.shape[0]
    a = np.ascontiguousarray(a, dtype=np.int32)
    C = np.empty_like(C_prev)
    norms = np.empty(k)
    obj = lib.oracle_update(X.n, X.d, _p(rp), _p(ci), _p(v), k, _p(a), _p(C_prev), _p(C),
                            _p(norms))
    return C, norms, obj


def lower_update(l, p, omp=None):
    """Guarded Eq. (6); omp = 1 - p (computed from p if not given)."""
    return _load().oracle_lower_update(l, p, (1.0 - p) if omp is None else omp)


def upper_update(u, p, omp=None):
    """Guarded Eq. (7); omp = 1 - p (computed from p if not given)."""
    return _load().oracle_upper_update(u, p, (1.0 - p) if omp is None else omp)


def upper_eq9(u, p, omp=None):
    """Eq. (9) where valid (u, p >= 0), guarded Eq. (7) elsewhere."""
    return _load().oracle_upper_eq9(u, p, (1.0 - p) if omp is None else omp)


def lower_unguarded(l, p):
    return _load().oracle_lower_unguarded(l, p)


def upper_unguarded(u, p):
    return _load().oracle_upper_unguarded(u, p)


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().oracle_threads())


def cc(g):
    """Half-angle centre-centre bound sqrt((g+1)/2) of Section 5.2."""
    return _load().oracle_cc(g)


@dataclass
class FitResult:
    a: np.ndarray
    C: np.ndarray
    iterations: int
    converged: bool
    changed: np.ndarray
    sims: np.ndarray
    ccsims: np.ndarray
    obj_assign: np.ndarray
    obj_update: np.ndarray
    a_trace: Optional[np.ndarray]
    violations: int


def fit(X, C_init: np.ndarray, variant="lloyd", max_iter: int = 100, bound_form: int = 0,
        check_bounds: bool = False, trace: bool = False) -> FitResult:
    """Full run of the chosen variant from C_init (k x d).  ``trace`` keeps the
    n x max_iter assignment history; ``check_bounds`` counts bound violations
    against exhaustively computed similarities."""
    lib = _load()
    v_id = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    rp, ci, v = _csr_args(X)
    C0 = np.ascontiguousarray(C_init, dtype=np.float64)
    k = C0.shape[0]
    a = np.empty(X.n, dtype=np.int32)
    C = np.empty_like(C0)
    ch = np.zeros(max_iter, dtype=np.int64)
    sm = np.zeros(max_iter, dtype=np.int64)
    cs = np.zeros(max_iter, dtype=np.int64)
    oa = np.full(max_iter, np.nan)
    ou = np.full(max_iter, np.nan)
    at = np.empty((X.n, max_iter), dtype=np.int32) if trace else None
    viol = ctypes.c_int64(0)
    conv = ctypes.c_int32(0)
    it = lib.oracle_fit(X.n, X.d, _p(rp), _p(ci), _p(v), k, _p(C0), v_id, max_iter, bound_form,
                        1 if check_bounds else 0, _p(a), _p(C), _p(ch), _p(sm), _p(cs), _p(oa),
                        _p(ou), _p(at), ctypes.byref(viol), ctypes.byref(conv))
    return FitResult(a, C, it, bool(conv.value), ch[:it], sm[:it], cs[:it], oa[:it], ou[:it],
                     None if at is None else at[:, :it], viol.value)


# --------------------------------------------------------------------------
# pure-Python helpers for tiny inputs
# --------------------------------------------------------------------------

def brute_force_best_partition(Xd: np.ndarray, k: int):
    """Exhaustive search over all k^n labelings of the rows of the small dense
    matrix Xd (n x d): returns (best objective, best labels) where the
    objective of a labeling is sum_j |sum_{a(i)=j} x(i)|, the quantity the
    spherical centre step maximises (Section 5; Cauchy-Schwarz makes
    sum_i <x(i), S_a/|S_a|> = sum_j |S_j|).  Only for n <= 10."""
    n = Xd.shape[0]
    best, best_lab = -1.0, None
    for lab in itertools.product(range(k), repeat=n):
        S = np.zeros((k, Xd.shape[1]))
        for i, j in enumerate(lab):
            S[j] += Xd[i]
        obj = float(np.sqrt((S * S).sum(axis=1)).sum())
        if obj > best + 1e-15:
            best, best_lab = obj, np.array(lab)
    return best, best_lab


def angle_lower(l: float, p: float) -> float:
    """cos(min(pi, acos l + acos p)): the exact worst case the lower bound
    has to cover after a centre moved by angle acos p (triangle inequality
    on arc length, Eq. (3))."""
    return math.cos(min(math.pi, math.acos(l) + math.acos(p)))


def angle_upper(u: float, p: float) -> float:
    """cos(max(0, acos u - acos p)): the exact worst case the upper bound has
    to cover (Eq. (3) applied the other way round)."""
    return math.cos(max(0.0, math.acos(u) - math.acos(p)))
