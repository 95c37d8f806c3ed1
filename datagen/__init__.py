"""Seeded synthetic workloads for spherical k-means.

This package produces inputs only: CSR tf-idf document vectors, dense
von Mises-Fisher mixtures, instance lists for batched runs and the seeded
choice of initial centres.  It performs none of the clustering arithmetic, so
the CPU oracle and the GPU library can both consume it without sharing any
of the method's code.

The heavy lifting is in ``gen.c`` (compiled to ``libskmgen.so`` with gcc and
OpenMP); this module wraps it with ctypes and numpy.

Workload presets follow the five measured configurations of the project:

* ``c1`` Simpsons-wiki-sized corpus, n=2,000, d=5,000, ~50 nnz/row, k=10.
* ``c2`` n=100,000, d=50,000, ~100 nnz/row, k=100 (Elkan/Hamerly vs Lloyd).
* ``c3`` n=1,000,000, d=100,000, ~150 nnz/row, k=1,000 (large Hamerly).
* ``c4`` dense vMF embeddings, n=2,000,000, d=256, 4,096 means, k=4,096.
* ``c5`` 256 independent sparse instances, d=20,000, ~80 nnz/row.

The paper's corpora (DBLP, Simpsons wiki, 20 Newsgroups, RCV-1; its Table 1)
are not available; these generators stand in for them with the same kind of
structure: Zipf term popularity, log-normal document lengths, tf-idf
weighting and unit-length rows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libskmgen.so")

BASE_SEED = 210704074


def build(force: bool = True) -> str:
    """Compile gen.c into libskmgen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, i32, u64, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
        p = ctypes.c_void_p
        lib.skmgen_row_lengths.restype = i64
        lib.skmgen_row_lengths.argtypes = [i64, i64, dbl, dbl, u64, p]
        lib.skmgen_sparse_fill.restype = i64
        lib.skmgen_sparse_fill.argtypes = [i64, i64, dbl, u64, p, p, p, p, p, p, p]
        lib.skmgen_sparse_fill_topics.restype = i64
        lib.skmgen_sparse_fill_topics.argtypes = [i64, i64, dbl, u64, i32, dbl, p, p, p, p,
                                                  p, p, p]
        lib.skmgen_vmf.restype = None
        lib.skmgen_vmf.argtypes = [i64, i64, i32, dbl, dbl, u64, p, p, p, p]
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class CSR:
    """Row-normalised sparse matrix; columns ascending within every row."""
    n: int
    d: int
    row_ptr: np.ndarray  # int64 [n+1]
    col: np.ndarray      # int32 [nnz]
    val: np.ndarray      # float32 [nnz]
    dropped_rows: int = 0

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def take_rows(self, rows: np.ndarray) -> "CSR":
        rows = np.asarray(rows, dtype=np.int64)
        lens = self.row_ptr[rows + 1] - self.row_ptr[rows]
        rp = np.zeros(len(rows) + 1, dtype=np.int64)
        np.cumsum(lens, out=rp[1:])
        idx = np.concatenate([np.arange(self.row_ptr[r], self.row_ptr[r + 1]) for r in rows]) \
            if len(rows) else np.zeros(0, dtype=np.int64)
        return CSR(len(rows), self.d, rp, self.col[idx].copy(), self.val[idx].copy())

    def to_dense(self) -> np.ndarray:
        out = np.zeros((self.n, self.d), dtype=np.float32)
        rows = np.repeat(np.arange(self.n), self.row_lengths())
        out[rows, self.col] = self.val
        return out


def sparse_tfidf(n: int, d: int, mean_nnz: float, seed: int,
                 sigma: float = 0.5, zipf_s: float = 1.1, topics: int = 0,
                 topic_share: float = 0.7) -> CSR:
    """SPARSE(n, d, mean_nnz, seed): log-normal row lengths (arithmetic mean
    ``mean_nnz``, sigma 0.5), distinct Zipf(1.1) terms, Geometric(1/2) term
    frequencies, ln(1+tf)*ln(n/df) weights, unit rows stored as float32.
    ``topics`` > 0: every row belongs to one of that many topics and takes
    each term, with probability ``topic_share``, through its topic's own
    rank -> column permutation (rows of a topic share their frequent terms);
    0 gives the plain rows above."""
    lib = _load()
    m = np.empty(n, dtype=np.int32)
    cap = lib.skmgen_row_lengths(n, d, float(mean_nnz), float(sigma), seed, _ptr(m))
    rp = np.empty(n + 1, dtype=np.int64)
    col = np.empty(max(cap, 1), dtype=np.int32)
    val = np.empty(max(cap, 1), dtype=np.float32)
    n_out = ctypes.c_int64(0)
    dropped = ctypes.c_int64(0)
    if topics > 0:
        nnz = lib.skmgen_sparse_fill_topics(n, d, float(zipf_s), seed, int(topics),
                                            float(topic_share), _ptr(m), _ptr(rp), _ptr(col),
                                            _ptr(val), ctypes.byref(n_out),
                                            ctypes.byref(dropped), None)
    else:
        nnz = lib.skmgen_sparse_fill(n, d, float(zipf_s), seed, _ptr(m), _ptr(rp),
                                     _ptr(col), _ptr(val), ctypes.byref(n_out),
                                     ctypes.byref(dropped), None)
    rows = n_out.value
    return CSR(rows, d, rp[: rows + 1].copy(), col[:nnz].copy(), val[:nnz].copy(),
               dropped.value)


def dense_vmf(n: int, d: int, n_means: int, seed: int, kappa_lo: float = 50.0,
              kappa_hi: float = 500.0, return_components: bool = False):
    """n unit vectors in R^d from an equal-weight mixture of ``n_means``
    von Mises-Fisher components with kappa ~ U[kappa_lo, kappa_hi]."""
    lib = _load()
    X = np.empty((n, d), dtype=np.float32)
    comp = np.empty(n, dtype=np.int32) if return_components else None
    lib.skmgen_vmf(n, d, n_means, float(kappa_lo), float(kappa_hi), seed, _ptr(X), None,
                   None, _ptr(comp))
    return (X, comp) if return_components else X


def init_rows(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct row indices drawn uniformly without replacement (seeded);
    centre j starts at row init_rows[j]."""
    rng = np.random.Generator(np.random.Philox(key=seed + 7))
    return rng.choice(n, size=k, replace=False).astype(np.int64)


def init_centers_csr(X: CSR, rows: np.ndarray) -> np.ndarray:
    """The chosen rows as a dense float32 k x d matrix (values copied
    exactly)."""
    C = np.zeros((len(rows), X.d), dtype=np.float32)
    for j, r in enumerate(rows):
        a, b = X.row_ptr[r], X.row_ptr[r + 1]
        C[j, X.col[a:b]] = X.val[a:b]
    return C


# --------------------------------------------------------------------------
# workload presets
# --------------------------------------------------------------------------

@dataclass
class SparseConfig:
    name: str
    n: int
    d: int
    mean_nnz: float
    k: int
    max_iter: int
    seed: int


CONFIGS = {
    "c1": SparseConfig("c1", 2_000, 5_000, 50.0, 10, 20, BASE_SEED + 1),
    "c2": SparseConfig("c2", 100_000, 50_000, 100.0, 100, 1000, BASE_SEED + 2),
    "c3": SparseConfig("c3", 1_000_000, 100_000, 150.0, 1000, 50, BASE_SEED + 3),
}

C4 = dict(name="c4", n=2_000_000, d=256, n_means=4096, k=4096, seed=BASE_SEED + 4,
          kappa_lo=50.0, kappa_hi=500.0, subsample=20_000)

C5 = dict(name="c5", n_inst=256, d=20_000, mean_nnz=80.0, n_lo=1_000, n_hi=50_000,
          max_iter=30, seed=BASE_SEED + 5)


def sparse_workload(name: str, n: Optional[int] = None):
    """(CSR, init rows, config) for preset c1/c2/c3; ``n`` overrides the row
    count (same generator and seed) for reduced-size variants."""
    cfg = CONFIGS[name]
    rows = cfg.n if n is None else n
    X = sparse_tfidf(rows, cfg.d, cfg.mean_nnz, cfg.seed)
    init = init_rows(X.n, cfg.k, cfg.seed)
    return X, init, cfg


@dataclass
class Instance:
    X: CSR
    k: int
    init: np.ndarray
    max_iter: int


def batched_instances(n_inst: Optional[int] = None, scale: float = 1.0) -> List[Instance]:
    """The c5 instance list: n_b = clip(round(LogNormal(ln sqrt(1e3*5e4),
    ln(50)/4)), 1e3, 5e4) rows each, k_b = 8*U{1..32}, d = 20,000, ~80 nnz per
    row, every instance from its own seed.  ``scale`` shrinks every n_b (for
    quick tests); k_b is capped at n_b."""
    cfg = C5
    count = cfg["n_inst"] if n_inst is None else n_inst
    rng = np.random.Generator(np.random.Philox(key=cfg["seed"]))
    mu = np.log(np.sqrt(cfg["n_lo"] * cfg["n_hi"]))
    sig = np.log(cfg["n_hi"] / cfg["n_lo"]) / 4.0
    ns = np.clip(np.rint(rng.lognormal(mu, sig, size=cfg["n_inst"])), cfg["n_lo"], cfg["n_hi"])
    ks = 8 * rng.integers(1, 33, size=cfg["n_inst"])
    out = []
    for b in range(count):
        nb = max(int(ns[b] * scale), 16)
        sb = cfg["seed"] * 1000 + b
        X = sparse_tfidf(nb, cfg["d"], cfg["mean_nnz"], sb)
        kb = int(min(ks[b], X.n))
        out.append(Instance(X, kb, init_rows(X.n, kb, sb), cfg["max_iter"]))
    return out
