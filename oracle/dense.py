"""FP64 oracle of plain spherical Lloyd for dense row matrices.

TEST INFRASTRUCTURE ONLY (as the rest of ``oracle/``): used to write the
stored trajectory of the full-size dense embedding workload and by the tests
that pin it.  The GPU library never uses it.

The definition is the same as the CSR oracle's Lloyd (Section 5 of the
paper: assignment a(i) = argmax_j <x(i), c(j)>, centre c(j) = S(j)/|S(j)|
with S(j) the member sum; readings ARGMAX, STOP, EMPTY and INIT of
``skm_oracle.c``).  The one library primitive is numpy's FP64 matrix
product for the similarities, which sums in its own order: values differ
from the sequential sums of the CSR oracle by a few units of 1e-16, which
only matters for rows whose top-2 gap is that small (pinned against the CSR
oracle in the tests).
"""
from __future__ import annotations

import numpy as np


def _blocks(n, size=65536):
    for b in range(0, n, size):
        yield b, min(n, b + size)


def assign(X: np.ndarray, C: np.ndarray, a_prev=None):
    """Exhaustive assignment step over the rows of X (n x d, promoted to
    FP64): (a, best, second) with the tie rule "keep the previous centre if
    it attains the maximum, else the lowest index"."""
    n, k = X.shape[0], C.shape[0]
    CT = np.ascontiguousarray(np.asarray(C, np.float64).T)
    a = np.empty(n, np.int32)
    s1 = np.empty(n)
    s2 = np.empty(n)
    for b, e in _blocks(n):
        S = np.asarray(X[b:e], np.float64) @ CT
        mx = S.max(axis=1)
        at_max = S == mx[:, None]
        pick = np.argmax(at_max, axis=1)  # lowest index among the maxima
        if a_prev is not None:
            prev = np.asarray(a_prev[b:e], np.int64)
            keep = (prev >= 0) & at_max[np.arange(e - b), np.maximum(prev, 0)]
            pick = np.where(keep, prev, pick)
        a[b:e] = pick
        s1[b:e] = mx
        if k > 1:
            S[np.arange(e - b), pick] = -np.inf
            s2[b:e] = S.max(axis=1)
        else:
            s2[b:e] = -np.inf
    return a, s1, s2


def update(X: np.ndarray, a: np.ndarray, C_prev: np.ndarray):
    """Centre step: (C, norms, objective) with c(j) = S(j)/|S(j)| (FP64 member
    sums); a cluster without members keeps C_prev(j); objective = sum_j |S(j)|."""
    k, d = C_prev.shape
    S = np.zeros((k, d))
    for b, e in _blocks(X.shape[0]):
        np.add.at(S, a[b:e], np.asarray(X[b:e], np.float64))
    norms = np.sqrt((S * S).sum(axis=1))
    C = np.array(C_prev, np.float64, copy=True)
    nz = norms > 0
    C[nz] = S[nz] / norms[nz, None]
    return C, norms, float(norms.sum())


def init_centres(C0: np.ndarray) -> np.ndarray:
    """INIT reading: the initial rows rescaled to unit length in FP64."""
    C = np.array(C0, np.float64, copy=True)
    nrm = np.sqrt((C * C).sum(axis=1))
    nz = nrm > 0
    C[nz] /= nrm[nz, None]
    return C


def lloyd_trajectory(X: np.ndarray, C0: np.ndarray, max_iter: int, on_step=None):
    """Plain spherical Lloyd from C0; ``on_step(t, a, C, best, second, changed,
    objective)`` after assignment step t as in the CSR oracle's
    ``lloyd_trajectory``.  Returns (a, C, iterations, converged)."""
    C = init_centres(C0)
    a = None
    it, conv = 0, False
    for t in range(1, max_iter + 1):
        a_new, s1, s2 = assign(X, C, a)
        changed = X.shape[0] if a is None else int(np.count_nonzero(a_new != a))
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
