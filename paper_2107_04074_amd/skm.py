"""ctypes binding of libskm (include/skm.h).

Argument marshalling only: every step of the clustering runs in the HIP
library.  Device memory comes from torch tensors on a ROCm device and work is
enqueued on torch's current stream.  There is no fallback: without the built
library every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libskm.so")

LLOYD, ELKAN, HAMERLY, SIMP_ELKAN, SIMP_HAMERLY, YINYANG = range(6)
VARIANTS = {"lloyd": LLOYD, "elkan": ELKAN, "hamerly": HAMERLY,
            "simp_elkan": SIMP_ELKAN, "simp_hamerly": SIMP_HAMERLY, "yinyang": YINYANG}
CSR_F32, DENSE_F32 = 0, 1
OK, ERR_INVALID_ARG, ERR_NOT_NORMALIZED, ERR_OUT_OF_MEMORY, ERR_HIP, ERR_UNSUPPORTED = range(6)

# Every symbol include/skm.h declares.
EXPORTS = ("skm_workspace_size", "skm_assign_workspace_size", "skm_fit", "skm_assign",
           "skm_assign_noalloc",
           "skm_seed_workspace_size", "skm_seed_kmeanspp",
           "skm_seed_afkmc2_workspace_size", "skm_seed_afkmc2",
           "skm_fit_batched_workspace_size", "skm_fit_batched",
           "skm_status_string", "skm_last_error", "skm_version")


class SkmMatrix(ctypes.Structure):
    _fields_ = [("fmt", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("n", ctypes.c_int64), ("d", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("dense", ctypes.c_void_p), ("ld", ctypes.c_int64)]


class SkmOptions(ctypes.Structure):
    _fields_ = [("bound_form", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("norm_tol", ctypes.c_double), ("warm_assign", ctypes.c_void_p),
                ("warm_best", ctypes.c_void_p), ("warm_second", ctypes.c_void_p),
                ("schedule", ctypes.c_int32), ("batch_tile_rows", ctypes.c_int32),
                ("walk_layout", ctypes.c_int32), ("chunk_walk", ctypes.c_int32)]


class SkmStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("objective", ctypes.c_double), ("sims_point_center", ctypes.c_int64),
                ("sims_center_center", ctypes.c_int64), ("rechecks", ctypes.c_int64),
                ("changed_per_iter", ctypes.c_void_p), ("sims_per_iter", ctypes.c_void_p),
                ("objective_per_iter", ctypes.c_void_p), ("per_iter_len", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("sim_kernel_launches", ctypes.c_int64),
                ("sim_kernel_rows", ctypes.c_int64), ("sim_kernel_nnz", ctypes.c_int64),
                ("sim_kernel_ms", ctypes.c_double)]


class SkmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("skm status %d: %s" % (status, msg))
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Loads libskm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libskm.so not built (expected at %s); run "
                           "`python -m paper_2107_04074_amd.build`" % path)
    lib = ctypes.CDLL(path)
    p, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    lib.skm_workspace_size.restype = sz
    lib.skm_workspace_size.argtypes = [ctypes.POINTER(SkmMatrix), i32, i32,
                                       ctypes.POINTER(SkmOptions)]
    lib.skm_assign_workspace_size.restype = sz
    lib.skm_assign_workspace_size.argtypes = [ctypes.POINTER(SkmMatrix), i32]
    lib.skm_fit.restype = ctypes.c_int
    lib.skm_fit.argtypes = [ctypes.POINTER(SkmMatrix), i32, p, i32, i32,
                            ctypes.POINTER(SkmOptions), p, sz, p, p, p,
                            ctypes.POINTER(SkmStats), p]
    lib.skm_assign.restype = ctypes.c_int
    lib.skm_assign.argtypes = [ctypes.POINTER(SkmMatrix), i32, p, p, p, p, p, sz, p]
    lib.skm_assign_noalloc.restype = ctypes.c_int
    lib.skm_assign_noalloc.argtypes = [ctypes.POINTER(SkmMatrix), i32, p, p, p, p, p]
    lib.skm_fit_batched_workspace_size.restype = sz
    lib.skm_fit_batched_workspace_size.argtypes = [i32, ctypes.POINTER(SkmMatrix), p, i32,
                                                   ctypes.POINTER(SkmOptions), i32]
    lib.skm_fit_batched.restype = ctypes.c_int
    lib.skm_fit_batched.argtypes = [i32, ctypes.POINTER(SkmMatrix), p, p, i32, p,
                                    ctypes.POINTER(SkmOptions), i32, p, sz, p, p,
                                    ctypes.POINTER(SkmStats), p]
    lib.skm_seed_workspace_size.restype = sz
    lib.skm_seed_workspace_size.argtypes = [ctypes.POINTER(SkmMatrix), i32]
    lib.skm_seed_kmeanspp.restype = ctypes.c_int
    lib.skm_seed_kmeanspp.argtypes = [ctypes.POINTER(SkmMatrix), i32, ctypes.c_double, p, p, p,
                                      p, p, p, p, sz, p]
    lib.skm_seed_afkmc2_workspace_size.restype = sz
    lib.skm_seed_afkmc2_workspace_size.argtypes = [ctypes.POINTER(SkmMatrix), i32, i32]
    lib.skm_seed_afkmc2.restype = ctypes.c_int
    lib.skm_seed_afkmc2.argtypes = [ctypes.POINTER(SkmMatrix), i32, i32, ctypes.c_double, p, p,
                                    p, p, sz, p]
    lib.skm_status_string.restype = ctypes.c_char_p
    lib.skm_status_string.argtypes = [ctypes.c_int]
    lib.skm_last_error.restype = ctypes.c_char_p
    lib.skm_last_error.argtypes = []
    lib.skm_version.restype = ctypes.c_int
    lib.skm_version.argtypes = []
    _ = i64
    _lib = lib
    return lib


def _check(status: int):
    if status != OK:
        raise SkmError(status, load().skm_last_error().decode(errors="replace"))


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


@dataclass
class DeviceCSR:
    """CSR matrix resident on the GPU (torch tensors)."""
    n: int
    d: int
    row_ptr: "object"  # torch.int64 [n+1]
    col: "object"      # torch.int32 [nnz]
    val: "object"      # torch.float32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @staticmethod
    def from_host(X, device="cuda") -> "DeviceCSR":
        """From any object with n, d, row_ptr, col, val (numpy)."""
        import torch
        return DeviceCSR(int(X.n), int(X.d),
                         torch.from_numpy(np.ascontiguousarray(X.row_ptr, np.int64)).to(device),
                         torch.from_numpy(np.ascontiguousarray(X.col, np.int32)).to(device),
                         torch.from_numpy(np.ascontiguousarray(X.val, np.float32)).to(device))

    def matrix(self) -> SkmMatrix:
        return SkmMatrix(CSR_F32, 0, self.n, self.d, self.nnz, _ptr(self.row_ptr),
                         _ptr(self.col), _ptr(self.val), None, 0)


@dataclass
class DeviceDense:
    """Dense row-major float32 matrix resident on the GPU (n x ld, first d
    columns used)."""
    X: "object"  # torch.float32 [n, ld]
    d: int = 0

    def __post_init__(self):
        if not self.d:
            self.d = int(self.X.shape[1])

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def col(self):  # device of the matrix (shared with DeviceCSR)
        return self.X

    @staticmethod
    def from_host(Xh: np.ndarray, device="cuda") -> "DeviceDense":
        import torch
        return DeviceDense(torch.from_numpy(np.ascontiguousarray(Xh, np.float32)).to(device))

    def matrix(self) -> SkmMatrix:
        return SkmMatrix(DENSE_F32, 0, self.n, self.d, 0, None, None, None, _ptr(self.X),
                         int(self.X.stride(0)))


@dataclass
class FitStats:
    iterations: int
    converged: bool
    objective: float
    sims_point_center: int
    sims_center_center: int
    rechecks: int
    sim_kernel_launches: int = 0
    sim_kernel_rows: int = 0
    sim_kernel_nnz: int = 0
    sim_kernel_ms: float = 0.0
    changed_per_iter: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    sims_per_iter: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    objective_per_iter: np.ndarray = field(default_factory=lambda: np.zeros(0))


def _options(bound_form=0, precision=0, validate=0, norm_tol=0.0, profile=0, warm=None,
             schedule=0, batch_tile_rows=0, walk_layout=0, chunk_walk=0):
    """warm: (assign, best, second) device tensors from seed_kmeanspp;
    schedule: 1 runs the bound tests at every step (0 = adaptive);
    batch_tile_rows: rows per work item of the lockstep batched walk (0 =
    the library's table; that driver is switched off);
    walk_layout: row-walk layout of FP32 Lloyd/Hamerly whole-row walks at
    16 < k <= 512 (0 = the library's tuning table, 1 = default, 2 = alternative);
    chunk_walk: FP32 CSR fits at 256 < k: 0 = the tuning table (sliced above
    a 256 MB copy; Yin-Yang at 128 < k and Elkan at 256 < k on whole rows
    time both walks of their steps with tests and keep the faster), 1 =
    256-centre slices (Elkan and
    Yin-Yang at 128 < k <= 256: one packed slice), 2 = whole rows."""
    w = (None, None, None) if warm is None else tuple(_ptr(t) for t in warm)
    return SkmOptions(bound_form, precision, validate, profile, norm_tol, *w, schedule,
                      batch_tile_rows, walk_layout, chunk_walk)


def seed_kmeanspp(X: "DeviceCSR | DeviceDense", k: int, uniforms, alpha: float = 1.0,
                  workspace=None):
    """Runs skm_seed_kmeanspp (CSR or dense rows) with the caller's uniforms
    (k floats in [0, 1)).  Returns (chosen int32, centers float32 (k, d), assign int32,
    best float64, second float64) device tensors; asynchronous."""
    import torch
    lib = load()
    dev = X.col.device
    m = X.matrix()
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    if u.shape != (k,):
        raise ValueError("need k uniforms")
    if workspace is None:
        size = lib.skm_seed_workspace_size(ctypes.byref(m), k)
        if size == 0:
            raise SkmError(ERR_INVALID_ARG, lib.skm_last_error().decode(errors="replace"))
        workspace = torch.empty(size, dtype=torch.uint8, device=dev)
    chosen = torch.empty(k, dtype=torch.int32, device=dev)
    centers = torch.empty((k, X.d), dtype=torch.float32, device=dev)
    a = torch.empty(X.n, dtype=torch.int32, device=dev)
    best = torch.empty(X.n, dtype=torch.float64, device=dev)
    second = torch.empty(X.n, dtype=torch.float64, device=dev)
    _check(lib.skm_seed_kmeanspp(ctypes.byref(m), k, float(alpha), u.ctypes.data, _ptr(chosen),
                                 _ptr(centers), _ptr(a), _ptr(best), _ptr(second),
                                 _ptr(workspace), workspace.numel(), _stream()))
    return chosen, centers, a, best, second


def seed_afkmc2(X: "DeviceCSR | DeviceDense", k: int, chain: int, uniforms,
                alpha: float = 1.0, workspace=None):
    """Runs skm_seed_afkmc2 (CSR or dense rows) with the caller's draws (1 + (k-1)(2 chain - 1)
    floats in [0, 1)).  Returns (chosen int32, centers float32 (k, d));
    asynchronous."""
    import torch
    lib = load()
    dev = X.col.device
    m = X.matrix()
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    if u.shape != (1 + (k - 1) * (2 * chain - 1),):
        raise ValueError("need 1 + (k - 1)(2 chain - 1) uniforms")
    if workspace is None:
        size = lib.skm_seed_afkmc2_workspace_size(ctypes.byref(m), k, chain)
        if size == 0:
            raise SkmError(ERR_INVALID_ARG, lib.skm_last_error().decode(errors="replace"))
        workspace = torch.empty(size, dtype=torch.uint8, device=dev)
    chosen = torch.empty(k, dtype=torch.int32, device=dev)
    centers = torch.empty((k, X.d), dtype=torch.float32, device=dev)
    _check(lib.skm_seed_afkmc2(ctypes.byref(m), k, chain, float(alpha), u.ctypes.data,
                               _ptr(chosen), _ptr(centers), _ptr(workspace), workspace.numel(),
                               _stream()))
    return chosen, centers


def workspace_size(X: DeviceCSR, k: int, variant="hamerly", **opts) -> int:
    lib = load()
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    m = X.matrix()
    o = _options(**opts)
    size = lib.skm_workspace_size(ctypes.byref(m), k, v, ctypes.byref(o))
    if size == 0:
        raise SkmError(ERR_INVALID_ARG, lib.skm_last_error().decode(errors="replace"))
    return int(size)


def fit(X: DeviceCSR, k: int, init_centers, variant="hamerly", max_iter: int = 100,
        workspace=None, want_centers=True, want_centers64=False, per_iter=True, **opts):
    """Runs skm_fit.  init_centers: float32 (k, d) device tensor.
    Returns (assign int32 tensor, centers float32 or None, centers64 or None,
    FitStats)."""
    import torch
    lib = load()
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    dev = X.col.device
    m = X.matrix()
    o = _options(**opts)
    if workspace is None:
        size = lib.skm_workspace_size(ctypes.byref(m), k, v, ctypes.byref(o))
        if size == 0:
            raise SkmError(ERR_INVALID_ARG, lib.skm_last_error().decode(errors="replace"))
        workspace = torch.empty(size, dtype=torch.uint8, device=dev)
    assign = torch.empty(X.n, dtype=torch.int32, device=dev)
    centers = torch.empty((k, X.d), dtype=torch.float32, device=dev) if want_centers else None
    centers64 = torch.empty((k, X.d), dtype=torch.float64, device=dev) if want_centers64 else None
    init = init_centers.contiguous()
    st = SkmStats()
    ch = sm = ob = None
    if per_iter:
        ch = np.zeros(max_iter, np.int64)
        sm = np.zeros(max_iter, np.int64)
        ob = np.zeros(max_iter, np.float64)
        st.changed_per_iter = ch.ctypes.data
        st.sims_per_iter = sm.ctypes.data
        st.objective_per_iter = ob.ctypes.data
        st.per_iter_len = max_iter
    _check(lib.skm_fit(ctypes.byref(m), k, _ptr(init), v, max_iter, ctypes.byref(o),
                       _ptr(workspace), workspace.numel(), _ptr(assign), _ptr(centers),
                       _ptr(centers64), ctypes.byref(st), _stream()))
    it = st.iterations
    stats = FitStats(it, bool(st.converged), st.objective, st.sims_point_center,
                     st.sims_center_center, st.rechecks, st.sim_kernel_launches,
                     st.sim_kernel_rows, st.sim_kernel_nnz, st.sim_kernel_ms)
    if per_iter:
        stats.changed_per_iter = ch[:it].copy()
        stats.sims_per_iter = sm[:it].copy()
        stats.objective_per_iter = ob[:it].copy()
    return assign, centers, centers64, stats


def assign(X: DeviceCSR, centers, workspace=None, want_second=True):
    """Runs skm_assign against fixed float32 (k, d) centres.  Returns
    (assign, best, second) device tensors; asynchronous on the current
    stream."""
    import torch
    lib = load()
    dev = X.col.device
    k = int(centers.shape[0])
    m = X.matrix()
    if workspace is None:
        size = lib.skm_assign_workspace_size(ctypes.byref(m), k)
        if size == 0:
            raise SkmError(ERR_INVALID_ARG, lib.skm_last_error().decode(errors="replace"))
        workspace = torch.empty(size, dtype=torch.uint8, device=dev)
    a = torch.empty(X.n, dtype=torch.int32, device=dev)
    best = torch.empty(X.n, dtype=torch.float32, device=dev)
    second = torch.empty(X.n, dtype=torch.float32, device=dev) if want_second else None
    c = centers.contiguous()
    _check(lib.skm_assign(ctypes.byref(m), k, _ptr(c), _ptr(a), _ptr(best), _ptr(second),
                          _ptr(workspace), workspace.numel(), _stream()))
    return a, best, second


NOALLOC_SCRATCH_BYTES = 64 << 20


def assign_noalloc(X: DeviceCSR, centers, a=None, best=None, second=None):
    """Runs skm_assign_noalloc (CSR rows, library-owned scratch, no device
    allocation inside the call) into the given output tensors (allocated here
    when None).  Returns (assign, best, second); asynchronous on the current
    stream."""
    import torch
    lib = load()
    dev = X.col.device
    k = int(centers.shape[0])
    m = X.matrix()
    a = torch.empty(X.n, dtype=torch.int32, device=dev) if a is None else a
    best = torch.empty(X.n, dtype=torch.float32, device=dev) if best is None else best
    c = centers.contiguous()
    _check(lib.skm_assign_noalloc(ctypes.byref(m), k, _ptr(c), _ptr(a), _ptr(best),
                                  _ptr(second), _stream()))
    return a, best, second


def _batch_arrays(problems):
    ms = (SkmMatrix * len(problems))(*[X.matrix() for X, _, _, _ in problems])
    ks = np.array([int(k) for _, k, _, _ in problems], np.int32)
    its = np.array([int(it) for _, _, _, it in problems], np.int32)
    return ms, ks, its


def batched_workspace_size(problems, variant="hamerly", workers=0, **opts) -> int:
    """problems: list of (X, k, init_centers, max_iter)."""
    lib = load()
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    ms, ks, _ = _batch_arrays(problems)
    o = _options(**opts)
    size = lib.skm_fit_batched_workspace_size(len(problems), ms, ks.ctypes.data, v,
                                              ctypes.byref(o), workers)
    if size == 0:
        raise SkmError(ERR_INVALID_ARG, lib.skm_last_error().decode(errors="replace"))
    return int(size)


def fit_batched(problems, variant="hamerly", workers=0, workspace=None, want_centers=True,
                **opts):
    """Runs skm_fit_batched over problems = [(X, k, init (k, d) float32
    device tensor, max_iter), ...].  Returns a list of (assign, centers or
    None, FitStats) per problem."""
    import torch
    lib = load()
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    nb = len(problems)
    ms, ks, its = _batch_arrays(problems)
    o = _options(**opts)
    if workspace is None:
        workspace = torch.empty(batched_workspace_size(problems, variant, workers, **opts),
                                dtype=torch.uint8, device=problems[0][0].col.device)
    inits = [init.contiguous() for _, _, init, _ in problems]
    outs = [torch.empty(X.n, dtype=torch.int32, device=X.col.device) for X, _, _, _ in problems]
    cents = ([torch.empty((int(k), X.d), dtype=torch.float32, device=X.col.device)
              for X, k, _, _ in problems] if want_centers else None)
    init_p = (ctypes.c_void_p * nb)(*[_ptr(t) for t in inits])
    out_p = (ctypes.c_void_p * nb)(*[_ptr(t) for t in outs])
    cen_p = (ctypes.c_void_p * nb)(*[_ptr(t) for t in cents]) if want_centers else None
    st = (SkmStats * nb)()
    _check(lib.skm_fit_batched(nb, ms, ks.ctypes.data, init_p, v, its.ctypes.data,
                               ctypes.byref(o), workers, _ptr(workspace), workspace.numel(),
                               out_p, cen_p, st, _stream()))
    res = []
    for b in range(nb):
        x = st[b]
        res.append((outs[b], cents[b] if want_centers else None,
                    FitStats(x.iterations, bool(x.converged), x.objective, x.sims_point_center,
                             x.sims_center_center, x.rechecks, x.sim_kernel_launches,
                             x.sim_kernel_rows, x.sim_kernel_nnz, x.sim_kernel_ms)))
    return res
