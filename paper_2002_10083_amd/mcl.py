"""ctypes binding of ``libmcl.so`` (include/mcl.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the shared library.  PyTorch provides device memory (through the
library's allocator callback, backed by torch's caching allocator) and the
stream.  If the library is missing this module raises at import time -- there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmcl.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libmcl.so is not built: run `python -m paper_2002_10083_amd.build` "
                      "(or __graft_entry__.build()) first")

_lib = ctypes.CDLL(LIB_PATH)

MCL_OK, MCL_EINVAL, MCL_ENOMEM, MCL_EHIP = 0, -1, -2, -3
EST_BOUND, EST_COHEN, EST_MLP = 0, 1, 2


class MclError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("mcl error %d: %s" % (code, msg))
        self.code = code


# --------------------------------------------------------------------------
# C structs
# --------------------------------------------------------------------------
class _CSC(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("colptr", ctypes.c_void_p), ("rowidx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("prune_threshold", ctypes.c_double), ("select_num", ctypes.c_int32),
                ("recover_num", ctypes.c_int32), ("recover_pct", ctypes.c_double),
                ("inflation", ctypes.c_double), ("estimator", ctypes.c_int32),
                ("cohen_keys", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("iteration", ctypes.c_int32), ("est_scale", ctypes.c_double),
                ("mlp_weights", ctypes.c_void_p), ("validate", ctypes.c_int32),
                ("bin_policy", ctypes.c_int32), ("est_out", ctypes.c_void_p),
                ("nnz_out", ctypes.c_void_p),
                ("phase_bytes", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("flops", ctypes.c_int64), ("nnz_product", ctypes.c_int64),
                ("nnz_kept", ctypes.c_int64), ("n_overflow", ctypes.c_int64),
                ("n_selected", ctypes.c_int64), ("n_recovered", ctypes.c_int64),
                ("n_global", ctypes.c_int64),
                ("t_symbolic_ms", ctypes.c_double), ("t_estimate_ms", ctypes.c_double),
                ("t_numeric_ms", ctypes.c_double), ("t_fallback_ms", ctypes.c_double),
                ("t_compact_ms", ctypes.c_double), ("t_merge_ms", ctypes.c_double),
                ("t_total_ms", ctypes.c_double), ("max_change", ctypes.c_double),
                ("peak_workspace_bytes", ctypes.c_int64),
                ("bin_cols", ctypes.c_int64 * 8), ("bin_ms", ctypes.c_double * 8),
                ("bin_flops", ctypes.c_int64 * 8), ("bin_bnnz", ctypes.c_int64 * 8),
                ("bin_out", ctypes.c_int64 * 8), ("n_phases", ctypes.c_int64),
                ("bin_part_ms", ctypes.c_double * 8), ("bin_prod", ctypes.c_int64 * 8),
                ("n_dense", ctypes.c_int64)]

    def as_dict(self):
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            d[k] = list(v) if k.startswith("bin_") else v
        return d


_P = ctypes.c_void_p
_lib.mcl_default_params.argtypes = [ctypes.POINTER(Params)]
_lib.mcl_last_error.restype = ctypes.c_char_p
_lib.mcl_normalize.argtypes = [ctypes.POINTER(_CSC), _P]
_lib.mcl_expand.argtypes = [ctypes.POINTER(_CSC), ctypes.POINTER(_CSC), ctypes.POINTER(_CSC),
                            ctypes.POINTER(Params), ctypes.POINTER(_Allocator), _P,
                            ctypes.POINTER(Stats)]
_lib.mcl_prune.argtypes = [ctypes.POINTER(_CSC), ctypes.POINTER(_CSC), ctypes.POINTER(Params),
                           ctypes.POINTER(_Allocator), _P, ctypes.POINTER(Stats)]
_lib.mcl_inflate.argtypes = [ctypes.POINTER(_CSC), ctypes.c_double, _P,
                             ctypes.POINTER(ctypes.c_double)]
_lib.mcl_iterate.argtypes = [ctypes.POINTER(_CSC), ctypes.POINTER(_CSC), _P, ctypes.c_int64, _P,
                             ctypes.POINTER(Params), ctypes.POINTER(_Allocator), _P,
                             ctypes.POINTER(Stats), ctypes.POINTER(ctypes.c_double)]
_lib.mcl_merge_partials.argtypes = [ctypes.POINTER(_CSC), ctypes.c_int32, ctypes.POINTER(_CSC),
                                    ctypes.POINTER(_Allocator), _P, ctypes.POINTER(Stats)]
_lib.mcl_symbolic.argtypes = [ctypes.POINTER(_CSC), ctypes.POINTER(_CSC), _P, _P,
                              ctypes.POINTER(_Allocator), _P]
_lib.mcl_estimate.argtypes = [ctypes.POINTER(_CSC), ctypes.POINTER(_CSC), ctypes.POINTER(Params),
                              _P, _P, ctypes.POINTER(_Allocator), _P]
_lib.mcl_components.argtypes = [ctypes.POINTER(_CSC), _P, ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(_Allocator), _P]
_lib.mcl_components_noalloc.argtypes = [ctypes.POINTER(_CSC), _P, ctypes.POINTER(ctypes.c_int64), _P]
_lib.mcl_mlp_packed_bytes.restype = ctypes.c_size_t
_lib.mcl_mlp_state_floats.restype = ctypes.c_size_t
_lib.mcl_mlp_forward.argtypes = [_P, _P, ctypes.c_int64, _P, _P]
_lib.mcl_mlp_init.argtypes = [_P, ctypes.c_uint64, _P]
_lib.mcl_mlp_train_step.argtypes = [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_float,
                                    ctypes.POINTER(ctypes.c_float), _P, _P]

_lib.mcl_expand_host.argtypes = [ctypes.POINTER(_CSC), ctypes.POINTER(_CSC), ctypes.POINTER(_CSC),
                                 ctypes.c_int32, ctypes.POINTER(Stats)]
_lib.mcl_host_free.argtypes = [ctypes.POINTER(_CSC)]
_lib.mcl_expand_dispatch.argtypes = [ctypes.POINTER(_CSC), ctypes.POINTER(_CSC), ctypes.POINTER(_CSC),
                                     ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(Params),
                                     ctypes.POINTER(_Allocator), _P, ctypes.POINTER(Stats),
                                     ctypes.POINTER(ctypes.c_int32)]

#: every symbol include/mcl.h declares
EXPORTS = ("mcl_default_params", "mcl_normalize", "mcl_expand", "mcl_prune", "mcl_inflate",
           "mcl_iterate", "mcl_merge_partials", "mcl_components", "mcl_components_noalloc",
           "mcl_symbolic", "mcl_estimate",
           "mcl_mlp_packed_bytes", "mcl_mlp_forward", "mcl_mlp_state_floats", "mcl_mlp_init",
           "mcl_mlp_train_step", "mcl_last_error", "mcl_expand_host", "mcl_host_free",
           "mcl_expand_dispatch")

#: default flops threshold of mcl_expand_dispatch (include/mcl.h)
DISPATCH_GPU_MIN_FLOPS = 3_000_000


def _check(rc):
    if rc != MCL_OK:
        raise MclError(rc, (_lib.mcl_last_error() or b"").decode())


# --------------------------------------------------------------------------
# torch-backed allocator
# --------------------------------------------------------------------------
class _TorchAllocator:
    """Stream-ordered allocator for the library, backed by torch's caching
    allocator.  Blocks stay referenced in ``live`` until the library frees
    them or Python takes ownership of an output array."""

    def __init__(self):
        self.live = {}
        self.lock = threading.Lock()
        self.fail_after = None     # test hook: return NULL after this many allocations
        self.count = 0

        def _alloc(ctx, nbytes, stream):
            try:
                with self.lock:
                    self.count += 1
                    if self.fail_after is not None and self.count > self.fail_after:
                        return None
                t = torch.empty(max(int(nbytes), 8), dtype=torch.uint8, device="cuda")
                p = t.data_ptr()
                with self.lock:
                    self.live[p] = t
                return p
            except Exception:          # out of memory -> NULL -> MCL_ENOMEM
                return None

        def _free(ctx, ptr, stream):
            with self.lock:
                self.live.pop(ptr, None)

        self._cb_alloc = _ALLOC_FN(_alloc)
        self._cb_free = _FREE_FN(_free)
        self.struct = _Allocator(self._cb_alloc, self._cb_free, None)

    def take(self, ptr, dtype, n):
        """Claim an output block as a typed tensor of n elements."""
        if not ptr:
            return torch.empty(0, dtype=dtype, device="cuda")
        with self.lock:
            t = self.live.pop(ptr)
        return t.view(dtype)[:n] if n > 0 else t.view(dtype)[:0]


_ALLOCATOR = None


def _allocator() -> _TorchAllocator:
    global _ALLOCATOR
    if _ALLOCATOR is None:
        _ALLOCATOR = _TorchAllocator()
    return _ALLOCATOR


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# --------------------------------------------------------------------------
# device CSC
# --------------------------------------------------------------------------
@dataclass
class DeviceCSC:
    """CSC matrix resident in device memory (int64 colptr, int32 rowidx, f64 val)."""

    nrows: int
    ncols: int
    colptr: torch.Tensor
    rowidx: torch.Tensor
    val: torch.Tensor

    @property
    def nnz(self) -> int:
        return int(self.rowidx.numel())

    @staticmethod
    def from_host(m, device="cuda") -> "DeviceCSC":
        return DeviceCSC(int(m.nrows), int(m.ncols),
                         torch.from_numpy(np.ascontiguousarray(m.colptr, np.int64)).to(device),
                         torch.from_numpy(np.ascontiguousarray(m.rowidx, np.int32)).to(device),
                         torch.from_numpy(np.ascontiguousarray(m.val, np.float64)).to(device))

    def to_host(self):
        from mclgen import CSC
        return CSC(self.nrows, self.ncols, self.colptr.cpu().numpy(), self.rowidx.cpu().numpy(),
                   self.val.cpu().numpy())

    def clone(self) -> "DeviceCSC":
        return DeviceCSC(self.nrows, self.ncols, self.colptr.clone(), self.rowidx.clone(),
                         self.val.clone())

    def _c(self) -> _CSC:
        return _CSC(self.nrows, self.ncols, self.nnz, self.colptr.data_ptr(),
                    self.rowidx.data_ptr() if self.nnz else 0,
                    self.val.data_ptr() if self.nnz else 0)


def _wrap_out(c: _CSC, al: _TorchAllocator) -> DeviceCSC:
    nnz = int(c.nnz)
    colptr = al.take(c.colptr, torch.int64, int(c.ncols) + 1)
    rowidx = al.take(c.rowidx, torch.int32, nnz)
    val = al.take(c.val, torch.float64, nnz)
    return DeviceCSC(int(c.nrows), int(c.ncols), colptr, rowidx, val)


def default_params(**kw) -> Params:
    p = Params()
    _lib.mcl_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        if isinstance(v, torch.Tensor):
            v = v.data_ptr()
        setattr(p, k, v)
    return p


def _params(params, kw) -> Params:
    if params is None:
        return default_params(**kw)
    if kw:
        p = Params()
        ctypes.pointer(p)[0] = params
        for k, v in kw.items():
            setattr(p, k, v.data_ptr() if isinstance(v, torch.Tensor) else v)
        return p
    return params


# --------------------------------------------------------------------------
# entry points
# --------------------------------------------------------------------------
def normalize_(A: DeviceCSC) -> DeviceCSC:
    """Column-stochastic normalisation in place."""
    c = A._c()
    _check(_lib.mcl_normalize(ctypes.byref(c), _stream()))
    return A


def expand(A: DeviceCSC, B: DeviceCSC, params: Optional[Params] = None, **kw):
    """C = A B (unpruned).  Returns (C, stats dict)."""
    p = _params(params, kw)
    al = _allocator()
    out = _CSC()
    st = Stats()
    a, b = A._c(), B._c()
    _check(_lib.mcl_expand(ctypes.byref(a), ctypes.byref(b), ctypes.byref(out), ctypes.byref(p),
                           ctypes.byref(al.struct), _stream(), ctypes.byref(st)))
    return _wrap_out(out, al), st.as_dict()


def prune(B: DeviceCSC, params: Optional[Params] = None, **kw):
    p = _params(params, kw)
    al = _allocator()
    out = _CSC()
    st = Stats()
    b = B._c()
    _check(_lib.mcl_prune(ctypes.byref(b), ctypes.byref(out), ctypes.byref(p),
                          ctypes.byref(al.struct), _stream(), ctypes.byref(st)))
    return _wrap_out(out, al), st.as_dict()


def inflate_(C: DeviceCSC, r: float = 2.0) -> float:
    """In-place inflation; returns max |column sum - 1|."""
    c = C._c()
    err = ctypes.c_double(0.0)
    _check(_lib.mcl_inflate(ctypes.byref(c), float(r), _stream(), ctypes.byref(err)))
    return err.value


def iterate(A: DeviceCSC, params: Optional[Params] = None, comp_ptr: Optional[torch.Tensor] = None,
            active: Optional[torch.Tensor] = None, **kw):
    """One fused MCL iteration.  Returns (A_next, max_change, stats); max_change
    is a float, or a numpy array per component in batched form."""
    p = _params(params, kw)
    al = _allocator()
    out = _CSC()
    st = Stats()
    a = A._c()
    if comp_ptr is not None:
        ncomp = int(comp_ptr.numel()) - 1
        mc = (ctypes.c_double * ncomp)()
        _check(_lib.mcl_iterate(ctypes.byref(a), ctypes.byref(out), comp_ptr.data_ptr(), ncomp,
                                active.data_ptr(), ctypes.byref(p), ctypes.byref(al.struct),
                                _stream(), ctypes.byref(st), mc))
        change = np.frombuffer(mc, dtype=np.float64).copy()
    else:
        mc = ctypes.c_double(0.0)
        _check(_lib.mcl_iterate(ctypes.byref(a), ctypes.byref(out), None, 0, None, ctypes.byref(p),
                                ctypes.byref(al.struct), _stream(), ctypes.byref(st),
                                ctypes.byref(mc)))
        change = mc.value
    return _wrap_out(out, al), change, st.as_dict()


def merge_partials(parts: Sequence[DeviceCSC]):
    """C = sum of the parts, equal rows summed in list order."""
    al = _allocator()
    arr = (_CSC * len(parts))(*[p._c() for p in parts])
    out = _CSC()
    st = Stats()
    _check(_lib.mcl_merge_partials(arr, len(parts), ctypes.byref(out), ctypes.byref(al.struct),
                                   _stream(), ctypes.byref(st)))
    return _wrap_out(out, al), st.as_dict()


def components(A: DeviceCSC):
    """Connected components of the pattern of a square A (undirected): returns
    (labels, ncomp) with labels a device int32 tensor holding, per vertex, the
    smallest vertex id of its component."""
    al = _allocator()
    labels = torch.empty(A.ncols, dtype=torch.int32, device="cuda")
    nc = ctypes.c_int64(0)
    a = A._c()
    _check(_lib.mcl_components(ctypes.byref(a), labels.data_ptr() if A.ncols else None,
                               ctypes.byref(nc), ctypes.byref(al.struct), _stream()))
    return labels, int(nc.value)


#: largest vertex count mcl_components_noalloc accepts (its fixed scratch)
NOALLOC_MAX_VERTICES = 1 << 22


def components_noalloc(A: DeviceCSC, labels=None, sync: bool = True):
    """mcl_components_noalloc: the same labels as components(), computed in the
    library's fixed per-GPU scratch (no device allocation by the library).
    `labels` may be a caller-provided device int32 tensor of A.ncols entries.
    Returns (labels, ncomp); ncomp is None when sync is False (the call then
    only enqueues its kernels)."""
    if labels is None:
        labels = torch.empty(A.ncols, dtype=torch.int32, device="cuda")
    nc = ctypes.c_int64(0)
    a = A._c()
    _check(_lib.mcl_components_noalloc(ctypes.byref(a), labels.data_ptr() if A.ncols else None,
                                       ctypes.byref(nc) if sync else None, _stream()))
    return labels, (int(nc.value) if sync else None)


def symbolic(A: DeviceCSC, B: DeviceCSC, exact: bool = False):
    """flops per column (and exact product nnz per column when exact=True)."""
    al = _allocator()
    flops = torch.empty(B.ncols, dtype=torch.int64, device="cuda")
    nnz = torch.empty(B.ncols, dtype=torch.int64, device="cuda") if exact else None
    a, b = A._c(), B._c()
    _check(_lib.mcl_symbolic(ctypes.byref(a), ctypes.byref(b), flops.data_ptr(),
                             nnz.data_ptr() if exact else None, ctypes.byref(al.struct), _stream()))
    return flops, nnz


def estimate(A: DeviceCSC, B: DeviceCSC, params: Optional[Params] = None, features=False, **kw):
    """Per-column output-size estimate (and the 12 MLP features if asked)."""
    p = _params(params, kw)
    al = _allocator()
    est = torch.empty(B.ncols, dtype=torch.float32, device="cuda")
    feat = torch.empty(B.ncols * 12, dtype=torch.float32, device="cuda") if features else None
    a, b = A._c(), B._c()
    _check(_lib.mcl_estimate(ctypes.byref(a), ctypes.byref(b), ctypes.byref(p), est.data_ptr(),
                             feat.data_ptr() if features else None, ctypes.byref(al.struct),
                             _stream()))
    return (est, feat.view(B.ncols, 12)) if features else est


# ---- host matrices: CPU hash SpGEMM and the CPU/GPU dispatch
def _host_c(m):
    """C descriptor of a host CSC (numpy arrays, kept alive by the caller)."""
    cp = np.ascontiguousarray(m.colptr, np.int64)
    ri = np.ascontiguousarray(m.rowidx, np.int32)
    va = np.ascontiguousarray(m.val, np.float64)
    keep = (cp, ri, va)
    c = _CSC(int(m.nrows), int(m.ncols), int(cp[-1]) if cp.size else 0, cp.ctypes.data,
             ri.ctypes.data if ri.size else 0, va.ctypes.data if va.size else 0)
    return c, keep


def _take_host(c: _CSC):
    """Copy a library-allocated host matrix into numpy arrays and free it."""
    from mclgen import CSC
    n, nz = int(c.ncols), int(c.nnz)
    try:
        cp = np.ctypeslib.as_array(ctypes.cast(c.colptr, ctypes.POINTER(ctypes.c_int64)), (n + 1,)).copy()
        if nz:
            ri = np.ctypeslib.as_array(ctypes.cast(c.rowidx, ctypes.POINTER(ctypes.c_int32)), (nz,)).copy()
            va = np.ctypeslib.as_array(ctypes.cast(c.val, ctypes.POINTER(ctypes.c_double)), (nz,)).copy()
        else:
            ri, va = np.zeros(0, np.int32), np.zeros(0, np.float64)
    finally:
        _lib.mcl_host_free(ctypes.byref(c))
    return CSC(int(c.nrows), n, cp, ri, va)


def expand_host(A, B, nthreads: int = 0):
    """mcl_expand_host: C = A B on the host's cores (multithreaded hash
    SpGEMM) for host CSC matrices.  Returns (C as a host CSC, stats dict)."""
    a, ka = _host_c(A)
    b, kb = _host_c(B)
    out = _CSC()
    st = Stats()
    _check(_lib.mcl_expand_host(ctypes.byref(a), ctypes.byref(b), ctypes.byref(out), int(nthreads),
                                ctypes.byref(st)))
    del ka, kb
    return _take_host(out), st.as_dict()


def expand_dispatch(A, B, gpu_min_flops: int = 0, nthreads: int = 0, params: Optional[Params] = None,
                    **kw):
    """mcl_expand_dispatch: host matrices in and out; the product runs on the
    CPU when its flops are below gpu_min_flops (0 = the library's measured
    default), else on the GPU.  Returns (C, stats dict, "cpu" | "gpu")."""
    p = _params(params, kw)
    al = _allocator()
    a, ka = _host_c(A)
    b, kb = _host_c(B)
    out = _CSC()
    st = Stats()
    where = ctypes.c_int32(-1)
    _check(_lib.mcl_expand_dispatch(ctypes.byref(a), ctypes.byref(b), ctypes.byref(out),
                                    int(gpu_min_flops), int(nthreads), ctypes.byref(p),
                                    ctypes.byref(al.struct),
                                    _stream() if torch.cuda.is_available() else None,
                                    ctypes.byref(st), ctypes.byref(where)))
    del ka, kb
    return _take_host(out), st.as_dict(), ("gpu" if where.value == 1 else "cpu")


# ---- learned estimator
def mlp_packed_bytes() -> int:
    return int(_lib.mcl_mlp_packed_bytes())


def mlp_state_floats() -> int:
    return int(_lib.mcl_mlp_state_floats())


def mlp_init(seed: int = 0):
    """Returns (state, packed): FP32 master + Adam state, and the BF16 blob."""
    state = torch.zeros(mlp_state_floats(), dtype=torch.float32, device="cuda")
    packed = torch.zeros(mlp_packed_bytes() // 2, dtype=torch.int16, device="cuda")
    _check(_lib.mcl_mlp_init(state.data_ptr(), int(seed), _stream()))
    return state, packed


def mlp_forward(packed: torch.Tensor, feat: torch.Tensor) -> torch.Tensor:
    feat = feat.contiguous().float()
    rows = feat.numel() // 12
    out = torch.empty(rows, dtype=torch.float32, device="cuda")
    _check(_lib.mcl_mlp_forward(packed.data_ptr(), feat.data_ptr(), rows, out.data_ptr(), _stream()))
    return out


def mlp_train_step(state, packed, feat, target, lr=1e-3, want_grad=False):
    feat = feat.contiguous().float()
    target = target.contiguous().float()
    rows = target.numel()
    loss = ctypes.c_float(0.0)
    grad = torch.empty(mlp_state_floats(), dtype=torch.float32, device="cuda") if want_grad else None
    _check(_lib.mcl_mlp_train_step(state.data_ptr(), packed.data_ptr(), feat.data_ptr(),
                                   target.data_ptr(), rows, float(lr), ctypes.byref(loss),
                                   grad.data_ptr() if want_grad else None, _stream()))
    return (loss.value, grad) if want_grad else loss.value
