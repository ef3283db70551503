"""Python binding of libsigntri.so (the C ABI in include/signtri.h).

Argument marshalling only: every step of sign(T) runs in the library's HIP
kernels.  PyTorch provides device memory and the current HIP stream.  There
is no fallback: if the library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading
from collections.abc import Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
# SIGNTRI_LIB: another build of the same library (the host-sanitizer build of
# the CPU checks); by default the in-tree one
LIB_PATH = os.environ.get("SIGNTRI_LIB") or os.path.join(HERE, "libsigntri.so")

R64, C128 = 0, 1
COL_MAJOR, ROW_MAJOR = 0, 1
MODES = {"fp64": 0, "mixed": 1, "fp32": 2}
ALGOS = {"auto": 0, "ph": 1, "ps": 2, "proj": 3}
PATH_NAMES = {0: "trivial", 1: "ph", 2: "ps", 3: "proj"}
SWEEPS = {"auto": 0, "dataflow": 1, "superdiag": 2}
PRODUCTS = {"masked": 0, "dense": 1}
SWEEP_NAMES = {0: "-", 1: "dataflow", 2: "superdiag"}

EXPORTS = ("signtri", "signtri_workspace_size", "signtri_batched",
           "signtri_batched_workspace_size", "signtri_strerror", "sign_tri",
           "signtri_plan_host", "signtri_release", "signtri_profile_enable",
           "signtri_profile_read", "signtri_autotune", "signtri_tune_lookup",
           "signtri_tune_save", "signtri_tune_load", "signtri_tune_clear", "signtri_noalloc",
           "signtri_autotune_batched", "signtri_fun", "signtri_signm_batched")
FAMILIES = {"scan": 0, "diag": 1, "gemm": 2, "solve": 3, "aux": 4, "resid": 5,
            "corr": 6, "syl": 7, "flow": 8, "batched": 9, "convert": 10, "proj": 11,
            "proj_out": 12}


class Info(ctypes.Structure):
    _fields_ = [
        ("path", ctypes.c_int32), ("model_pick", ctypes.c_int32),
        ("n_pos", ctypes.c_int64), ("n_neg", ctypes.c_int64), ("swaps", ctypes.c_int64),
        ("w_ph", ctypes.c_double), ("w_ps", ctypes.c_double),
        ("refine_steps", ctypes.c_int32), ("tile", ctypes.c_int32),
        ("fallback_tiles", ctypes.c_int64), ("correction_rel", ctypes.c_double),
        ("bad_index", ctypes.c_int64), ("sweep", ctypes.c_int32),
        ("wgs_per_cu", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["path_name"] = PATH_NAMES.get(self.path, "?")
        d["sweep_name"] = SWEEP_NAMES.get(self.sweep, "?")
        d["model_pick_name"] = PATH_NAMES.get(self.model_pick, "?")
        return d


class Options(ctypes.Structure):
    _fields_ = [
        ("tile", ctypes.c_int32), ("max_refine_steps", ctypes.c_int32),
        ("stall_ratio", ctypes.c_double), ("no_fallback", ctypes.c_int32),
        ("max_splits", ctypes.c_int32), ("force_stall", ctypes.c_int64),
        ("sweep", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32),
        ("products", ctypes.c_int32),
    ]


class TuneEntry(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int32), ("mode", ctypes.c_int32), ("path", ctypes.c_int32),
        ("log2n", ctypes.c_int32), ("sweep", ctypes.c_int32), ("tile", ctypes.c_int32),
        ("wgs_per_cu", ctypes.c_int32), ("ms", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["sweep_name"] = SWEEP_NAMES.get(self.sweep, "?")
        return d


class SignTriError(RuntimeError):
    def __init__(self, code: int, message: str, info: dict | None = None):
        super().__init__("signtri error %d: %s" % (code, message))
        self.code = code
        self.info = info or {}


_lock = threading.Lock()
_lib = None


def lib() -> ctypes.CDLL:
    """Load libsigntri.so, raising if it is not built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libsigntri.so is not built (%s); run __graft_entry__.build()"
                                   % LIB_PATH)
            L = ctypes.CDLL(LIB_PATH)
            i64, p, sz, i32 = ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
            L.signtri.argtypes = [p, i64, p, i64, i64, i32, i32, i32, i32, p, sz, p,
                                  ctypes.POINTER(Options), ctypes.POINTER(Info)]
            L.signtri.restype = i32
            L.signtri_workspace_size.argtypes = [i64, i32, i32, i32, i32]
            L.signtri_workspace_size.restype = sz
            L.signtri_batched.argtypes = [ctypes.POINTER(p), ctypes.POINTER(i64), ctypes.POINTER(p),
                                          ctypes.POINTER(i64), ctypes.POINTER(i64), i64, i32, i32,
                                          i32, p, sz, p, ctypes.POINTER(Options),
                                          ctypes.POINTER(Info)]
            L.signtri_batched.restype = i32
            L.signtri_batched_workspace_size.argtypes = [ctypes.POINTER(i64), i64, i32, i32]
            L.signtri_batched_workspace_size.restype = sz
            L.signtri_signm_batched.argtypes = [ctypes.POINTER(p), ctypes.POINTER(i64),
                                                ctypes.POINTER(p), ctypes.POINTER(i64),
                                                ctypes.POINTER(i64), i64, i32, p,
                                                ctypes.POINTER(ctypes.c_int32)]
            L.signtri_signm_batched.restype = i32
            L.signtri_strerror.argtypes = [i32]
            L.signtri_strerror.restype = ctypes.c_char_p
            L.sign_tri.argtypes = [p, i64, i64, i32, p]
            L.sign_tri.restype = i32
            L.signtri_noalloc.argtypes = [p, i64, p, i64, i64, i32, p, ctypes.POINTER(Info)]
            L.signtri_noalloc.restype = i32
            L.signtri_plan_host.argtypes = [p, i64, i32, ctypes.POINTER(Info)]
            L.signtri_plan_host.restype = i32
            L.signtri_release.argtypes = []
            L.signtri_release.restype = None
            L.signtri_profile_enable.argtypes = [i32]
            L.signtri_profile_enable.restype = None
            L.signtri_profile_read.argtypes = [i32, ctypes.POINTER(ctypes.c_double),
                                               ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]
            L.signtri_profile_read.restype = i32
            L.signtri_autotune.argtypes = [p, i64, p, i64, i64, i32, i32, i32, p, i32,
                                           ctypes.POINTER(TuneEntry)]
            L.signtri_autotune.restype = i32
            L.signtri_fun.argtypes = [p, i64, p, p, i64, i64, i32, p, ctypes.POINTER(Info)]
            L.signtri_fun.restype = i32
            L.signtri_autotune_batched.argtypes = [ctypes.POINTER(p), ctypes.POINTER(i64),
                                                   ctypes.POINTER(p), ctypes.POINTER(i64),
                                                   ctypes.POINTER(i64), i64, i32, i32, p, i32,
                                                   ctypes.POINTER(TuneEntry)]
            L.signtri_autotune_batched.restype = i32
            L.signtri_tune_lookup.argtypes = [i32, i32, i32, i64, ctypes.POINTER(TuneEntry)]
            L.signtri_tune_lookup.restype = i32
            L.signtri_tune_save.argtypes = [ctypes.c_char_p]
            L.signtri_tune_save.restype = i32
            L.signtri_tune_load.argtypes = [ctypes.c_char_p]
            L.signtri_tune_load.restype = i32
            L.signtri_tune_clear.argtypes = []
            L.signtri_tune_clear.restype = None
            _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().signtri_strerror(int(code)).decode()


def workspace_size(n: int, complex_: bool = False, mode: str = "fp64", algo: str = "auto",
                   row_major: bool = False) -> int:
    return int(lib().signtri_workspace_size(n, C128 if complex_ else R64,
                                            ROW_MAJOR if row_major else COL_MAJOR, MODES[mode],
                                            ALGOS[algo]))


def plan_host(signs, complex_: bool = False) -> dict:
    """Section 3 planner on host signs (+1/-1), without a GPU."""
    import numpy as np

    s = np.ascontiguousarray(np.asarray(signs, dtype=np.int8))
    info = Info()
    rc = lib().signtri_plan_host(s.ctypes.data if s.size else None, int(s.size),
                                 C128 if complex_ else R64, ctypes.byref(info))
    if rc != 0:
        raise ValueError("invalid sign vector")
    return info.as_dict()


def _dtype_code(t) -> int:
    import torch

    if t.dtype == torch.float64:
        return R64
    if t.dtype == torch.complex128:
        return C128
    raise TypeError("T must be float64 or complex128, got %s" % t.dtype)


def _layout(t):
    """(layout code, leading dimension) of a 2-D strided tensor, or None."""
    n0, n1 = t.shape
    s0, s1 = t.stride()
    if s0 == 1 and (s1 >= max(1, n0) or n1 <= 1):
        return COL_MAJOR, max(s1, n0, 1)
    if s1 == 1 and (s0 >= max(1, n1) or n0 <= 1):
        return ROW_MAJOR, max(s0, n1, 1)
    return None


def empty_like_layout(t):
    """A new tensor with t's shape, dtype, device and storage order."""
    import torch

    lay = _layout(t)
    if lay is not None and lay[0] == COL_MAJOR and t.shape[0] > 1:
        return torch.empty(t.shape[1], t.shape[0], dtype=t.dtype, device=t.device).t()
    return torch.empty(t.shape, dtype=t.dtype, device=t.device)


def _stream_handle(t, stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream(t.device)
    return ctypes.c_void_p(int(stream.cuda_stream))


def _opts(options: dict | None):
    if not options:
        return None
    o = Options()
    for k, v in options.items():
        if k == "sweep" and isinstance(v, str):
            v = SWEEPS[v]
        if k == "products" and isinstance(v, str):
            v = PRODUCTS[v]
        setattr(o, k, v)
    return ctypes.byref(o)


def sign_tri(T, mode: str = "fp64", algo: str = "auto", out=None, workspace=None,
             stream=None, options: dict | None = None):
    """U = sign(T) for a square upper-triangular CUDA/HIP tensor T.

    T may be column- or row-major (with padding); U (``out`` or a new tensor)
    gets the same storage order.  Returns (U, info dict).  Raises
    SignTriError on a nonzero library return code.
    """
    if T.dim() != 2 or T.shape[0] != T.shape[1]:
        raise ValueError("T must be square")
    n = T.shape[0]
    dt = _dtype_code(T)
    lay = _layout(T)
    if lay is None:
        raise ValueError("T must be column- or row-major strided")
    layout, ldt = lay
    U = out if out is not None else empty_like_layout(T)
    ulay = _layout(U)
    if ulay is None or (n > 1 and ulay[0] != layout) or U.shape != T.shape or U.dtype != T.dtype:
        raise ValueError("out must match T's shape, dtype and storage order")
    ldu = ulay[1]
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    info = Info()
    rc = lib().signtri(T.data_ptr() if n else None, ldt, U.data_ptr() if n else None, ldu, n, dt,
                       layout, MODES[mode], ALGOS[algo], ws_ptr, ws_bytes,
                       _stream_handle(T, stream), _opts(options), ctypes.byref(info))
    if rc != 0:
        raise SignTriError(rc, strerror(rc), info.as_dict())
    return U, info.as_dict()


def sign_tri_noalloc(T, out=None, stream=None):
    """sign(T) through signtri_noalloc(): FP64, column-major T (and U), AUTO path,
    no allocation by the library (its fixed scratch; orders up to 8192).
    Returns (U, info dict); waits for the result."""
    if T.dim() != 2 or T.shape[0] != T.shape[1]:
        raise ValueError("T must be square")
    n = T.shape[0]
    lay = _layout(T)
    if lay is None or (n > 1 and lay[0] != COL_MAJOR):
        raise ValueError("signtri_noalloc takes a column-major T")
    U = out if out is not None else empty_like_layout(T)
    ulay = _layout(U)
    if ulay is None or (n > 1 and ulay[0] != COL_MAJOR) or U.shape != T.shape or U.dtype != T.dtype:
        raise ValueError("out must be column-major with T's shape and dtype")
    info = Info()
    rc = lib().signtri_noalloc(T.data_ptr() if n else None, lay[1], U.data_ptr() if n else None,
                               ulay[1], n, _dtype_code(T), _stream_handle(T, stream),
                               ctypes.byref(info))
    if rc != 0:
        raise SignTriError(rc, strerror(rc), info.as_dict())
    return U, info.as_dict()


def fun_tri(T, fdiag, out=None, stream=None):
    """F = phi(T) for a square upper-triangular column-major tensor T and phi's
    values on the diagonal, fdiag[i] = phi(t_ii) (a tensor of n values on the same
    device, same dtype), by Parlett's substitution (Algorithm 1).  Returns (F, info)."""
    if T.dim() != 2 or T.shape[0] != T.shape[1]:
        raise ValueError("T must be square")
    n = T.shape[0]
    lay = _layout(T)
    if lay is None or (n > 1 and lay[0] != COL_MAJOR):
        raise ValueError("fun_tri takes a column-major T")
    if fdiag.shape != (n,) or fdiag.dtype != T.dtype or fdiag.device != T.device:
        raise ValueError("fdiag must hold n values of T's dtype on T's device")
    fd = fdiag.contiguous()
    F = out if out is not None else empty_like_layout(T)
    info = Info()
    rc = lib().signtri_fun(T.data_ptr() if n else None, lay[1], fd.data_ptr() if n else None,
                           F.data_ptr() if n else None, _layout(F)[1] if n else 1, n,
                           _dtype_code(T), _stream_handle(T, stream), ctypes.byref(info))
    if rc != 0:
        raise SignTriError(rc, strerror(rc), info.as_dict())
    return F, info.as_dict()


def _batch_args(Ts, outs):
    """Host arrays of pointers, leading dimensions and orders for a batch."""
    layouts = [_layout(t) if t.shape[0] else (COL_MAJOR, 1) for t in Ts]
    if any(l is None for l in layouts):
        raise ValueError("every T must be column- or row-major strided")
    nonempty = [l for t, l in zip(Ts, layouts) if t.shape[0] > 1]
    layout = nonempty[0][0] if nonempty else COL_MAJOR
    Us = outs if outs is not None else [empty_like_layout(t) for t in Ts]
    B = len(Ts)
    P = ctypes.c_void_p * B
    I = ctypes.c_int64 * B
    tp = P(*[t.data_ptr() if t.shape[0] else None for t in Ts])
    up = P(*[u.data_ptr() if u.shape[0] else None for u in Us])
    ldt = I(*[l[1] for l in layouts])
    ldu = I(*[_layout(u)[1] if u.shape[0] else 1 for u in Us])
    ns = I(*[t.shape[0] for t in Ts])
    return layout, Us, tp, ldt, up, ldu, ns


def autotune_batched(Ts, mode: str = "fp64", reps: int = 3, outs=None, stream=None) -> dict:
    """Time every dataflow grid on this batch (column-major) and record the fastest
    for the size class of its largest order (used by later batched calls that
    leave wgs_per_cu at 0)."""
    if not Ts:
        raise ValueError("empty batch")
    layout, Us, tp, ldt, up, ldu, ns = _batch_args(Ts, outs)
    if layout != COL_MAJOR:
        raise ValueError("autotune_batched takes column-major matrices")
    best = TuneEntry()
    rc = lib().signtri_autotune_batched(tp, ldt, up, ldu, ns, len(Ts), _dtype_code(Ts[0]),
                                        MODES[mode], _stream_handle(Ts[0], stream), int(reps),
                                        ctypes.byref(best))
    if rc != 0:
        raise SignTriError(rc, strerror(rc))
    return best.as_dict()


class InfoList(Sequence):
    """The infos of a batched call, each turned into a dict when it is read (a
    batch of thousands of matrices would otherwise spend milliseconds on dicts
    nobody reads)."""

    def __init__(self, infos):
        self._infos = infos

    def __len__(self):
        return len(self._infos)

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self._infos[k].as_dict() for k in range(*i.indices(len(self._infos)))]
        return self._infos[i].as_dict()


def sign_tri_batched(Ts, mode: str = "fp64", outs=None, workspace=None, stream=None,
                     options: dict | None = None):
    """Batched form: list of square upper-triangular tensors (same dtype, device
    and storage order).  Returns (list of U, sequence of info dicts)."""
    if not Ts:
        return [], []
    dt = _dtype_code(Ts[0])
    Us = outs if outs is not None else [empty_like_layout(t) for t in Ts]
    B = len(Ts)
    if len(Us) != B:
        raise ValueError("outs must hold one tensor per T")
    tp, up = (ctypes.c_void_p * B)(), (ctypes.c_void_p * B)()
    ldt, ldu, ns = (ctypes.c_int64 * B)(), (ctypes.c_int64 * B)(), (ctypes.c_int64 * B)()
    layout = None
    # one pass over the tensors: each attribute read costs a fraction of a
    # microsecond, which adds up over a large batch
    for b in range(B):
        t, u = Ts[b], Us[b]
        n = t.shape[0]
        ns[b] = n
        if n == 0:
            ldt[b] = ldu[b] = 1
            continue
        lt, lu = _layout(t), _layout(u)
        if lt is None or lu is None:
            raise ValueError("every T and U must be column- or row-major strided")
        if n > 1:
            if layout is None:
                layout = lt[0]
            if lt[0] != layout or lu[0] != layout:
                raise ValueError("every T and U of more than one row must share one storage order")
        tp[b], up[b] = t.data_ptr(), u.data_ptr()
        ldt[b], ldu[b] = lt[1], lu[1]
    infos = (Info * B)()
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    rc = lib().signtri_batched(tp, ldt, up, ldu, ns, B, dt,
                               COL_MAJOR if layout is None else layout, MODES[mode], ws_ptr,
                               ws_bytes, _stream_handle(Ts[0], stream), _opts(options), infos)
    if rc != 0:
        raise SignTriError(rc, strerror(rc))
    return Us, InfoList(infos)


def sign_general_batched(As, outs=None, stream=None):
    """sign(A) for a list of square column-major tensors of order at most 64 (all
    float64 or all complex128, on one device): a Schur decomposition, the
    triangular sign and the back-transformation, in the library's kernels.
    Returns (list of S, list of status codes); raises SignTriError when the
    call fails as a whole (argument errors) or, after filling every S it could,
    with the first failing matrix's code."""
    if not As:
        return [], []
    dt = _dtype_code(As[0])
    Ss = outs if outs is not None else [empty_like_layout(a) for a in As]
    B = len(As)
    if len(Ss) != B:
        raise ValueError("outs must hold one tensor per A")
    ap, sp = (ctypes.c_void_p * B)(), (ctypes.c_void_p * B)()
    lda, lds, ns = (ctypes.c_int64 * B)(), (ctypes.c_int64 * B)(), (ctypes.c_int64 * B)()
    for b in range(B):
        a, o = As[b], Ss[b]
        if a.dim() != 2 or a.shape[0] != a.shape[1] or _dtype_code(a) != dt:
            raise ValueError("every A must be square with the first one's dtype")
        nb = a.shape[0]
        ns[b] = nb
        if nb == 0:
            lda[b] = lds[b] = 1
            continue
        la, lo = _layout(a), _layout(o)
        if nb > 1 and (la is None or lo is None or la[0] != COL_MAJOR or lo[0] != COL_MAJOR):
            raise ValueError("every A and S must be column-major strided")
        ap[b], sp[b] = a.data_ptr(), o.data_ptr()
        lda[b] = la[1] if la else 1
        lds[b] = lo[1] if lo else 1
    st = (ctypes.c_int32 * B)()
    rc = lib().signtri_signm_batched(ap, lda, sp, lds, ns, B, dt, _stream_handle(As[0], stream),
                                     st)
    codes = [int(st[b]) for b in range(B)]
    if rc != 0:
        raise SignTriError(rc, strerror(rc), {"status": codes})
    return Ss, codes


def release() -> None:
    lib().signtri_release()


def profile_enable(on: bool = True) -> None:
    """Start (clearing counters) or stop the library's per-family kernel timers."""
    lib().signtri_profile_enable(1 if on else 0)


def profile_read() -> dict:
    """{family: (milliseconds, launches, algorithmic flops)} for families with launches."""
    out = {}
    for name, k in FAMILIES.items():
        ms, cnt, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        rc = lib().signtri_profile_read(k, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(fl))
        if rc != 0:
            raise SignTriError(rc, strerror(rc))
        if cnt.value:
            out[name] = (ms.value, cnt.value, fl.value)
    return out


def autotune(T, mode: str = "fp64", algo: str = "auto", reps: int = 3, out=None, stream=None) -> dict:
    """Time every sweep variant on the column-major T and record the fastest in the
    library's tuning table (used by later calls that leave those options at 0)."""
    if T.dim() != 2 or T.shape[0] != T.shape[1]:
        raise ValueError("T must be square")
    n = T.shape[0]
    lay = _layout(T)
    if lay is None or (n > 1 and lay[0] != COL_MAJOR):
        raise ValueError("autotune takes a column-major T")
    U = out if out is not None else empty_like_layout(T)
    best = TuneEntry()
    rc = lib().signtri_autotune(T.data_ptr() if n else None, lay[1], U.data_ptr() if n else None,
                                _layout(U)[1], n, _dtype_code(T), MODES[mode], ALGOS[algo],
                                _stream_handle(T, stream), int(reps), ctypes.byref(best))
    if rc != 0:
        raise SignTriError(rc, strerror(rc))
    return best.as_dict()


def tune_lookup(complex_: bool, mode: str, path: str, n: int) -> dict | None:
    e = TuneEntry()
    code = {"ph": 1, "ps": 2, "batched": 8}[path]
    if lib().signtri_tune_lookup(C128 if complex_ else R64, MODES[mode], code, int(n),
                                 ctypes.byref(e)):
        return e.as_dict()
    return None


def tune_save(path: str) -> None:
    if lib().signtri_tune_save(os.fsencode(path)) != 0:
        raise OSError("cannot write tuning table to %s" % path)


def tune_load(path: str) -> None:
    if lib().signtri_tune_load(os.fsencode(path)) != 0:
        raise OSError("cannot read tuning table from %s" % path)


def tune_clear() -> None:
    lib().signtri_tune_clear()
