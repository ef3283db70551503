"""TEST INFRASTRUCTURE ONLY: CPU oracle for U = sign(T), T upper triangular.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library
behind ``include/signtri.h`` and its Python binding) never imports it, and it
never imports the product path.

``sign_tri`` runs the element-by-element Parlett-Higham substitution
(Algorithm 3 of Stotland, Schwartz and Toledo, with Eq. (1) where the two
diagonal signs differ and Eq. (2) where they agree), in FP64 or complex128,
from ``signtri_oracle.c``.  ``trsyl`` solves the triangular Sylvester equation
A X - X B = C that the sign-split (Parlett-Sylvester) form reduces to
(Algorithm 2 with the diagonal blocks of the sign equal to +I and -I).

The C file is compiled with gcc the first time it is needed, with
``-ffp-contract=off`` and no fast-math, so results are reproducible.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

from . import workmodel  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "signtri_oracle.c")
# SIGNTRI_ORACLE_LIB: another build of the same C file (the sanitizer build of
# the CPU checks); by default the one built here
_LIB = os.environ.get("SIGNTRI_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle's C code into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-std=c99", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            path = _LIB if os.path.exists(_LIB) else build()
            lib = ctypes.CDLL(path)
            i64, p, i32 = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
            for name in ("oracle_sign_tri_d", "oracle_sign_tri_z"):
                f = getattr(lib, name)
                f.argtypes = [i64, p, i64, p, i64, i32]
                f.restype = i64
            for name in ("oracle_parlett_d", "oracle_parlett_z"):
                f = getattr(lib, name)
                f.argtypes = [i64, p, i64, p, p, i64]
                f.restype = i64
            for name in ("oracle_trsyl_d", "oracle_trsyl_z"):
                f = getattr(lib, name)
                f.argtypes = [i64, i64, p, i64, p, i64, p, i64, p, i64]
                f.restype = i64
            lib.oracle_num_threads.argtypes = []
            lib.oracle_num_threads.restype = i32
            _lib = lib
    return _lib


class DomainError(ValueError):
    """sign(T) is undefined: a diagonal entry has a zero or non-finite real part."""

    def __init__(self, index: int):
        super().__init__("sign undefined at diagonal entry %d (1-based)" % index)
        self.index = index


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def _colmajor(a: np.ndarray, dtype) -> np.ndarray:
    return np.asfortranarray(np.asarray(a, dtype=dtype))


def sign_tri(T: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """U = sign(T) for a square upper-triangular T (real -> float64, complex -> complex128).

    Only the upper triangle of T is read; U's strict lower triangle is zero.
    Raises DomainError if some Re(t_ii) is zero or a diagonal entry is not finite.
    """
    T = np.asarray(T)
    if T.ndim != 2 or T.shape[0] != T.shape[1]:
        raise ValueError("T must be square")
    n = T.shape[0]
    lib = _load()
    if np.iscomplexobj(T):
        Tf = _colmajor(T, np.complex128)
        U = np.zeros((n, n), dtype=np.complex128, order="F")
        rc = lib.oracle_sign_tri_z(n, Tf.ctypes.data, max(n, 1), U.ctypes.data, max(n, 1), nthreads)
    else:
        Tf = _colmajor(T, np.float64)
        U = np.zeros((n, n), dtype=np.float64, order="F")
        rc = lib.oracle_sign_tri_d(n, Tf.ctypes.data, max(n, 1), U.ctypes.data, max(n, 1), nthreads)
    if rc > 0:
        raise DomainError(int(rc))
    if rc < 0:
        raise MemoryError("oracle could not allocate its work arrays")
    return U


def trsyl(A: np.ndarray, B: np.ndarray, C: np.ndarray) -> np.ndarray:
    """X with A X - X B = C, A and B upper triangular (upper triangles read)."""
    A, B, C = np.asarray(A), np.asarray(B), np.asarray(C)
    m, p = C.shape
    if A.shape != (m, m) or B.shape != (p, p):
        raise ValueError("shape mismatch")
    cplx = np.iscomplexobj(A) or np.iscomplexobj(B) or np.iscomplexobj(C)
    dt = np.complex128 if cplx else np.float64
    Af, Bf, Cf = _colmajor(A, dt), _colmajor(B, dt), _colmajor(C, dt)
    X = np.zeros((m, p), dtype=dt, order="F")
    lib = _load()
    f = lib.oracle_trsyl_z if cplx else lib.oracle_trsyl_d
    rc = f(m, p, Af.ctypes.data, max(m, 1), Bf.ctypes.data, max(p, 1),
           Cf.ctypes.data, max(m, 1), X.ctypes.data, max(m, 1))
    if rc != 0:
        raise ZeroDivisionError("singular Sylvester pivot at linear index %d" % (rc - 1))
    return X


def parlett(T: np.ndarray, fdiag) -> np.ndarray:
    """F = phi(T) by Parlett's recurrence (Algorithm 1) from phi's values on the
    diagonal, fdiag[i] = phi(t_ii); T upper triangular with distinct diagonal
    entries (only its upper triangle is read)."""
    T = np.asarray(T)
    if T.ndim != 2 or T.shape[0] != T.shape[1]:
        raise ValueError("T must be square")
    n = T.shape[0]
    fd = np.asarray(fdiag)
    if fd.shape != (n,):
        raise ValueError("fdiag must have one value per diagonal entry")
    cplx = np.iscomplexobj(T) or np.iscomplexobj(fd)
    dt = np.complex128 if cplx else np.float64
    Tf = _colmajor(T, dt)
    fdc = np.ascontiguousarray(fd, dtype=dt)
    F = np.zeros((n, n), dtype=dt, order="F")
    lib = _load()
    f = lib.oracle_parlett_z if cplx else lib.oracle_parlett_d
    rc = f(n, Tf.ctypes.data, max(n, 1), fdc.ctypes.data, F.ctypes.data, max(n, 1))
    if rc != 0:
        raise ZeroDivisionError("repeated diagonal entries at linear index %d" % (rc - 1))
    return F
