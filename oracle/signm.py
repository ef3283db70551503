"""TEST INFRASTRUCTURE ONLY: CPU oracle for sign(A) of a general square A.

Section 1 of Stotland, Schwartz and Toledo computes the sign of a general
matrix from a complex Schur decomposition A = Q T Q* (the first step of
Algorithm 3), U = sign(T) of the triangular factor, and sign(A) = Q U Q*.  This
module takes those three steps in that order: the Schur decomposition is
LAPACK's (through scipy, a library routine serving as a step), U comes from the
package's element-by-element oracle of Algorithm 3, and the two products are
plain matrix products.  A real A returns the real part of the result (the sign
of a real matrix is real).  Nothing here is shared with the HIP path.
"""
from __future__ import annotations

import numpy as np


def sign_general(A: np.ndarray) -> np.ndarray:
    """sign(A) = Q sign(T) Q* for square A (real -> float64, complex -> complex128).

    Raises the package's DomainError when an eigenvalue has a zero real part
    (sign(T) undefined at that diagonal entry of the Schur form)."""
    import scipy.linalg

    from . import sign_tri

    A = np.asarray(A)
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be square")
    n = A.shape[0]
    if n == 0:
        return np.zeros((0, 0), dtype=A.dtype)
    T, Q = scipy.linalg.schur(A.astype(np.complex128), output="complex")
    U = sign_tri(np.triu(T))
    S = Q @ U @ Q.conj().T
    return S.real.copy() if not np.iscomplexobj(A) else S
