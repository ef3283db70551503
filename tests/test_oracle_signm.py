"""Pins of the general-matrix oracle sign(A) = Q sign(T) Q* (Section 1) against
results fixed independently of it: 2 x 2 matrices with A^2 a multiple of I
(sign(A) = A / sqrt of that multiple, worked by hand), matrices built from a
known eigendecomposition (sign(A) = X sign(D) X^-1), the Newton iteration
X <- (X + X^-1) / 2 (another algorithm converging to sign(A)), the defining
invariants, the triangular special case and the undefined case.  A transposed
instead of conjugated Q, a dropped product or a real part taken of a complex
result fails the complex pins."""
import numpy as np
import pytest

import oracle
from oracle.signm import sign_general
from paper_1607_06303_amd import workloads as wl
from tests.conftest import rel_fro


def newton_sign(A, iters=60):
    X = np.array(A, dtype=np.complex128 if np.iscomplexobj(A) else np.float64)
    for _ in range(iters):
        Xn = 0.5 * (X + np.linalg.inv(X))
        if np.linalg.norm(Xn - X) <= 1e-15 * np.linalg.norm(Xn):
            return Xn
        X = Xn
    return X


def test_two_by_two_by_hand():
    # A^2 = 7 I: sign(A) = A / sqrt(7)
    A = np.array([[1.0, 2.0], [3.0, -1.0]])
    assert rel_fro(sign_general(A), A / np.sqrt(7.0)) <= 1e-15
    # complex: A^2 = (6 + 2i) I, sign(A) = A / sqrt(6 + 2i) (principal root)
    B = np.array([[1 + 1j, 2.0], [3.0, -1 - 1j]])
    assert np.allclose(B @ B, (6 + 2j) * np.eye(2), atol=1e-15)
    assert rel_fro(sign_general(B), B / np.sqrt(6 + 2j)) <= 1e-15


@pytest.mark.parametrize("cplx", [False, True])
def test_known_eigendecomposition(cplx):
    rng = np.random.default_rng(91)
    n = 24
    d = rng.uniform(0.5, 2.0, n) * rng.choice([-1.0, 1.0], n)
    if cplx:
        d = d + 1j * rng.uniform(-1.0, 1.0, n)
    X = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    if cplx:
        X = X + 0.3j * rng.standard_normal((n, n)) / np.sqrt(n)
    Xi = np.linalg.inv(X)
    A = X @ np.diag(d) @ Xi
    ref = X @ np.diag(np.sign(d.real)) @ Xi
    if not cplx:
        A, ref = A.real, ref.real
    assert rel_fro(sign_general(A), ref) <= 1e-12


@pytest.mark.parametrize("cplx", [False, True])
def test_matches_newton_iteration(cplx):
    rng = np.random.default_rng(92)
    for n in (5, 17, 40):
        A = wl.general_A(n, rng, complex_=cplx)
        S = sign_general(A)
        assert rel_fro(S, newton_sign(A)) <= 1e-12, n
        assert S.dtype == (np.complex128 if cplx else np.float64)


def test_invariants_on_the_paper_recipe():
    rng = np.random.default_rng(93)
    A = wl.uniform_A(48, rng)
    S = sign_general(A)
    n = A.shape[0]
    assert np.linalg.norm(S @ S - np.eye(n)) <= 1e-8 * np.linalg.norm(S) ** 2
    assert np.linalg.norm(S @ A - A @ S) <= 1e-8 * np.linalg.norm(S) * np.linalg.norm(A)
    # the trace of sign(A) counts eigenvalues by the sign of their real parts
    ev = np.linalg.eigvals(A)
    assert round(np.trace(S).real) == int(np.sum(ev.real > 0) - np.sum(ev.real < 0))


def test_triangular_input_reduces_to_sign_tri():
    rng = np.random.default_rng(94)
    T = wl.make_T(30, rng)
    assert rel_fro(sign_general(T), oracle.sign_tri(T)) <= 1e-13


def test_imaginary_eigenvalues_are_rejected():
    with pytest.raises(oracle.DomainError):
        sign_general(np.array([[0.0, 1.0], [-1.0, 0.0]]))


def test_order_one_and_zero():
    assert sign_general(np.array([[-3.0]])).tolist() == [[-1.0]]
    assert sign_general(np.zeros((0, 0))).shape == (0, 0)
