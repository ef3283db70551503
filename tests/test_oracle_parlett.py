"""Pins of the general-function oracle (Parlett's recurrence, Algorithm 1) against
results fixed independently of it: a hand-worked 2 x 2 case, polynomial and
rational functions whose values are products and triangular solves, the
exponential by scipy's Pade-based expm, and the sign function by the sign
oracle (Algorithm 3) on a diagonal with distinct entries.  A wrong sign,
index or dropped term in the recurrence fails the polynomial or rational pins."""
import numpy as np
import pytest
import scipy.linalg

import oracle
from tests.conftest import rel_fro


def separated_T(n, rng, cplx=False, scale=0.3):
    """Upper triangular with distinct, well separated diagonal entries."""
    d = np.linspace(1.0, 3.0, n) * rng.choice([-1.0, 1.0], n)
    d = d[rng.permutation(n)]
    T = np.triu(rng.standard_normal((n, n)), 1) * scale / np.sqrt(n)
    if cplx:
        T = T + 1j * np.triu(rng.standard_normal((n, n)), 1) * scale / np.sqrt(n)
        d = d + 1j * rng.uniform(-1.0, 1.0, n)
    return T + np.diag(d)


def test_two_by_two_by_hand():
    # f(x) = x^2 on [[3, 5], [0, 1]]: f_12 = 5 (9 - 1) / (3 - 1) = 20 = 3*5 + 5*1
    T = np.array([[3.0, 5.0], [0.0, 1.0]])
    F = oracle.parlett(T, np.array([9.0, 1.0]))
    assert F.tolist() == [[9.0, 20.0], [0.0, 1.0]]


@pytest.mark.parametrize("cplx", [False, True])
def test_square_is_the_product(cplx):
    T = separated_T(60, np.random.default_rng(1), cplx)
    F = oracle.parlett(T, np.diag(T) ** 2)
    assert rel_fro(F, T @ T) <= 1e-13


@pytest.mark.parametrize("cplx", [False, True])
def test_reciprocal_is_the_inverse(cplx):
    T = separated_T(60, np.random.default_rng(2), cplx)
    F = oracle.parlett(T, 1.0 / np.diag(T))
    inv = scipy.linalg.solve_triangular(T, np.eye(60, dtype=T.dtype))
    assert rel_fro(F, inv) <= 1e-13


@pytest.mark.parametrize("cplx", [False, True])
def test_exponential_matches_pade(cplx):
    T = separated_T(40, np.random.default_rng(3), cplx)
    F = oracle.parlett(T, np.exp(np.diag(T)))
    assert rel_fro(F, scipy.linalg.expm(T)) <= 1e-12


def test_sign_matches_the_sign_oracle():
    T = separated_T(80, np.random.default_rng(4))
    F = oracle.parlett(T, np.sign(np.diag(T).real))
    assert rel_fro(F, oracle.sign_tri(T)) <= 1e-13


def test_identity_function_and_lower_triangle():
    T = separated_T(30, np.random.default_rng(5))
    G = T + np.tril(np.full_like(T, 7.0), -1)  # garbage below: not read
    F = oracle.parlett(G, np.diag(T))
    assert rel_fro(F, T) <= 1e-15 and not np.any(np.tril(F, -1))


def test_repeated_diagonal_entries_are_rejected():
    T = np.array([[2.0, 1.0], [0.0, 2.0]])
    with pytest.raises(ZeroDivisionError):
        oracle.parlett(T, np.array([4.0, 4.0]))
