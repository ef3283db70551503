"""Pins for the CPU oracle against facts that do not come from the oracle.

Each check would fail for a plausible mistake in the oracle (a dropped t_ij
term, a wrong sign in Eq. (1), a wrong k range, a transposed operand, a wrong
branch choice):

* hand-derived closed forms (tests/golden/closed_forms.txt);
* special cases: diagonal T, all signs equal, sign-split T against the LAPACK
  Sylvester solver (scipy.linalg.solve_sylvester);
* the defining properties U^2 = I and TU = UT, which with the diagonal fix U
  uniquely;
* the eigendecomposition definition Z sign(D) Z^-1 (Section 1) on tiny
  matrices with distinct eigenvalues;
* the Newton sign iteration and scipy.linalg.signm (independent algorithms);
* exact symmetries (negation, power-of-two scaling and diagonal similarity are
  bitwise; conjugation is bitwise; reversal-transpose to rounding);
* exact rational arithmetic on dyadic inputs bounds the oracle's rounding.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

from paper_1607_06303_amd import workloads as wl
from tests.conftest import rel_fro
from tests.golden import closed_forms

EPS = np.finfo(np.float64).eps


def _inv_err(T, U):
    n = T.shape[0]
    nu = np.linalg.norm(U)
    e1 = np.linalg.norm(U @ U - np.eye(n)) / max(nu * nu, 1.0)
    e2 = np.linalg.norm(T @ U - U @ T) / max(np.linalg.norm(T) * nu, 1e-300)
    return e1, e2


@pytest.mark.parametrize("case", list(closed_forms()), ids=lambda c: c[0])
def test_closed_forms(oracle_mod, case):
    name, T, U_expected, exact = case
    U = oracle_mod.sign_tri(T)
    assert U.dtype == (np.complex128 if np.iscomplexobj(T) else np.float64)
    np.testing.assert_allclose(U, U_expected, rtol=4 * EPS, atol=4 * EPS)
    # entries that are exact binary fractions must come out bitwise
    for i in range(T.shape[0]):
        for j in range(T.shape[0]):
            v = exact[i][j]
            if isinstance(v, Fraction) and v.denominator & (v.denominator - 1) == 0:
                assert U[i, j] == float(v), (name, i, j)


def test_diagonal_input_bitwise(oracle_mod):
    rng = np.random.default_rng(11)
    d = rng.uniform(0.5, 2, 40) * np.where(rng.random(40) < 0.5, 1, -1)
    U = oracle_mod.sign_tri(np.diag(d))
    assert np.array_equal(U, np.diag(np.sign(d)))


@pytest.mark.parametrize("sgn", [1.0, -1.0])
@pytest.mark.parametrize("cplx", [False, True])
def test_all_same_sign_is_pm_identity_bitwise(oracle_mod, sgn, cplx):
    rng = np.random.default_rng(12)
    T = wl.make_T(70, rng, complex_=cplx, signs=np.full(70, sgn))
    U = oracle_mod.sign_tri(T)
    assert np.array_equal(U, sgn * np.eye(70))


def test_lower_triangle_ignored_and_zeroed(oracle_mod):
    rng = np.random.default_rng(13)
    T = wl.make_T(30, rng)
    G = T + np.tril(rng.standard_normal((30, 30)), -1) * 1e3
    U1 = oracle_mod.sign_tri(T)
    U2 = oracle_mod.sign_tri(G)
    assert np.array_equal(U1, U2)
    assert not np.any(np.tril(U2, -1))


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_eigendecomposition_definition(oracle_mod, n, cplx):
    """sign(A) = Z diag(sign(d_ii)) Z^-1 (Section 1), distinct well-separated eigenvalues."""
    rng = np.random.default_rng(100 + n + 50 * cplx)
    # well-separated real parts: a shuffled grid +-(0.5 + k)
    re = (0.5 + np.arange(n)) * np.where(rng.random(n) < 0.5, 1, -1)
    re = rng.permutation(re)
    diag = re + (1j * rng.uniform(-1, 1, n) if cplx else 0)
    T = wl.assemble(np.asarray(diag), wl.upper_part(n, rng, cplx) * 0.7)
    w, Z = np.linalg.eig(T)
    ref = Z @ np.diag(np.sign(w.real)) @ np.linalg.inv(Z)
    if not cplx:
        ref = ref.real
    U = oracle_mod.sign_tri(T)
    assert rel_fro(U, ref) < 1e-12


@pytest.mark.parametrize("cplx", [False, True])
def test_invariants_random(oracle_mod, cplx):
    rng = np.random.default_rng(14)
    T = wl.make_T(300, rng, complex_=cplx)
    U = oracle_mod.sign_tri(T)
    e1, e2 = _inv_err(T, U)
    assert e1 < 300 * EPS and e2 < 300 * EPS


def test_invariants_near_imaginary(oracle_mod):
    rng = np.random.default_rng(15)
    T = wl.make_T(300, rng, complex_=True, re_range=(1e-3, 1.0), im_range=(-2, 2))
    U = oracle_mod.sign_tri(T)
    e1, e2 = _inv_err(T, U)
    assert e1 < 1e-12 and e2 < 1e-12


def test_repeated_diagonal_schur_recipe(oracle_mod):
    """Section 6's generator gives repeated values (conjugate pairs); Eq. (2) must
    avoid any division by t_ii - t_jj = 0 there."""
    rng = np.random.default_rng(16)
    T = wl.schur_like(80, None, rng)
    d = np.diag(T)
    assert len(np.unique(d)) < len(d)  # there are repeats
    U = oracle_mod.sign_tri(T)
    assert np.all(np.isfinite(U))
    e1, e2 = _inv_err(T, U)
    assert e1 < 1e-10 and e2 < 1e-10


def _newton_sign(T, iters=60):
    X = np.array(T, dtype=np.result_type(T.dtype, np.float64))
    for _ in range(iters):
        Xi = scipy.linalg.solve_triangular(X, np.eye(X.shape[0], dtype=X.dtype))
        # determinantal scaling (Higham) speeds convergence for near-imaginary spectra
        mu = float(np.exp(-np.mean(np.log(np.abs(np.diag(X))))))
        Xn = 0.5 * (mu * X + Xi / mu)
        if np.linalg.norm(Xn - X) <= 1e-15 * np.linalg.norm(Xn):
            X = Xn
            break
        X = Xn
    # a few unscaled steps to polish
    for _ in range(3):
        X = 0.5 * (X + scipy.linalg.solve_triangular(X, np.eye(X.shape[0], dtype=X.dtype)))
    return np.triu(X)


@pytest.mark.parametrize("kind", ["real", "complex", "near_imag"])
def test_newton_iteration(oracle_mod, kind):
    rng = np.random.default_rng(17)
    if kind == "real":
        T = wl.make_T(256, rng)
    elif kind == "complex":
        T = wl.make_T(256, rng, complex_=True)
    else:
        T = wl.make_T(256, rng, complex_=True, re_range=(1e-3, 1.0), im_range=(-2, 2))
    U = oracle_mod.sign_tri(T)
    assert rel_fro(U, _newton_sign(T)) < 1e-12


def test_scipy_signm_real_well_separated(oracle_mod):
    rng = np.random.default_rng(18)
    T = wl.make_T(128, rng)
    U = oracle_mod.sign_tri(T)
    assert rel_fro(U, scipy.linalg.signm(T)) < 1e-12


@pytest.mark.parametrize("cplx", [False, True])
def test_sign_split_matches_lapack_sylvester(oracle_mod, cplx):
    """Positives first: U = [[I, X], [0, -I]] with T11 X - X T22 = 2 T12 (Section 2)."""
    rng = np.random.default_rng(19)
    T = wl.sorted_positive_first(wl.make_T(96, rng, complex_=cplx))
    npos = int(np.sum(np.diag(T).real > 0))
    U = oracle_mod.sign_tri(T)
    assert np.array_equal(U[:npos, :npos], np.eye(npos))
    assert np.array_equal(U[npos:, npos:], -np.eye(96 - npos))
    T11, T12, T22 = T[:npos, :npos], T[:npos, npos:], T[npos:, npos:]
    X = scipy.linalg.solve_sylvester(T11, -T22, 2 * T12)
    assert rel_fro(U[:npos, npos:], X) < 1e-13
    # negatives first: U = [[-I, X], [0, I]] with right-hand side -2 T12
    d = np.diag(T).copy()
    S = np.array(T)
    order = np.concatenate([np.flatnonzero(d.real < 0), np.flatnonzero(d.real > 0)])
    S[np.arange(96), np.arange(96)] = d[order]
    nneg = 96 - npos
    U2 = oracle_mod.sign_tri(S)
    X2 = scipy.linalg.solve_sylvester(S[:nneg, :nneg], -S[nneg:, nneg:], -2 * S[:nneg, nneg:])
    assert np.array_equal(U2[:nneg, :nneg], -np.eye(nneg))
    assert rel_fro(U2[:nneg, nneg:], X2) < 1e-13


@pytest.mark.parametrize("cplx", [False, True])
def test_trsyl_matches_lapack(oracle_mod, cplx):
    rng = np.random.default_rng(20)
    A = wl.make_T(40, rng, complex_=cplx, signs=np.ones(40))
    B = wl.make_T(30, rng, complex_=cplx, signs=-np.ones(30))
    C = rng.standard_normal((40, 30)) + (1j * rng.standard_normal((40, 30)) if cplx else 0)
    X = oracle_mod.trsyl(A, B, C)
    assert rel_fro(X, scipy.linalg.solve_sylvester(A, -B, C)) < 1e-13


def test_symmetries_bitwise(oracle_mod):
    rng = np.random.default_rng(21)
    T = wl.make_T(120, rng)
    U = oracle_mod.sign_tri(T)
    # sign(-T) = -sign(T)
    assert np.array_equal(oracle_mod.sign_tri(-T), -U)
    # sign(2^m T) = sign(T)
    for m in (-3, 5):
        assert np.array_equal(oracle_mod.sign_tri(T * 2.0 ** m), U)
    # sign(D T D^-1) = D sign(T) D^-1 for a diagonal of powers of two
    e = rng.integers(-4, 5, 120)
    D = 2.0 ** e
    Ts = T * D[:, None] / D[None, :]
    assert np.array_equal(oracle_mod.sign_tri(Ts), U * D[:, None] / D[None, :])


def test_conjugation_bitwise(oracle_mod):
    rng = np.random.default_rng(22)
    T = wl.make_T(90, rng, complex_=True)
    assert np.array_equal(oracle_mod.sign_tri(np.conj(T)), np.conj(oracle_mod.sign_tri(T)))


def test_reversal_transpose(oracle_mod):
    """J T^T J is upper triangular and sign(J T^T J) = J sign(T)^T J."""
    rng = np.random.default_rng(23)
    T = wl.make_T(150, rng, complex_=True)
    R = T.T[::-1, ::-1]
    U = oracle_mod.sign_tri(T)
    assert rel_fro(oracle_mod.sign_tri(R), U.T[::-1, ::-1]) < 1e-14


def _exact_sign(Tq, s):
    n = len(s)
    U = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        U[i][i] = Fraction(s[i])
    for j in range(1, n):
        for i in range(j - 1, -1, -1):
            if s[i] + s[j] == 0:
                acc = Tq[i][j] * (s[i] - s[j])
                for k in range(i + 1, j):
                    acc += U[i][k] * Tq[k][j] - Tq[i][k] * U[k][j]
                U[i][j] = acc / (Tq[i][i] - Tq[j][j])
            else:
                acc = Fraction(0)
                for k in range(i + 1, j):
                    acc += U[i][k] * U[k][j]
                U[i][j] = -acc / (s[i] + s[j])
    return U


def test_exact_rational_rounding_bound(oracle_mod):
    """Dyadic T: the exact result bounds the oracle's FP64 rounding error."""
    rng = np.random.default_rng(24)
    n = 18
    T = np.triu(np.round(rng.standard_normal((n, n)) * 64) / 64, 1)
    d = (rng.integers(32, 128, n) / 64.0) * np.where(rng.random(n) < 0.5, 1, -1)
    T[np.arange(n), np.arange(n)] = d
    s = [1 if x > 0 else -1 for x in d]
    Tq = [[Fraction(float(T[i, j])) for j in range(n)] for i in range(n)]
    Ue = _exact_sign(Tq, s)
    U = oracle_mod.sign_tri(T)
    Uef = np.array([[float(Ue[i][j]) for j in range(n)] for i in range(n)])
    err = np.linalg.norm(U - Uef) / np.linalg.norm(Uef)
    assert err < 50 * EPS


def test_domain_errors(oracle_mod):
    T = np.triu(np.ones((5, 5)))
    T[2, 2] = 0.0
    with pytest.raises(oracle_mod.DomainError) as ei:
        oracle_mod.sign_tri(T)
    assert ei.value.index == 3
    T[2, 2] = np.nan
    with pytest.raises(oracle_mod.DomainError):
        oracle_mod.sign_tri(T)
    Tc = np.triu(np.ones((4, 4))).astype(complex)
    Tc[3, 3] = 2j  # purely imaginary
    with pytest.raises(oracle_mod.DomainError) as ei:
        oracle_mod.sign_tri(Tc)
    assert ei.value.index == 4


def test_empty_and_one(oracle_mod):
    assert oracle_mod.sign_tri(np.zeros((0, 0))).shape == (0, 0)
    assert oracle_mod.sign_tri(np.array([[-3.0]]))[0, 0] == -1.0
