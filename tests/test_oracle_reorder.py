"""Pins of the oracle's Parlett-Sylvester route for any inertia (Section 3:
Schur reordering by adjacent swaps, the sign-split Sylvester equation, the
transformation back).

It is pinned to things outside itself:
* the element-by-element Parlett-Higham oracle (Algorithm 3, a different
  algorithm in C) on real, complex, near-imaginary and repeated-eigenvalue
  inputs;
* the eigendecomposition definition V sign(D) V^-1 on tiny inputs;
* the properties a reordering must have: T_r upper triangular with the
  stable-partitioned diagonal, Q unitary, Q T_r Q* = T, and exactly the number
  of swaps that the Section 3 model counts (the inversion count).
Planted mistakes in a copy of the module must fail those pins.
"""
import os
import types

import numpy as np
import pytest

from paper_1607_06303_amd import workloads as wl
from tests.conftest import rel_fro

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "reorder.py")


def _reorder_mod():
    from oracle import reorder

    return reorder


def cases():
    out = []
    rng = wl.rng_for(3, salt=7)
    out.append(("skewed_real", wl.make_T(160, rng, signs=wl.signs_with_negatives(160, 6, rng))))
    out.append(("interleaved_real", wl.make_T(90, wl.rng_for(1, salt=7))))
    out.append(("positive_minority", wl.make_T(120, rng, signs=-wl.signs_with_negatives(120, 5, rng))))
    s = np.ones(70)
    s[[0, 1, 35, 68, 69]] = -1
    out.append(("ends_and_runs", wl.make_T(70, rng, signs=s)))
    out.append(("complex", wl.make_T(80, wl.rng_for(2, salt=7), complex_=True)))
    out.append(("near_imaginary", wl.make_T(80, wl.rng_for(5, salt=7), complex_=True,
                                             re_range=(1e-3, 1.0), im_range=(-2.0, 2.0))))
    out.append(("schur_recipe", wl.schur_like(60, 4, wl.rng_for(9, salt=7))))
    return out


CASES = cases()


@pytest.mark.parametrize("name,T", CASES, ids=[c[0] for c in CASES])
def test_matches_parlett_higham(oracle_mod, name, T):
    ro = _reorder_mod()
    U, info = ro.sign_tri_reordered(T)
    ref = oracle_mod.sign_tri(T)
    assert rel_fro(U, ref) <= 1e-12, (name, info)


@pytest.mark.parametrize("n,cplx", [(5, False), (7, True), (8, False)])
def test_eigendecomposition_definition(n, cplx):
    ro = _reorder_mod()
    rng = np.random.default_rng(100 + n)
    for _ in range(5):
        d = rng.uniform(0.5, 2.0, n) * np.where(rng.random(n) < 0.5, 1, -1)
        if cplx:
            d = d + 1j * rng.uniform(-1, 1, n)
        T = np.triu(rng.standard_normal((n, n)) / np.sqrt(n), 1).astype(d.dtype) + np.diag(d)
        w, V = np.linalg.eig(T)
        ref = V @ np.diag(np.sign(w.real)) @ np.linalg.inv(V)
        U, _ = ro.sign_tri_reordered(T)
        assert rel_fro(U, ref) <= 1e-12


@pytest.mark.parametrize("name,T", CASES, ids=[c[0] for c in CASES])
def test_reordering_properties(oracle_mod, name, T):
    ro = _reorder_mod()
    kp, kn = ro.swap_counts(T)
    first = 1 if kp <= kn else -1
    Tr, Q, k = ro.reorder_by_sign(T, first)
    n = T.shape[0]
    d = np.diag(T)
    order = np.concatenate([np.flatnonzero(np.sign(d.real) == first),
                            np.flatnonzero(np.sign(d.real) != first)])
    assert k == min(kp, kn)
    assert np.array_equal(np.diag(Tr), d[order])            # swapped exactly
    assert not np.any(np.tril(Tr, -1))                       # still upper triangular
    assert np.linalg.norm(Q.conj().T @ Q - np.eye(n)) <= 1e-13 * n
    back = Q @ Tr @ Q.conj().T
    assert rel_fro(back, np.triu(T)) <= 1e-13


def test_swap_counts_match_work_model(oracle_mod):
    ro = _reorder_mod()
    for name, T in CASES:
        s = [1 if v > 0 else -1 for v in np.diag(T).real]
        assert ro.swap_counts(T) == tuple(oracle_mod.workmodel.swaps(s)), name


def test_grouped_needs_no_swap(oracle_mod):
    ro = _reorder_mod()
    T = wl.sorted_positive_first(wl.make_T(50, wl.rng_for(2, salt=8), complex_=True))
    U, info = ro.sign_tri_reordered(T)
    assert info["k"] == 0 and info["split"] == int(np.sum(np.diag(T).real > 0))
    assert rel_fro(U, oracle_mod.sign_tri(T)) <= 1e-12


def test_trivial_inertia(oracle_mod):
    ro = _reorder_mod()
    T = wl.make_T(20, wl.rng_for(1, salt=9), signs=-np.ones(20))
    U, info = ro.sign_tri_reordered(T)
    assert np.array_equal(U, -np.eye(20)) and info["k"] == 0


MUTATIONS = {
    "rotation_column_sign": ("x, y = b, c - a", "x, y = b, a - c"),
    "no_column_rotation": ("    T[:, i:i + 2] = T[:, i:i + 2] @ G\n", ""),
    "no_schur_vectors": ("    Q[:, i:i + 2] = Q[:, i:i + 2] @ G\n", ""),
    "sylvester_rhs_sign": ("X = trsyl(T11, T22, 2.0 * first * T12)", "X = trsyl(T11, T22, -2.0 * first * T12)"),
    "sylvester_rhs_factor": ("X = trsyl(T11, T22, 2.0 * first * T12)", "X = trsyl(T11, T22, first * T12)"),
    "blocks_swapped": ("Ur[:split, :split] = first * np.eye(split)", "Ur[:split, :split] = -first * np.eye(split)"),
    "no_conjugate_back": ("U = Q @ Ur @ Q.conj().T", "U = Q @ Ur @ Q.T"),
    "unstable_partition_stop": ("for i in range(j - 1, placed - 1, -1):", "for i in range(j - 1, placed, -1):"),
}


def _mutant(name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    mod = types.ModuleType("reorder_mutant_" + name)
    exec(compile(src.replace(old, new), SRC + ":" + name, "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_planted_mistakes(oracle_mod, name):
    mod = _mutant(name)
    caught = False
    for cname, T in CASES:
        try:
            U, _ = mod.sign_tri_reordered(T, trsyl=oracle_mod.trsyl)
        except Exception:
            caught = True
            break
        if not np.all(np.isfinite(U)) or rel_fro(U, oracle_mod.sign_tri(T)) > 1e-12:
            caught = True
            break
    assert caught, name
