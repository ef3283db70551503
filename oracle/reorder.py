"""TEST INFRASTRUCTURE ONLY: the Parlett-Sylvester route for any diagonal inertia.

Section 3 (Arithmetic Efficiency) describes it in three steps, followed here in
that order, plainly and without blocking:

1. Schur reordering: adjacent diagonal entries of the upper-triangular T are
   swapped by plane rotations (the Bai-Demmel swap of two 1 x 1 blocks) until
   the entries of one sign all precede those of the other.  The order kept is
   the stable partition with the fewer swaps, k = min(k_pos_first, k_neg_first)
   of the Section 3 model; ties put the positive entries first.  T_r = Q* T Q
   stays upper triangular and Q accumulates the rotations.
2. The Sylvester equation for the off-diagonal block of the reordered matrix:
   with T_r = [[T11, T12], [0, T22]] and the sign of T11's entries s1, the sign
   of T_r is [[s1 I, X], [0, -s1 I]] where T11 X - X T22 = 2 s1 T12 (the
   sign-split case of Algorithm 2, whose diagonal blocks are s1 I and -s1 I).
3. The transformation back: sign(T) = Q sign(T_r) Q*.

The rotation for a swap of t_ii = a and t_{i+1,i+1} = c with coupling b: the
first column of the rotation is the eigenvector (b, c - a) of the 2 x 2 block
for the eigenvalue c, normalised; conjugating by it brings c to the top, a to
the bottom, keeps the block upper triangular, and the rotation is applied to
the whole rows i, i+1 and columns i, i+1 of T.  The diagonal entries are
swapped exactly and the new subdiagonal entry is set to zero, as a swap
routine does.

Nothing here is shared with the HIP library; ``trsyl`` is the oracle's own C
Sylvester solver.
"""
from __future__ import annotations

import numpy as np


def _rotation(a, b, c):
    """Unitary G whose first column is (b, c - a) / ||.||: G* [[a, b], [0, c]] G = [[c, *], [0, a]]."""
    x, y = b, c - a
    r = np.sqrt(abs(x) ** 2 + abs(y) ** 2)
    g1 = np.array([x, y]) / r
    return np.array([[g1[0], -np.conj(g1[1])], [g1[1], np.conj(g1[0])]])


def swap_adjacent(T: np.ndarray, Q: np.ndarray, i: int) -> None:
    """Swap the diagonal entries i and i+1 of the upper-triangular T in place, and
    accumulate the rotation into Q (T <- G* T G on rows/columns i, i+1; Q <- Q G)."""
    a, b, c = T[i, i], T[i, i + 1], T[i + 1, i + 1]
    G = _rotation(a, b, c)
    T[:, i:i + 2] = T[:, i:i + 2] @ G
    T[i:i + 2, :] = G.conj().T @ T[i:i + 2, :]
    T[i, i], T[i + 1, i + 1] = c, a
    T[i + 1, i] = 0
    Q[:, i:i + 2] = Q[:, i:i + 2] @ G


def reorder_by_sign(T: np.ndarray, first: int):
    """Stable partition of the diagonal by the sign of its real parts, entries of
    sign ``first`` (+1 or -1) first, by adjacent swaps.  Returns (T_r, Q, k)."""
    T = np.array(np.triu(T), dtype=np.result_type(T.dtype, np.float64), copy=True)
    n = T.shape[0]
    Q = np.eye(n, dtype=T.dtype)
    k = 0
    placed = 0  # entries of the first sign already at the front
    for j in range(n):
        if np.sign(T[j, j].real) == first:
            # bubble entry j up past the entries of the other sign before it
            for i in range(j - 1, placed - 1, -1):
                swap_adjacent(T, Q, i)
                k += 1
            placed += 1
    return T, Q, k


def swap_counts(T: np.ndarray):
    """(swaps with positives first, swaps with negatives first): the inversion counts."""
    s = np.sign(np.diag(T).real)
    pos_first = neg_first = 0
    neg_seen = pos_seen = 0
    for v in s:
        if v > 0:
            pos_first += neg_seen
            pos_seen += 1
        else:
            neg_first += pos_seen
            neg_seen += 1
    return pos_first, neg_first


def sign_tri_reordered(T: np.ndarray, trsyl=None):
    """sign(T) by reordering, the sign-split Sylvester equation and the transformation
    back.  Returns (U, info) with info = {"k", "first", "split"}."""
    if trsyl is None:
        from . import trsyl
    T = np.asarray(T)
    n = T.shape[0]
    d = np.diag(T).real
    if n == 0:
        return np.zeros((0, 0), dtype=T.dtype), {"k": 0, "first": 1, "split": 0}
    if np.all(d > 0) or np.all(d < 0):
        s = 1.0 if d[0] > 0 else -1.0
        return s * np.eye(n, dtype=np.result_type(T.dtype, np.float64)), {"k": 0, "first": int(s), "split": n}
    kp, kn = swap_counts(T)
    first = 1 if kp <= kn else -1
    Tr, Q, k = reorder_by_sign(T, first)
    split = int(np.sum(np.sign(d) == first))
    T11, T12, T22 = Tr[:split, :split], Tr[:split, split:], Tr[split:, split:]
    X = trsyl(T11, T22, 2.0 * first * T12)
    Ur = np.zeros_like(Tr)
    Ur[:split, :split] = first * np.eye(split)
    Ur[split:, split:] = -first * np.eye(n - split)
    Ur[:split, split:] = X
    U = Q @ Ur @ Q.conj().T
    return np.triu(U), {"k": k, "first": first, "split": split}
