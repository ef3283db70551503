"""TEST INFRASTRUCTURE ONLY: brute-force flop counts of Section 3 (Arithmetic Efficiency).

These loops count, pair by pair, the work models the paper states, so that the
library's O(n) planner can be checked against them on small inputs.

* Parlett-Higham (Algorithm 3): each pair i < j costs one inner product over
  k = i+1 .. j-1 when Eq. (2) is used (signs agree) and two when Eq. (1) is
  used (signs differ).  One real multiply-add is counted as 2 flops; a complex
  one as 8 (factor 4).  This is the n^3/3 .. 2n^3/3 range of Section 3.
* Parlett-Sylvester: k adjacent swaps to group the eigenvalues by sign (the
  fewer of the two target orders), 12 n k flops for the reordering including
  the Schur vectors, n_- n_+ (n_- + n_+) flops for the Sylvester equation, and
  the transformation back, which Section 3 leaves unquantified beyond "nothing
  when no swap was made, cubic at worst"; it is read here as applying the same
  rotations once more to the n x n sign matrix, 12 n k flops.
"""
from __future__ import annotations


def ph_flops(signs, complex_: bool = False) -> int:
    n = len(signs)
    total = 0
    for j in range(n):
        for i in range(j):
            terms = j - i - 1
            total += terms * (2 if signs[i] == signs[j] else 4)
    return total * (4 if complex_ else 1)


def swaps(signs) -> tuple[int, int]:
    """(swaps to put positives first, swaps to put negatives first)."""
    n = len(signs)
    pos_first = 0
    neg_first = 0
    for i in range(n):
        for j in range(i + 1, n):
            if signs[i] < 0 < signs[j]:
                pos_first += 1
            if signs[j] < 0 < signs[i]:
                neg_first += 1
    return pos_first, neg_first


def ps_flops(signs, complex_: bool = False) -> int:
    n = len(signs)
    npos = sum(1 for s in signs if s > 0)
    nneg = n - npos
    k = min(swaps(signs))
    reorder = 12 * n * k
    sylvester = nneg * npos * (nneg + npos)
    back = 12 * n * k
    return (reorder + sylvester + back) * (4 if complex_ else 1)
