"""Pins for the brute-force work models (Section 3) and for the input generators."""
import numpy as np
import pytest

from oracle import workmodel
from paper_1607_06303_amd import workloads as wl


def comb3(n):
    return n * (n - 1) * (n - 2) // 6


@pytest.mark.parametrize("n", [3, 10, 41])
def test_ph_work_extremes(n):
    # all signs equal: every pair takes Eq. (2), one inner product: 2 C(n,3) ~ n^3/3
    assert workmodel.ph_flops([1] * n) == 2 * comb3(n)
    assert workmodel.ph_flops([-1] * n, complex_=True) == 8 * comb3(n)
    # any pattern lies between n^3/3 and 2n^3/3 to leading order: 2C(n,3) .. 4C(n,3)
    rng = np.random.default_rng(n)
    s = list(np.where(rng.random(n) < 0.5, 1, -1))
    w = workmodel.ph_flops(s)
    assert 2 * comb3(n) <= w <= 4 * comb3(n)


def test_ps_work_bounds():
    # Section 3: n^2 - n <= n_- n_+ (n_- + n_+) <= n^3/4 with extremes n_- = 1 and n/2
    n = 20
    one_neg = [1] * (n - 1) + [-1]
    half = [1] * (n // 2) + [-1] * (n // 2)
    assert workmodel.ps_flops(one_neg) == n * n - n  # already grouped: no swaps
    assert workmodel.ps_flops(half) == n ** 3 // 4
    # swaps range from 0 to n^2/4 (reversed grouping of a balanced split)
    rev = [-1] * (n // 2) + [1] * (n // 2)
    assert workmodel.swaps(rev) == (n * n // 4, 0)
    assert workmodel.swaps(half) == (0, n * n // 4)


def test_hand_counted_small_cases():
    """Section 3 counts worked out by hand, term by term.

    [+, +, -]: pairs (0,1) and (1,2) have empty sums; pair (0,2) has one term
    (k = 1) and opposite signs, so Eq. (1) costs two multiply-adds: 4 flops.
    [+, -, +, -]: (0,2) and (1,3) have one term each with equal signs (Eq. (2),
    one multiply-add, 2 flops each); (0,3) has two terms with opposite signs
    (2 x 2 multiply-adds, 8 flops); the adjacent pairs have none: 12 flops.
    Swaps of [+, -, +, -]: positives first needs the pair (1,2) exchanged (1);
    negatives first needs (0,1), (0,3), (2,3) (3).  The Parlett-Sylvester
    estimate with k = 1: reordering 12 n k = 48, Sylvester n- n+ (n- + n+) =
    2 * 2 * 4 = 16, transformation back 12 n k = 48: 112.
    """
    assert workmodel.ph_flops([1, 1, -1]) == 4
    assert workmodel.ph_flops([1, 1, -1], complex_=True) == 16
    assert workmodel.ph_flops([1, -1, 1, -1]) == 12
    # [+, +, +, +]: terms (0,2): 1, (1,3): 1, (0,3): 2, C(4,3) = 4 in all, 2 flops each
    assert workmodel.ph_flops([1, 1, 1, 1]) == 8
    assert workmodel.swaps([1, -1, 1, -1]) == (1, 3)
    assert workmodel.swaps([-1, 1]) == (1, 0)
    assert workmodel.ps_flops([1, -1, 1, -1]) == 112
    assert workmodel.ps_flops([1, -1, 1, -1], complex_=True) == 448
    # [+, -, -]: positives first: nothing to move (0); negatives first: the +
    # passes both - (2).  k = 0, so no reordering term: Sylvester 2 * 1 * 3 = 6
    assert workmodel.swaps([1, -1, -1]) == (0, 2)
    assert workmodel.ps_flops([1, -1, -1]) == 6


def test_workloads_deterministic_and_shaped():
    a = wl.workload1(64)
    b = wl.workload1(64)
    assert np.array_equal(a, b)
    assert np.all(np.tril(a, -1) == 0)
    d = np.abs(np.diag(a))
    assert d.min() >= 0.5 and d.max() <= 2.0
    T3 = wl.workload3(512, n_neg=64)
    assert int(np.sum(np.diag(T3) < 0)) == 64
    T2 = wl.workload2(128)
    T2s = wl.workload2(128, sorted_=True)
    assert np.array_equal(np.triu(T2, 1), np.triu(T2s, 1))
    npos = int(np.sum(np.diag(T2s).real > 0))
    assert np.all(np.diag(T2s)[:npos].real > 0) and np.all(np.diag(T2s)[npos:].real < 0)
    assert np.array_equal(np.sort_complex(np.diag(T2)), np.sort_complex(np.diag(T2s)))


def test_workload4_sizes():
    sizes = wl.workload4_sizes()
    assert len(sizes) == 2000 and sizes.min() >= 32 and sizes.max() <= 1024
    mats = wl.workload4(count=5)
    assert [m.shape[0] for m in mats] == list(wl.workload4_sizes(count=5))
