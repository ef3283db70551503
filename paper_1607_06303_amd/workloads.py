"""Seeded synthetic inputs: upper-triangular T with a prescribed diagonal inertia.

This module only draws random numbers; it holds none of the sign method's
arithmetic, and both the HIP path's tests and the CPU oracle's tests take
their inputs from it.

Every matrix has a zero strict lower triangle, a strict upper triangle of
N(0, 1)/sqrt(n) entries (complex: (a + ib)/sqrt(2) with a, b ~ N(0, 1), so
unit variance, then /sqrt(n)), and a diagonal whose real parts have random
magnitudes and a chosen sign pattern.  The paper's experiments (Section 6)
use random triangular matrices with a prescribed inertia; ``schur_like`` also
reproduces its own recipe (real part of the complex Schur form of a random
square matrix with U[-50, 50] entries, signs forced positive except at k
random positions), which has repeated diagonal values from conjugate pairs.

Draw order for a fixed generator: signs, |Re| magnitudes, imaginary parts of
the diagonal, then the strict upper triangle, real part before imaginary part.

Named workloads (seed 1607063030 + c for workload c):

1. real n=512, diagonal +-U[0.5, 2], each sign + with p = 0.5;
2. complex n=4096, Re +-U[0.5, 2] (p = 0.5), Im U[-1, 1]; variant "sorted"
   stable-partitions the same diagonal so positives come first (a sign-split
   T for the Parlett-Sylvester form), with the same strict upper part;
3. real n=8192, n-64 entries +U[0.5, 2], 64 entries -U[0.5, 2] at distinct
   random positions;
4. a batch of 2000 real matrices, n log-uniform in [32, 1024] (rounded to an
   integer), per-matrix positive fraction f ~ U[0, 1], each sign Bernoulli(f);
5. complex n=16384, Re +-U[1e-3, 1] (p = 0.5), Im U[-2, 2] (near-imaginary).
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 1607063030


def rng_for(config: int, salt: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + config + 1000 * salt)


def upper_part(n: int, rng: np.random.Generator, complex_: bool) -> np.ndarray:
    """Strict upper triangle with N(0,1)/sqrt(n) entries (unit-variance complex)."""
    scale = 1.0 / np.sqrt(max(n, 1))
    re = np.triu(rng.standard_normal((n, n)), 1)
    if not complex_:
        return re * scale
    im = np.triu(rng.standard_normal((n, n)), 1)
    return (re + 1j * im) * (scale / np.sqrt(2.0))


def assemble(diag: np.ndarray, upper: np.ndarray) -> np.ndarray:
    n = diag.shape[0]
    T = np.array(upper, dtype=np.result_type(diag.dtype, upper.dtype), order="F", copy=True)
    T[np.arange(n), np.arange(n)] = diag
    return T


def random_signs(n: int, rng: np.random.Generator, p_pos: float = 0.5) -> np.ndarray:
    return np.where(rng.random(n) < p_pos, 1.0, -1.0)


def signs_with_negatives(n: int, n_neg: int, rng: np.random.Generator) -> np.ndarray:
    s = np.ones(n)
    if n_neg > 0:
        s[rng.choice(n, size=n_neg, replace=False)] = -1.0
    return s


def make_T(n: int, rng: np.random.Generator, *, complex_: bool = False,
           signs: np.ndarray | None = None, p_pos: float = 0.5,
           re_range=(0.5, 2.0), im_range=(-1.0, 1.0)) -> np.ndarray:
    """Upper-triangular T with diagonal real parts signs * U[re_range]."""
    if signs is None:
        signs = random_signs(n, rng, p_pos)
    mag = rng.uniform(re_range[0], re_range[1], n)
    diag = signs * mag
    if complex_:
        diag = diag + 1j * rng.uniform(im_range[0], im_range[1], n)
    return assemble(diag, upper_part(n, rng, complex_))


def sorted_positive_first(T: np.ndarray) -> np.ndarray:
    """Same diagonal values, stably partitioned so positive real parts come first;
    the strict upper triangle is kept as is (a sign-split T)."""
    d = np.diag(T).copy()
    order = np.concatenate([np.flatnonzero(d.real > 0), np.flatnonzero(d.real < 0)])
    S = np.array(T, order="F", copy=True)
    n = T.shape[0]
    S[np.arange(n), np.arange(n)] = d[order]
    return S


def workload1(n: int = 512) -> np.ndarray:
    return make_T(n, rng_for(1))


def workload2(n: int = 4096, sorted_: bool = False) -> np.ndarray:
    T = make_T(n, rng_for(2), complex_=True, im_range=(-1.0, 1.0))
    return sorted_positive_first(T) if sorted_ else T


def workload3(n: int = 8192, n_neg: int = 64) -> np.ndarray:
    rng = rng_for(3)
    return make_T(n, rng, signs=signs_with_negatives(n, n_neg, rng))


def workload4_sizes(count: int = 2000, lo: int = 32, hi: int = 1024) -> np.ndarray:
    rng = rng_for(4)
    return np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), count))).astype(np.int64)


def workload4(count: int = 2000, lo: int = 32, hi: int = 1024):
    """List of real matrices; matrix b uses its own child generator."""
    sizes = workload4_sizes(count, lo, hi)
    children = np.random.SeedSequence(SEED_BASE + 4).spawn(count)
    out = []
    for n, ss in zip(sizes, children):
        rng = np.random.default_rng(ss)
        f = rng.random()
        out.append(make_T(int(n), rng, p_pos=f))
    return out


def workload5(n: int = 16384) -> np.ndarray:
    return make_T(n, rng_for(5), complex_=True, re_range=(1e-3, 1.0), im_range=(-2.0, 2.0))


def schur_like(n: int, n_neg: int | None, rng: np.random.Generator) -> np.ndarray:
    """The paper's recipe: real part of the complex Schur form of a random real
    matrix with U[-50, 50] entries; optionally force all but n_neg random
    diagonal signs positive (keeping |t_ii|).  Conjugate eigenvalue pairs give
    repeated diagonal values."""
    import scipy.linalg

    A = rng.uniform(-50.0, 50.0, (n, n))
    Tc, _ = scipy.linalg.schur(A.astype(np.complex128), output="complex")
    T = np.triu(Tc.real)
    # conjugate pairs agree only to rounding after the Schur form; rounding the
    # diagonal to 1e-8 makes them exact repeats, which is the case to exercise
    T[np.arange(n), np.arange(n)] = np.round(np.diag(T), 8)
    if n_neg is not None:
        d = np.abs(np.diag(T))
        s = signs_with_negatives(n, n_neg, rng)
        T[np.arange(n), np.arange(n)] = s * d
    return np.asfortranarray(T)


def general_A(n: int, rng: np.random.Generator, *, complex_: bool = False, gap: float = 0.5,
              pairs: int | None = None, coupling: float = 0.3) -> np.ndarray:
    """A general square matrix with known, well separated eigenvalues: A = V B V*,
    V a random orthogonal (unitary) matrix, B block upper triangular with
    eigenvalues whose real parts lie in +-[gap, 2] (random signs) and coupling
    entries of size coupling / sqrt(n) above the diagonal blocks.  A real A gets
    `pairs` complex-conjugate pairs (2 x 2 blocks [[a, b], [-b, a]], eigenvalues
    a +- ib; default n // 4), the rest real eigenvalues; a complex A gets complex
    eigenvalues with imaginary parts in [-1, 1]."""
    dt = np.complex128 if complex_ else np.float64
    B = np.zeros((n, n), dtype=dt)
    re = rng.uniform(gap, 2.0, n) * rng.choice([-1.0, 1.0], n)
    if complex_:
        B[np.arange(n), np.arange(n)] = re + 1j * rng.uniform(-1.0, 1.0, n)
        step = np.ones(n, dtype=int)
    else:
        k = n // 4 if pairs is None else min(pairs, n // 2)
        i = 0
        for p in range(k):
            a, b = re[i], rng.uniform(0.2, 1.0)
            B[i:i + 2, i:i + 2] = [[a, b], [-b, a]]
            i += 2
        B[np.arange(i, n), np.arange(i, n)] = re[i:]
    upper = np.triu(rng.standard_normal((n, n)), 1)
    if complex_:
        upper = upper + 1j * np.triu(rng.standard_normal((n, n)), 1)
    # above the 2 x 2 blocks only: keep the block structure of B
    mask = np.triu(np.ones((n, n), dtype=bool), 1)
    if not complex_:
        for j in range(0, 2 * (n // 4 if pairs is None else min(pairs, n // 2)), 2):
            mask[j, j + 1] = False
    B = B + np.where(mask, upper, 0.0) * (coupling / np.sqrt(max(n, 1)))
    G = rng.standard_normal((n, n)) + (1j * rng.standard_normal((n, n)) if complex_ else 0.0)
    V, R = np.linalg.qr(G)
    V = V * (np.diag(R) / np.abs(np.diag(R)))  # a Haar-distributed factor
    return np.asfortranarray(V @ B @ V.conj().T)


def uniform_A(n: int, rng: np.random.Generator) -> np.ndarray:
    """The paper's test matrices before their Schur form: U[-50, 50] entries."""
    return np.asfortranarray(rng.uniform(-50.0, 50.0, (n, n)))
