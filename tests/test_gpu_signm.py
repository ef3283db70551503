"""GPU parity of sign(A) for general matrices of small order (Section 1: Schur
form, triangular sign, back-transformation) through the C ABI, against the
CPU oracle (LAPACK's Schur form, the element oracle of Algorithm 3, two
products).  The two sides share no code; sign(A) is unique, so the results are
compared entry by entry although the two Schur forms differ.

Tolerance: both sides are backward stable (Householder and plane rotations,
then Algorithm 3), so they differ by about the sign function's condition at A
times the unit roundoff.  The matrices with eigenvalues kept at distance 0.5
from the imaginary axis (well conditioned) are held to 1e-11, the FP64 bar of
the triangular path; the paper's uniform test matrices, whose eigenvalues come
arbitrarily near that axis, to 1e-11 times the condition estimate
||S||_F^2 / n (at least 1) together with the defining invariants.
"""
import numpy as np
import pytest

from paper_1607_06303_amd import workloads as wl
from tests.conftest import rel_fro

pytestmark = pytest.mark.gpu

TOL = 1e-11


@pytest.fixture(scope="module")
def dev():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_06303_amd import signtri

    signtri.lib()
    return torch.device("cuda:0")


def to_dev(A, dev, ld=None):
    import torch

    n = A.shape[0]
    ld = ld or max(n, 1)
    buf = np.zeros((ld, n), dtype=A.dtype, order="F")
    buf[:n, :n] = A
    G = torch.from_numpy(np.ascontiguousarray(buf.T)).to(dev)
    return G.t()[:n, :n]


def run(As, dev, ld_pad=0, sentinel=None):
    import torch

    from paper_1607_06303_amd import signtri

    Ag = [to_dev(A, dev, A.shape[0] + ld_pad) for A in As]
    outs = []
    for A in As:
        n = A.shape[0]
        o = to_dev(np.full((n, n), np.nan if sentinel is None else sentinel, dtype=A.dtype), dev,
                   n + ld_pad)
        outs.append(o)
    print("signm batch: orders %s, dtype %s, pad %d" % ([A.shape[0] for A in As], As[0].dtype,
                                                        ld_pad), flush=True)
    try:
        Ss, codes = signtri.sign_general_batched(Ag, outs=outs)
        err = None
    except signtri.SignTriError as e:
        Ss, codes, err = outs, e.info.get("status"), e
    torch.cuda.synchronize()
    return [S.cpu().numpy() for S in Ss], codes, err


@pytest.mark.parametrize("cplx", [False, True])
def test_mixed_orders_match_the_oracle(dev, cplx):
    from oracle.signm import sign_general

    rng = np.random.default_rng(5100 + cplx)
    orders = [1, 2, 3, 7, 16, 31, 32, 33, 47, 64, 5, 64]
    As = [wl.general_A(n, rng, complex_=cplx) for n in orders]
    Ss, codes, err = run(As, dev)
    assert err is None and codes == [0] * len(As)
    for A, S in zip(As, Ss):
        ref = sign_general(A)
        assert S.dtype == ref.dtype
        assert rel_fro(S, ref) <= TOL, (A.shape, rel_fro(S, ref))


def test_padded_leading_dimensions_and_empty_entries(dev):
    from oracle.signm import sign_general

    rng = np.random.default_rng(5200)
    As = [wl.general_A(n, rng) for n in (20, 40)]
    Ss, codes, err = run(As, dev, ld_pad=5)
    assert err is None
    for A, S in zip(As, Ss):
        assert rel_fro(S, sign_general(A)) <= TOL

    import torch

    from paper_1607_06303_amd import signtri

    A = wl.general_A(9, rng)
    empty = torch.empty(0, 0, dtype=torch.float64, device=dev)
    Ss, codes = signtri.sign_general_batched([empty, to_dev(A, dev), empty])
    torch.cuda.synchronize()
    assert codes == [0, 0, 0] and Ss[0].shape == (0, 0)
    assert rel_fro(Ss[1].cpu().numpy(), sign_general(A)) <= TOL


@pytest.mark.parametrize("n", [48, 64])
def test_paper_recipe_matrices(dev, n):
    from oracle.signm import sign_general

    rng = np.random.default_rng(5300 + n)
    As = [wl.uniform_A(n, rng) for _ in range(3)]
    Ss, codes, err = run(As, dev)
    assert err is None
    for A, S in zip(As, Ss):
        ref = sign_general(A)
        kappa = max(1.0, np.linalg.norm(ref) ** 2 / n)
        assert rel_fro(S, ref) <= TOL * kappa, (rel_fro(S, ref), kappa)
        assert np.linalg.norm(S @ S - np.eye(n)) <= 1e-9 * kappa * n
        assert np.linalg.norm(S @ A - A @ S) <= 1e-9 * kappa * np.linalg.norm(A) * n


def test_imaginary_eigenvalues_leave_the_output_untouched(dev):
    from oracle.signm import sign_general

    from paper_1607_06303_amd import signtri

    rng = np.random.default_rng(5400)
    good = wl.general_A(12, rng)
    rot = np.array([[0.0, 2.0], [-2.0, 0.0]])  # eigenvalues +-2i
    Ss, codes, err = run([good, rot, good], dev, sentinel=7.0)
    assert isinstance(err, signtri.SignTriError) and err.code == 1
    assert codes == [0, 1, 0]
    assert np.all(Ss[1] == 7.0)
    assert rel_fro(Ss[0], sign_general(good)) <= TOL
    assert rel_fro(Ss[2], sign_general(good)) <= TOL


def test_not_converged_is_reported_and_leaves_the_output(dev, monkeypatch):
    # the library's testing hook limits the QR iteration to one sweep per matrix:
    # an order-16 matrix needs more, an order-1 matrix none
    from oracle.signm import sign_general

    from paper_1607_06303_amd import signtri

    rng = np.random.default_rng(5500)
    A = wl.general_A(16, rng)
    one = np.array([[-0.5]])
    monkeypatch.setenv("SIGNTRI_DEBUG_SIGNM_SWEEPS", "1")
    Ss, codes, err = run([A, one], dev, sentinel=3.0)
    assert isinstance(err, signtri.SignTriError) and err.code == 4
    assert codes == [4, 0]
    assert np.all(Ss[0] == 3.0) and Ss[1].tolist() == [[-1.0]]
    monkeypatch.delenv("SIGNTRI_DEBUG_SIGNM_SWEEPS")
    Ss, codes, err = run([A], dev)
    assert err is None and rel_fro(Ss[0], sign_general(A)) <= TOL


@pytest.mark.parametrize("cplx", [False, True])
def test_power_of_two_scaling_passes_through_exactly(dev, cplx):
    # sign(c A) = sign(A) for c > 0; the kernel scales A by a power of two to
    # [1, 2) first, so 2^600 A and 2^-600 A run the same arithmetic as A
    from oracle.signm import sign_general

    rng = np.random.default_rng(5600 + cplx)
    A = wl.general_A(40, rng, complex_=cplx)
    Ss, codes, err = run([A, A * 2.0 ** 600, A * 2.0 ** -600], dev)
    assert err is None
    assert np.array_equal(Ss[0], Ss[1]) and np.array_equal(Ss[0], Ss[2])
    assert rel_fro(Ss[0], sign_general(A)) <= TOL
