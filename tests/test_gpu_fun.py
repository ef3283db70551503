"""GPU parity of the general-function entry point (Parlett's substitution,
Algorithm 1) against the Parlett oracle, through the C ABI: the square, the
exponential, the reciprocal, the square root and the sign, real and complex,
one block to several blocks with ragged tails; garbage below the diagonal and
padded leading dimensions; phi = sign against signtri()."""
import numpy as np
import pytest

import oracle
from tests.conftest import rel_fro
from tests.test_gpu_parity import TOL_FP64, dev, to_dev_colmajor  # noqa: F401
from tests.test_oracle_parlett import separated_T

pytestmark = pytest.mark.gpu

FUNS = {
    "square": lambda d: d ** 2,
    "exp": np.exp,
    "recip": lambda d: 1.0 / d,
    "sqrt": lambda d: np.sqrt(d.astype(np.complex128)),
    "sign": lambda d: np.sign(d.real).astype(d.dtype),
}


def run_fun(T, fd, dev, ld=None):
    import torch

    from paper_1607_06303_amd import signtri

    Tg = to_dev_colmajor(T, dev, ld=ld)
    fdg = torch.from_numpy(np.ascontiguousarray(fd)).to(dev)
    F, info = signtri.fun_tri(Tg, fdg)
    torch.cuda.synchronize()
    return F.cpu().numpy(), info


@pytest.mark.parametrize("n", [1, 2, 31, 33, 100, 257, 600])
@pytest.mark.parametrize("fname", ["square", "exp", "recip", "sign"])
def test_fun_real_matches_oracle(dev, n, fname):
    T = separated_T(n, np.random.default_rng(100 + n))
    fd = FUNS[fname](np.diag(T))
    F, info = run_fun(T, fd, dev)
    assert info["path_name"] == "ph"
    ref = oracle.parlett(T, fd)
    assert rel_fro(F, ref) <= TOL_FP64, (n, fname)
    assert not np.any(np.tril(F, -1))


@pytest.mark.parametrize("n", [2, 33, 200])
@pytest.mark.parametrize("fname", ["square", "exp", "sqrt"])
def test_fun_complex_matches_oracle(dev, n, fname):
    T = separated_T(n, np.random.default_rng(200 + n), cplx=True)
    fd = FUNS[fname](np.diag(T)).astype(np.complex128)
    F, _ = run_fun(T, fd, dev)
    ref = oracle.parlett(T, fd)
    assert rel_fro(F, ref) <= TOL_FP64, (n, fname)


def test_fun_garbage_below_padding_and_known_results(dev):
    import scipy.linalg

    n = 130
    T = separated_T(n, np.random.default_rng(300))
    G = T + np.tril(np.full_like(T, 1e300), -1)
    F, _ = run_fun(G, np.diag(T) ** 2, dev, ld=n + 7)
    assert rel_fro(F, T @ T) <= 1e-13
    F, _ = run_fun(T, np.exp(np.diag(T)), dev)
    assert rel_fro(F, scipy.linalg.expm(T)) <= 1e-12


def test_fun_sign_matches_signtri(dev):
    from tests.test_gpu_parity import run_gpu

    T = separated_T(300, np.random.default_rng(400))
    F, _ = run_fun(T, np.sign(np.diag(T)), dev)
    U, _ = run_gpu(T, dev, algo="ph")
    assert rel_fro(F, U) <= TOL_FP64


def test_fun_empty(dev):
    import torch

    from paper_1607_06303_amd import signtri

    T = torch.empty((0, 0), dtype=torch.float64, device=dev)
    F, _ = signtri.fun_tri(T, torch.empty((0,), dtype=torch.float64, device=dev))
    assert F.shape == (0, 0)
