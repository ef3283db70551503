"""The no-allocation entry point, signtri_noalloc(), against signtri(), the
entry point it is a variant of, through the C ABI.

Two calls in a row share the fixed scratch: the largest order first (real,
n = 8192 with 64 negatives: the projector form), then a smaller one (real,
interleaved: the dataflow sweep), then a complex one; each result must match
signtri()'s on the same input to the FP64 bar (and the oracle's).  An order
beyond the fixed scratch is rejected with SIGNTRI_ETOOBIG before any device
work, leaving U untouched.
"""
import numpy as np
import pytest

from paper_1607_06303_amd import workloads as wl
from tests.conftest import rel_fro
from tests.test_gpu_parity import TOL_FP64, dev, to_dev_colmajor  # noqa: F401

pytestmark = pytest.mark.gpu

ETOOBIG = 7


def _pair(T, dev, options=None):
    import torch

    from paper_1607_06303_amd import signtri

    Tg = to_dev_colmajor(T, dev)
    Un, info_n = signtri.sign_tri_noalloc(Tg)
    Ur, info_r = signtri.sign_tri(Tg, options=options)
    torch.cuda.synchronize()
    return Un.cpu().numpy(), info_n, Ur.cpu().numpy(), info_r


def test_noalloc_matches_signtri(dev):
    import oracle

    rng = np.random.default_rng(21)
    # 1: the largest order, real, skewed inertia (AUTO: the projector form)
    T1 = wl.workload3(8192, 64)
    Un, inf_n, Ur, inf_r = _pair(T1, dev)
    assert inf_n["path_name"] == inf_r["path_name"] == "proj"
    err = rel_fro(Un, Ur)
    print("n=8192 proj: noalloc vs signtri %.3e, max |diff| %.3e" % (err, np.max(np.abs(Un - Ur))))
    assert err <= TOL_FP64
    # 2: a smaller one in the same scratch, interleaved signs (the dataflow sweep)
    T2 = wl.make_T(700, rng)
    Un, inf_n, Ur, inf_r = _pair(T2, dev, options={"sweep": "dataflow"})
    assert inf_n["path_name"] == inf_r["path_name"] == "ph"
    assert inf_n["sweep_name"] == "dataflow"
    assert rel_fro(Un, Ur) <= TOL_FP64
    assert rel_fro(Un, oracle.sign_tri(T2)) <= TOL_FP64
    # 3: complex, smaller again
    T3 = wl.make_T(300, rng, complex_=True)
    Un, inf_n, Ur, inf_r = _pair(T3, dev, options={"sweep": "dataflow"})
    assert rel_fro(Un, Ur) <= TOL_FP64
    assert rel_fro(Un, oracle.sign_tri(T3)) <= TOL_FP64


def test_noalloc_rejects_orders_beyond_its_scratch(dev):
    import torch

    from paper_1607_06303_amd import signtri

    n = 8193
    Tg = torch.zeros((n, n), dtype=torch.float64, device=dev).t()  # column-major, never read
    U = torch.full((n, n), 7.0, dtype=torch.float64, device=dev).t()
    with pytest.raises(signtri.SignTriError) as e:
        signtri.sign_tri_noalloc(Tg, out=U)
    assert e.value.code == ETOOBIG
    torch.cuda.synchronize()
    assert bool(torch.all(U == 7.0))
