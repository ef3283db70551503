"""GPU parity of the batched entry point against the CPU oracle, matrix by matrix.

The batch mixes orders (a single block, ragged last blocks, several blocks),
inertias (interleaved, all one sign, grouped by sign so the Parlett-Sylvester
form runs), and empty matrices; every result must meet the single-matrix bar.
Repeated calls replay a captured graph, so the tests also change T in place
between calls and interleave other calls.
"""
import numpy as np
import pytest

from paper_1607_06303_amd import workloads as wl
from tests.conftest import rel_fro
from tests.test_gpu_parity import TOL_FP64, dev, to_dev_colmajor  # noqa: F401

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-4


def make_batch(seed, sizes):
    rng = np.random.default_rng(seed)
    Ts = []
    for k, n in enumerate(sizes):
        kind = k % 4
        if n == 0:
            Ts.append(np.zeros((0, 0)))
            continue
        if kind == 0:
            s = wl.random_signs(n, rng)
        elif kind == 1:
            s = np.full(n, 1.0 if k % 8 == 1 else -1.0)
        elif kind == 2:
            p = max(1, n // 3)
            s = np.concatenate([np.ones(p), -np.ones(n - p)])
        else:
            s = wl.signs_with_negatives(n, max(1, n // 20), rng)
        Ts.append(wl.make_T(n, rng, signs=s))
    return Ts


SIZES = [1, 2, 17, 32, 33, 64, 100, 129, 300, 45, 250, 96]


def run_batch(Ts, dev, **kw):
    import torch

    from paper_1607_06303_amd import signtri

    Tg = [to_dev_colmajor(T, dev) for T in Ts]
    Us, infos = signtri.sign_tri_batched(Tg, **kw)
    torch.cuda.synchronize()
    return [U.cpu().numpy() for U in Us], infos, Tg, Us


def check_all(Ts, Us, tol):
    import oracle

    for T, U in zip(Ts, Us):
        ref = oracle.sign_tri(T)
        err = rel_fro(U, ref) if T.shape[0] else 0.0
        assert err <= tol, (T.shape, err)
        assert not np.any(np.tril(U, -1))


@pytest.mark.parametrize("mode,tol", [("fp64", TOL_FP64), ("mixed", TOL_FP64), ("fp32", TOL_FP32)])
def test_batched_modes(dev, mode, tol):
    Ts = make_batch(8000, SIZES)
    Us, infos, _, _ = run_batch(Ts, dev, mode=mode)
    check_all(Ts, Us, tol)
    if mode == "mixed":
        assert all(i["fallback_tiles"] == 0 for i in infos)
    paths = {i["path_name"] for i in infos}
    assert paths == {"trivial", "ph", "ps"}, paths


def test_batched_empty_and_single(dev):
    Ts = make_batch(8100, [0, 5, 0])
    Us, infos, _, _ = run_batch(Ts, dev)
    check_all(Ts, Us, TOL_FP64)


def test_batched_graph_replay_sees_new_data(dev):
    """Same pointers twice (graph replay), then T changed in place, with another
    batch in between: every result must follow the current T."""
    import torch

    from paper_1607_06303_amd import signtri

    Ts = make_batch(8200, [70, 130, 33, 200])
    Tg = [to_dev_colmajor(T, dev) for T in Ts]
    Us = [signtri.empty_like_layout(t) for t in Tg]
    for _ in range(3):
        signtri.sign_tri_batched(Tg, outs=Us)
    torch.cuda.synchronize()
    check_all(Ts, [U.cpu().numpy() for U in Us], TOL_FP64)
    other = make_batch(8300, [64, 90])
    Uo, _, _, _ = run_batch(other, dev)
    check_all(other, Uo, TOL_FP64)
    # new values, same signs and pointers: the cached graph must use them
    rng = np.random.default_rng(8400)
    Ts2 = []
    for T, g in zip(Ts, Tg):
        T2 = T.copy()
        T2[np.triu_indices(T.shape[0], 1)] = rng.standard_normal(T.shape[0] * (T.shape[0] - 1) // 2) / 10
        g.copy_(torch.from_numpy(T2).to(dev))
        Ts2.append(T2)
    signtri.sign_tri_batched(Tg, outs=Us)
    torch.cuda.synchronize()
    check_all(Ts2, [U.cpu().numpy() for U in Us], TOL_FP64)


def test_batched_matches_single_calls(dev):
    import torch

    from paper_1607_06303_amd import signtri

    Ts = make_batch(8500, [40, 160, 257])
    Ub, _, Tg, _ = run_batch(Ts, dev)
    for T, g, U in zip(Ts, Tg, Ub):
        Us, _ = signtri.sign_tri(g)
        torch.cuda.synchronize()
        assert rel_fro(U, Us.cpu().numpy()) <= 1e-13


def test_batched_domain_error(dev):
    from paper_1607_06303_amd import signtri

    Ts = make_batch(8600, [40, 50, 60])
    Ts[1][7, 7] = 0.0
    with pytest.raises(signtri.SignTriError) as ei:
        run_batch(Ts, dev)
    assert ei.value.code == 1


def test_batched_workload4_sample(dev):
    """A sample of the 2000-matrix workload's size and inertia distribution."""
    Ts = wl.workload4(count=60)
    Us, infos, _, _ = run_batch(Ts, dev, mode="mixed")
    check_all(Ts, Us, TOL_FP64)


@pytest.mark.parametrize("mode,tol", [("fp64", TOL_FP64), ("mixed", TOL_FP64), ("fp32", TOL_FP32)])
def test_batched_complex(dev, mode, tol):
    """Complex matrices in one batched call: interleaved, grouped by sign
    (Parlett-Sylvester), one sign, near the imaginary axis, and empty."""
    rng = np.random.default_rng(8700)
    Ts = []
    for k, n in enumerate([1, 40, 97, 130, 0, 64, 200]):
        if n == 0:
            Ts.append(np.zeros((0, 0), dtype=complex))
        elif k % 3 == 1:
            p = n // 3
            s = np.concatenate([np.ones(p), -np.ones(n - p)])
            Ts.append(wl.make_T(n, rng, complex_=True, signs=s))
        elif k == 5:
            Ts.append(wl.make_T(n, rng, complex_=True, signs=np.ones(n)))
        else:
            Ts.append(wl.make_T(n, rng, complex_=True, re_range=(1e-2, 1.0)))
    Us, infos, _, _ = run_batch(Ts, dev, mode=mode)
    check_all(Ts, Us, tol)
    assert {i["path_name"] for i in infos} == {"trivial", "ph", "ps"}
    if mode == "mixed":
        assert all(i["fallback_tiles"] == 0 for i in infos)


def test_batched_mixed_graph_replays(dev):
    """The refined mode runs as one captured graph (its convergence tests and the
    FP64 recomputation decided on the device): three replays with other work
    between them, each checked, the infos of each replay filled; then T changed in
    place; then a forced stall of every block (a different graph), whose FP64
    recomputation covers every block."""
    import torch

    from paper_1607_06303_amd import signtri

    Ts = make_batch(8500, [70, 130, 33, 200, 300])
    Tg = [to_dev_colmajor(T, dev) for T in Ts]
    Us = [signtri.empty_like_layout(t) for t in Tg]
    for rep in range(3):
        for U in Us:
            U.fill_(float("nan"))
        _, infos = signtri.sign_tri_batched(Tg, outs=Us, mode="mixed")
        torch.cuda.synchronize()
        check_all(Ts, [U.cpu().numpy() for U in Us], TOL_FP64)
        for T, inf in zip(Ts, infos):
            if inf["path_name"] != "trivial" and T.shape[0] > 32:
                assert inf["refine_steps"] >= 1 and inf["fallback_tiles"] == 0, (rep, inf)
        # eager work on the same stream between replays
        Uo, _, _, _ = run_batch(make_batch(8600 + rep, [64, 90]), dev, mode="fp64")
    rng = np.random.default_rng(8700)
    Ts2 = []
    for T, g in zip(Ts, Tg):
        T2 = T.copy()
        T2[np.triu_indices(T.shape[0], 1)] = rng.standard_normal(T.shape[0] * (T.shape[0] - 1) // 2) / 10
        g.copy_(torch.from_numpy(T2).to(dev))
        Ts2.append(T2)
    signtri.sign_tri_batched(Tg, outs=Us, mode="mixed")
    torch.cuda.synchronize()
    check_all(Ts2, [U.cpu().numpy() for U in Us], TOL_FP64)
    for rep in range(2):
        _, infos = signtri.sign_tri_batched(Tg, outs=Us, mode="mixed", options={"force_stall": -1})
        torch.cuda.synchronize()
        check_all(Ts2, [U.cpu().numpy() for U in Us], TOL_FP64)
        for T, inf in zip(Ts2, infos):
            if inf["path_name"] == "ph":
                nb = (T.shape[0] + 31) // 32
                assert inf["fallback_tiles"] == nb * (nb - 1) // 2, inf
    with pytest.raises(signtri.SignTriError) as ei:
        signtri.sign_tri_batched(Tg, outs=Us, mode="mixed",
                                 options={"force_stall": -1, "no_fallback": 1})
    assert ei.value.code == 4


def test_batched_mixed_strips_without_graph(dev):
    # The timers switch the batched form from its captured graph to direct
    # launches, which take the host's copy of the signs: matrices whose minority
    # sign class has at most n / 32 entries then take the residual's entries of
    # differing signs from strips (the others from the equal-signs tiles), next
    # to matrices that keep the combined tiles.
    from paper_1607_06303_amd import signtri

    rng = np.random.default_rng(8700)
    Ts = []
    for k, n in enumerate([300, 520, 96, 700, 64, 450]):
        if k % 2 == 0:
            s = -np.ones(n) if k == 4 else np.ones(n)
            pick = rng.choice(n, max(1, n // 40), replace=False)
            s[pick] = -s[pick]
        else:
            s = wl.random_signs(n, rng)
        Ts.append(wl.make_T(n, rng, signs=s))
    signtri.profile_enable(True)
    try:
        Us, infos, _, _ = run_batch(Ts, dev, mode="mixed")
    finally:
        signtri.profile_enable(False)
    check_all(Ts, Us, TOL_FP64)
    assert all(i["fallback_tiles"] == 0 for i in infos)
