"""GPU parity of every sweep variant the autotuner chooses between, and the
autotuner itself: each variant (dataflow sweep at each persistent grid size,
superdiagonal sweep with 32 x 32 and 64 x 64 blocks) must meet the oracle's
bar, the tuner must record a choice that later default calls use, and the
result it leaves in U must be sign(T)."""
import numpy as np
import pytest

from paper_1607_06303_amd import workloads as wl
from tests.conftest import rel_fro
from tests.test_gpu_parity import TOL_FP64, check, dev, to_dev_colmajor  # noqa: F401

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-4


@pytest.fixture
def clean_table():
    from paper_1607_06303_amd import signtri

    signtri.tune_clear()
    yield
    signtri.tune_clear()


@pytest.mark.parametrize("n", [65, 300])
@pytest.mark.parametrize("sweep,tile", [("superdiag", 32), ("superdiag", 64), ("dataflow", 32)])
def test_real_fp64_sweep_variants(dev, clean_table, n, sweep, tile):
    rng = np.random.default_rng(9000 + n + tile)
    _, info, _ = check(wl.make_T(n, rng), dev, options={"sweep": sweep, "tile": tile})
    assert info["sweep_name"] == sweep and info["tile"] == tile
    assert (info["wgs_per_cu"] > 0) == (sweep == "dataflow")


@pytest.mark.parametrize("n", [77, 300, 517])
def test_complex_fp64_superdiag_sweep(dev, clean_table, n):
    # the complex superdiagonal sweep's products (K chunks pipelined through
    # registers, split over several workgroups for long superdiagonals) against
    # the oracle, ragged last block included
    rng = np.random.default_rng(9050 + n)
    _, info, _ = check(wl.make_T(n, rng, complex_=True), dev, options={"sweep": "superdiag"})
    assert info["sweep_name"] == "superdiag" and info["tile"] == 32


@pytest.mark.parametrize("mode,tol", [("fp64", TOL_FP64), ("mixed", TOL_FP64), ("fp32", TOL_FP32)])
@pytest.mark.parametrize("wgs", [1, 2, 3, 50])
def test_dataflow_grid_sizes(dev, clean_table, mode, tol, wgs):
    rng = np.random.default_rng(9100 + wgs)
    _, info, _ = check(wl.make_T(260, rng), dev, tol=tol, mode=mode,
                       options={"sweep": "dataflow", "wgs_per_cu": wgs})
    assert 1 <= info["wgs_per_cu"] <= wgs  # clamped to what fits
    if wgs == 1:
        assert info["wgs_per_cu"] == 1


def test_ps_with_superdiag_pinned_runs_ph(dev, clean_table):
    from paper_1607_06303_amd import signtri

    rng = np.random.default_rng(9200)
    s = np.concatenate([np.ones(40), -np.ones(160)])
    T = wl.make_T(200, rng, signs=s)
    _, info, _ = check(T, dev, options={"sweep": "superdiag"})
    assert info["path_name"] == "ph" and info["sweep_name"] == "superdiag"
    with pytest.raises(signtri.SignTriError) as ei:
        signtri.sign_tri(to_dev_colmajor(T, dev), algo="ps", options={"sweep": "superdiag"})
    assert ei.value.code == 5


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_autotune_records_and_is_used(dev, clean_table, mode):
    import torch

    import oracle
    from paper_1607_06303_amd import signtri

    rng = np.random.default_rng(9300)
    T = wl.make_T(400, rng)
    Tg = to_dev_colmajor(T, dev)
    U = signtri.empty_like_layout(Tg)
    best = signtri.autotune(Tg, mode=mode, reps=2, out=U)
    torch.cuda.synchronize()
    assert rel_fro(U.cpu().numpy(), oracle.sign_tri(T)) <= TOL_FP64
    assert best["path"] == 1 and best["log2n"] == 9 and best["ms"] > 0
    if mode == "fp64":
        assert best["sweep_name"] in ("dataflow", "superdiag")
    else:
        assert best["sweep_name"] == "dataflow"
    assert signtri.tune_lookup(False, mode, "ph", 400) == best
    # a default call of the same size class takes the recorded choice
    T2 = wl.make_T(300, np.random.default_rng(9301))
    _, info, _ = check(T2, dev, mode=mode)
    assert info["sweep"] == best["sweep"] and info["tile"] == best["tile"]
    if best["sweep_name"] == "dataflow":
        assert info["wgs_per_cu"] == best["wgs_per_cu"]
    # an explicit option still wins over the table
    _, info, _ = check(T2, dev, mode=mode, options={"sweep": "dataflow", "wgs_per_cu": 1})
    assert info["sweep_name"] == "dataflow" and info["wgs_per_cu"] == 1


def test_autotune_ps_and_complex_and_trivial(dev, clean_table):
    import torch

    from paper_1607_06303_amd import signtri

    rng = np.random.default_rng(9400)
    s = np.concatenate([np.ones(30), -np.ones(270)])
    Tps = to_dev_colmajor(wl.make_T(300, rng, signs=s), dev)
    b = signtri.autotune(Tps, reps=1)
    assert b["path"] == 2 and b["sweep_name"] == "dataflow"
    Tc = to_dev_colmajor(wl.make_T(150, rng, complex_=True), dev)
    b = signtri.autotune(Tc, reps=1)
    assert b["sweep_name"] in ("dataflow", "superdiag") and b["dtype"] == 1
    b = signtri.autotune(Tc, mode="mixed", reps=1)
    assert b["sweep_name"] == "dataflow" and b["mode"] == 1
    Tt = to_dev_colmajor(wl.make_T(100, rng, signs=np.ones(100)), dev)
    b = signtri.autotune(Tt, reps=1)
    assert b["path"] == 0 and b["sweep"] == 0
    torch.cuda.synchronize()


def test_batched_grid_option(dev, clean_table):
    import torch

    import oracle
    from paper_1607_06303_amd import signtri

    rng = np.random.default_rng(9500)
    Ts = [wl.make_T(n, rng) for n in (40, 130, 257)]
    Tg = [to_dev_colmajor(T, dev) for T in Ts]
    for wgs in (1, 2):
        Us, infos = signtri.sign_tri_batched(Tg, options={"wgs_per_cu": wgs})
        torch.cuda.synchronize()
        for T, U, inf in zip(Ts, Us, infos):
            assert rel_fro(U.cpu().numpy(), oracle.sign_tri(T)) <= TOL_FP64
            assert inf["wgs_per_cu"] == wgs and inf["sweep_name"] == "dataflow"


def test_tuning_table_file_round_trip(dev, clean_table, tmp_path):
    """A measured choice survives save / clear / load and steers a later call."""
    from paper_1607_06303_amd import signtri

    rng = np.random.default_rng(9600)
    T = wl.make_T(300, rng)
    Tg = to_dev_colmajor(T, dev)
    best = signtri.autotune(Tg, reps=1)
    path = str(tmp_path / "tune.txt")
    signtri.tune_save(path)
    signtri.tune_clear()
    assert signtri.tune_lookup(False, "fp64", "ph", 300) is None
    signtri.tune_load(path)
    got = signtri.tune_lookup(False, "fp64", "ph", 300)
    assert (got["sweep"], got["tile"], got["wgs_per_cu"]) == (best["sweep"], best["tile"],
                                                             best["wgs_per_cu"])
    _, info, _ = check(T, dev)
    assert (info["sweep"], info["tile"]) == (best["sweep"], best["tile"])


def test_autotune_batched_records_and_is_used(dev, clean_table):
    """The batched tuner times each grid on the batch, records the fastest for the
    size class of the largest order, and later batched calls (grid left at 0)
    run it; every matrix stays sign(T)."""
    import torch

    import oracle
    from paper_1607_06303_amd import signtri

    rng = np.random.default_rng(9700)
    Ts = [wl.make_T(n, rng) for n in (30, 100, 200)]
    Tg = [to_dev_colmajor(T, dev) for T in Ts]
    for mode, tol in (("fp64", TOL_FP64), ("mixed", TOL_FP64)):
        best = signtri.autotune_batched(Tg, mode=mode, reps=1)
        assert best["path"] == 8 and best["log2n"] == 8 and best["wgs_per_cu"] >= 1
        assert signtri.tune_lookup(False, mode, "batched", 256)["wgs_per_cu"] == best["wgs_per_cu"]
        Us, infos = signtri.sign_tri_batched(Tg, mode=mode)
        torch.cuda.synchronize()
        for T, U, inf in zip(Ts, Us, infos):
            assert rel_fro(U.cpu().numpy(), oracle.sign_tri(T)) <= tol
            assert inf["wgs_per_cu"] == best["wgs_per_cu"]

