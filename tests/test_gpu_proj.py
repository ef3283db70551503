"""GPU parity of the projector form (the Parlett-Sylvester result for an
ungrouped diagonal) against the oracle, through the C ABI.

The oracle sides: the element-by-element Parlett-Higham substitution (C), and
on some cases also the Section 3 route itself (Schur reordering by adjacent
swaps, the sign-split Sylvester equation, the transformation back).  Bar:
1e-11 relative Frobenius error.  Sizes span one to several 64-row blocks with
ragged tops; minority counts span 1..512 (real T) including 32/33, 63/64/65,
128 and 300; the minority class is negative or positive; its rows sit at the
ends, in runs and adjacent pairs, and in whole blocks of minority rows.
"""
import numpy as np
import pytest

from paper_1607_06303_amd import workloads as wl
from tests.conftest import rel_fro
from tests.test_gpu_parity import TOL_FP64, dev, run_gpu, to_dev_colmajor  # noqa: F401

pytestmark = pytest.mark.gpu


def skewed(n, m, seed, minority=-1, where=None):
    rng = wl.rng_for(3, salt=seed)
    s = -minority * np.ones(n)
    if where is None:
        where = rng.choice(n, size=m, replace=False)
    s[np.asarray(where)] = minority
    return wl.make_T(n, rng, signs=s)


CASES = [
    (2, 1, None),
    (3, 1, [1]),
    (64, 1, [63]),
    (64, 3, [0, 1, 63]),
    (65, 7, None),
    (127, 32, None),
    (128, 33, None),
    (200, 5, [0, 1, 2, 198, 199]),
    (333, 31, None),
    (333, 63, None),
    (700, 64, None),
    (700, 16, list(range(300, 316))),   # one contiguous run
]


@pytest.mark.parametrize("n,m,where", CASES)
@pytest.mark.parametrize("minority", [-1, 1])
def test_proj_matches_oracle(dev, n, m, where, minority):
    import oracle

    T = skewed(n, m, n * 7 + m, minority, where)
    U, info = run_gpu(T, dev, algo="proj")
    assert info["path_name"] == "proj", info
    err = rel_fro(U, oracle.sign_tri(T))
    assert err <= TOL_FP64, (n, m, err)
    assert not np.any(np.tril(U, -1))


@pytest.mark.parametrize("n,m", [(150, 4), (260, 20)])
def test_proj_matches_reordering_route(dev, n, m):
    from oracle import reorder

    T = skewed(n, m, 91 + n)
    U, info = run_gpu(T, dev, algo="proj")
    ref, rinfo = reorder.sign_tri_reordered(T)
    assert rinfo["k"] > 0
    assert rel_fro(U, ref) <= TOL_FP64


def test_proj_schur_recipe_and_grouped(dev):
    """Repeated diagonal values (the paper's Schur-form recipe), and a grouped diagonal
    where the projector form is the Sylvester form itself."""
    import oracle

    T = wl.schur_like(300, 6, wl.rng_for(9, salt=3))
    U, _ = run_gpu(T, dev, algo="proj")
    assert rel_fro(U, oracle.sign_tri(T)) <= TOL_FP64
    G = wl.sorted_positive_first(skewed(250, 12, 5))
    U, _ = run_gpu(G, dev, algo="proj")
    assert rel_fro(U, oracle.sign_tri(G)) <= TOL_FP64


def test_proj_garbage_below_and_row_major(dev):
    import torch

    import oracle
    from paper_1607_06303_amd import signtri

    T = skewed(190, 9, 17)
    Tg = T + np.tril(np.full_like(T, np.nan), -1)
    U, _ = run_gpu(Tg, dev, algo="proj")
    assert rel_fro(U, oracle.sign_tri(T)) <= TOL_FP64
    Tr = torch.from_numpy(np.ascontiguousarray(T)).to(dev)   # row-major
    Ur, info = signtri.sign_tri(Tr, algo="proj")
    torch.cuda.synchronize()
    assert info["path_name"] == "proj"
    assert rel_fro(Ur.cpu().numpy(), oracle.sign_tri(T)) <= TOL_FP64


def test_proj_repeated_calls_and_modes(dev):
    """Back-to-back calls reuse the workspace; every mode runs the FP64 form."""
    import oracle

    T1 = skewed(300, 40, 1)
    T2 = skewed(129, 3, 2, minority=1)
    for T in (T1, T2, T1):
        for mode in ("fp64", "mixed", "fp32"):
            U, info = run_gpu(T, dev, algo="proj", mode=mode)
            assert rel_fro(U, oracle.sign_tri(T)) <= TOL_FP64, mode


def test_auto_choice(dev):
    """AUTO: the projector form for a small minority class, the substitution for
    balanced inertia, the Sylvester form for a grouped diagonal."""
    _, info = run_gpu(skewed(512, 8, 3), dev)
    assert info["path_name"] == "proj"
    _, info = run_gpu(wl.workload1(256), dev)
    assert info["path_name"] == "ph"
    _, info = run_gpu(wl.sorted_positive_first(wl.workload1(256)), dev)
    assert info["path_name"] == "ps"


def test_proj_unsupported(dev):
    from paper_1607_06303_amd import signtri

    with pytest.raises(signtri.SignTriError):
        run_gpu(skewed(1100, 513, 8), dev, algo="proj")
    with pytest.raises(signtri.SignTriError):
        run_gpu(cskewed(300, 65, 8), dev, algo="proj")
    # all one sign: the trivial path, whatever the algorithm asked for
    U, info = run_gpu(wl.make_T(40, wl.rng_for(1, salt=4), signs=np.ones(40)), dev, algo="proj")
    assert info["path_name"] == "trivial" and np.array_equal(U, np.eye(40))


def test_proj_padded_and_workspace(dev):
    """Padded leading dimensions of T and U (the padding rows of U untouched), and a
    caller workspace of exactly the size the library asks for (smaller: an error)."""
    import torch

    import oracle
    from paper_1607_06303_amd import signtri

    n, ld = 230, 257
    T = skewed(n, 11, 41)
    G = T + np.tril(np.full_like(T, 1e300), -1)
    Tg = to_dev_colmajor(G, dev, ld=ld)
    Ubuf = torch.full((n, ld), 7.0, dtype=torch.float64, device=dev)  # column-major ld x n
    U = Ubuf.t()[:n, :]
    _, info = signtri.sign_tri(Tg, out=U, algo="proj")
    torch.cuda.synchronize()
    assert info["path_name"] == "proj"
    full = Ubuf.cpu().numpy().T
    assert np.all(full[n:, :] == 7.0), "padding rows must be untouched"
    assert rel_fro(full[:n, :], oracle.sign_tri(T)) <= TOL_FP64
    need = signtri.workspace_size(n, algo="proj")
    small = torch.empty(need - 256, dtype=torch.uint8, device=dev)
    with pytest.raises(signtri.SignTriError) as ei:
        signtri.sign_tri(to_dev_colmajor(T, dev), workspace=small, algo="proj")
    assert ei.value.code == 3
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    U2, _ = signtri.sign_tri(to_dev_colmajor(T, dev), workspace=ws, algo="proj")
    torch.cuda.synchronize()
    assert rel_fro(U2.cpu().numpy(), oracle.sign_tri(T)) <= TOL_FP64


@pytest.mark.parametrize("where", [[0], [99], [1, 98]])
def test_proj_minority_at_the_ends(dev, where):
    import oracle

    T = skewed(100, len(where), 50 + where[0], where=where)
    U, info = run_gpu(T, dev, algo="proj")
    assert info["path_name"] == "proj"
    assert rel_fro(U, oracle.sign_tri(T)) <= TOL_FP64


def test_proj_near_zero_diagonal(dev):
    """Real diagonal magnitudes down to 1e-3 on both sides of the imaginary axis: the
    substitutions divide by differences as small as 2e-3 (as Eq. (1) does)."""
    import oracle

    rng = wl.rng_for(5, salt=21)
    s = np.ones(400)
    s[rng.choice(400, 10, replace=False)] = -1
    T = wl.make_T(400, rng, signs=s, re_range=(1e-3, 1.0))
    U, info = run_gpu(T, dev, algo="proj")
    assert info["path_name"] == "proj"
    assert rel_fro(U, oracle.sign_tri(T)) <= TOL_FP64


def test_proj_full_size_positive_minority(dev):
    """n = 4096 with 40 positive entries (majority sign -1), through AUTO: invariants at
    full size, leading, trailing and interior principal blocks against the oracle."""
    import torch

    import oracle

    T = skewed(4096, 40, 77, minority=1)
    Tg = to_dev_colmajor(T, dev)
    from paper_1607_06303_amd import signtri

    U, info = signtri.sign_tri(Tg)
    torch.cuda.synchronize()
    assert info["path_name"] == "proj"
    Ut = U.contiguous()
    Tt = torch.triu(Tg.contiguous())
    nu = torch.linalg.norm(Ut).item()
    eye = torch.eye(4096, dtype=Ut.dtype, device=Ut.device)
    assert torch.linalg.norm(Ut @ Ut - eye).item() / (nu * nu) <= 1e-13
    com = torch.linalg.norm(Tt @ Ut - Ut @ Tt).item() / (torch.linalg.norm(Tt).item() * nu)
    assert com <= 1e-13
    Uh = U.cpu().numpy()
    for a in (0, 1500, 4096 - 600):
        ref = oracle.sign_tri(T[a:a + 600, a:a + 600])
        assert rel_fro(Uh[a:a + 600, a:a + 600], ref) <= TOL_FP64, a


def cskewed(n, m, seed, minority=-1, re_range=(0.5, 2.0), where=None):
    rng = wl.rng_for(2, salt=seed)
    s = -minority * np.ones(n)
    if where is None:
        where = rng.choice(n, size=m, replace=False)
    s[np.asarray(where)] = minority
    return wl.make_T(n, rng, complex_=True, signs=s, re_range=re_range, im_range=(-1.0, 1.0))


@pytest.mark.parametrize("n,m,where", [(2, 1, None), (33, 3, [0, 1, 32]), (100, 5, None),
                                       (257, 31, None), (300, 64, None)])
@pytest.mark.parametrize("minority", [-1, 1])
def test_proj_complex_matches_oracle(dev, n, m, where, minority):
    """Complex T: the same form with transposes (left basis of J T^T J), 32-row blocks."""
    import oracle

    T = cskewed(n, m, n + 3 * m, minority, where=where)
    U, info = run_gpu(T, dev, algo="proj")
    assert info["path_name"] == "proj"
    assert rel_fro(U, oracle.sign_tri(T)) <= TOL_FP64
    assert not np.any(np.tril(U, -1))


def test_proj_complex_reordering_route_and_near_imaginary(dev):
    import oracle
    from oracle import reorder

    T = cskewed(180, 7, 5)
    U, _ = run_gpu(T, dev, algo="proj")
    ref, rinfo = reorder.sign_tri_reordered(T)
    assert rinfo["k"] > 0 and rel_fro(U, ref) <= TOL_FP64
    T = cskewed(240, 12, 6, re_range=(1e-3, 1.0))
    U, _ = run_gpu(T, dev, algo="proj")
    assert rel_fro(U, oracle.sign_tri(T)) <= TOL_FP64


CLUSTERS = [
    # ten minority rows inside one 64-row block, two waves' worth of columns, with
    # majority rows between them (the in-wave chain and the L rows set within a wave)
    (256, [70, 72, 75, 77, 80, 90, 95, 100, 101, 102]),
    # 64 consecutive minority rows across block boundaries (every wave's columns set
    # their L rows within a block while later waves of the same block still solve)
    (200, list(range(100, 164))),
    # clusters at wave boundaries of the column order: columns 6..9 and 14..17
    (330, [5, 9, 20, 40, 60, 64, 65, 66, 67, 130, 131, 132, 140, 150, 151, 152, 153, 154, 300]),
    # one minority row per block, and one at each end
    (520, [0] + [64 * k + 17 for k in range(1, 8)] + [519]),
    # a block made only of minority rows, at the top and at the bottom (n = 1000: the
    # blocks are cut from the bottom, so the top block is short)
    (1000, list(range(0, 64))),
    (1000, list(range(936, 1000))),
    # a bottom group whose eigenvector-form column walk meets earlier columns'
    # minority rows in its blocks, the short top block (40 rows) included
    (1000, [5, 20, 33, 300, 301, 650, 651, 652] + list(range(992, 1000))),
]


@pytest.mark.parametrize("n,where", CLUSTERS,
                         ids=["one-block", "run64", "wave-edges", "spread", "top64", "bottom64",
                              "walk-windows"])
@pytest.mark.parametrize("minority", [-1, 1])
def test_proj_clustered_minority(dev, n, where, minority):
    """Minority rows clustered within blocks and across wave boundaries of the column order."""
    import oracle

    T = skewed(n, len(where), n + len(where), minority, where)
    U, info = run_gpu(T, dev, algo="proj")
    assert info["path_name"] == "proj"
    assert rel_fro(U, oracle.sign_tri(T)) <= TOL_FP64
    assert not np.any(np.tril(U, -1))


# More than 64 minority columns (real T): the coupling with the earlier columns
# whose rows lie in the blocks below is applied as FP64 MFMA products (the block
# just below between blocks, the rest ahead of time), and the owners take the
# columns in chunks of 64.
WIDE = [
    (300, 65, None),
    (520, 128, None),
    (700, 300, None),
    (1100, 512, None),
    # whole blocks of minority rows: near windows of 64 columns, and windows of the
    # block below wider than what the helpers fetch ahead
    (600, 200, list(range(150, 350))),
    (700, 130, list(range(0, 40)) + list(range(200, 250)) + list(range(660, 700))),
    # one column per group on every other block, then a dense run at the bottom
    (900, 100, [9 * k for k in range(60)] + list(range(860, 900))),
]


@pytest.mark.parametrize("n,m,where", WIDE,
                         ids=["65", "128", "300", "512", "run200", "three-runs", "sparse-dense"])
@pytest.mark.parametrize("minority", [-1, 1])
def test_proj_wide_minority(dev, n, m, where, minority):
    import oracle

    T = skewed(n, m, 13 * n + m, minority, where)
    U, info = run_gpu(T, dev, algo="proj")
    assert info["path_name"] == "proj", info
    assert rel_fro(U, oracle.sign_tri(T)) <= TOL_FP64, (n, m)
    assert not np.any(np.tril(U, -1))


@pytest.mark.parametrize("n,m", [(330, 65), (400, 128)])
def test_proj_wide_matches_reordering_route(dev, n, m):
    from oracle import reorder

    T = skewed(n, m, 17 + n)
    U, info = run_gpu(T, dev, algo="proj")
    assert info["path_name"] == "proj"
    ref, rinfo = reorder.sign_tri_reordered(T)
    assert rinfo["k"] > 0
    assert rel_fro(U, ref) <= TOL_FP64


def test_proj_wide_auto_and_repeat(dev):
    """AUTO takes the projector form past 64 minority entries while 3 n^2 m stays
    below W_PH; the same call twice gives the same bits."""
    import oracle

    from paper_1607_06303_amd import signtri

    T = skewed(2048, 100, 23)
    plan = signtri.plan_host(np.where(np.diag(T) > 0, 1, -1).astype(np.int8))
    assert 3.0 * 2048 ** 2 * 100 < plan["w_ph"]
    U1, info = run_gpu(T, dev)
    assert info["path_name"] == "proj"
    U2, _ = run_gpu(T, dev)
    assert np.array_equal(U1, U2)
    assert rel_fro(U1, oracle.sign_tri(T)) <= TOL_FP64



# Above a group's topmost minority row the substitution runs in the basis of
# the eigenvectors of the group's block of L (no coupling chain), when they are
# well conditioned; with equal or nearly equal minority eigenvalues, or a
# strongly coupled block, it keeps the chain.  Every case matches the oracle.
@pytest.mark.parametrize("kind", ["repeated", "near", "cluster", "spread", "strong"])
def test_proj_eigenvector_form_and_fallback(dev, kind):
    import oracle

    n, m = 700, 16
    rng = np.random.default_rng(9100)
    where = np.sort(rng.choice(n, size=m, replace=False))
    T = skewed(n, m, 9100, -1, where)
    d = np.diag(T).copy()
    if kind == "repeated":
        d[where] = -1.0
    elif kind == "near":
        d[where] = -1.0 - 1e-9 * np.arange(m)
    elif kind == "cluster":
        d[where] = -1.0 - 0.02 * np.arange(m)
    elif kind == "strong":
        T = T + np.triu(rng.standard_normal((n, n)), 1) * 0.5
    T[np.arange(n), np.arange(n)] = d
    U, info = run_gpu(T, dev, algo="proj")
    assert info["path_name"] == "proj", info
    err = rel_fro(U, oracle.sign_tri(T))
    assert err <= TOL_FP64, (kind, err)
