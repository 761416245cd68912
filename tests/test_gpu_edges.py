"""Edge cases of the FP32 sweep against the FP64 oracle (MI355X, through the
C ABI): direction counts outside the tiled kernels' set (D = 1, 3, 5, 7, 13,
arbitrary unit vectors), an all-zero field, a field with zero regions beside
refined clumps, and a dynamic range of densities far beyond the workloads'.
Gate: <= 1e-5 relative per output, plus an absolute floor of 1e-12 max(n)
box: the library drops chords shorter than 1e-12 of a cell (a ray grazing a
cell's edge or corner), which the FP64 oracle keeps as rounding slivers of
about 1e-16 cell; in a column that crosses only empty cells such a sliver is
the whole column.  Exact zeros where the oracle is zero."""
import numpy as np
import pytest

import oracle
from paper_1410_0624_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL_FP32 = 1e-5


@pytest.fixture(scope="module")
def colden():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1410_0624_amd import colden as c
    c.lib()
    return c


def _run(colden, tin, dirs):
    dev = torch.device("cuda:0")
    leaf = torch.from_numpy(tin.leaf_n).to(dev)
    tree = colden.Tree(tin, leaf)
    w = colden.Weights(dirs)
    N = torch.full((tin.n_leaf, dirs.shape[0]), float("nan"), dtype=torch.float32, device=dev)
    c = torch.full((tin.n_leaf,), float("nan"), dtype=torch.float32, device=dev)
    colden.column_densities(tree, w, N, c)
    torch.cuda.synchronize()
    return N.cpu().numpy().astype(np.float64), c.cpu().numpy().astype(np.float64)


def _dirs(D, seed):
    u = np.random.default_rng(seed).normal(size=(D, 3))
    return u / np.linalg.norm(u, axis=1, keepdims=True)


def _check(N, chi, ref, tin):
    assert np.isfinite(N).all() and np.isfinite(chi).all()
    zero = ref == 0
    assert (N[zero] == 0).all()
    floor = 1e-12 * float(tin.leaf_n.max()) * tin.box_cm
    err = np.abs(N[~zero] - ref[~zero])
    assert err.size == 0 or (err <= REL_FP32 * ref[~zero] + floor).all(), (err / ref[~zero]).max()
    assert np.abs(chi - oracle.screening(ref)).max() <= 2e-6
    big = ref > 1e3 * floor
    return (np.abs(N[big] - ref[big]) / ref[big]).max() if big.any() else 0.0


@pytest.mark.parametrize("L,D", [(3, 1), (5, 1), (5, 3), (5, 7), (6, 5), (6, 13)])
def test_direction_counts_outside_the_tiled_set_uniform(colden, L, D):
    """Per-oct kernel with the coarse-table path (L = 6) and without (L <= 5)."""
    tin = synth.workload_uniform(L, sigma=1.5, mean=10.0, seed=40 + D)
    dirs = _dirs(D, 100 + D)
    N, chi = _run(colden, tin, dirs)
    ref = oracle.Tree(tin).columns(dirs)
    print(f"uniform L={L} D={D}: max rel {_check(N, chi, ref, tin):.3e}")


@pytest.mark.parametrize("Lf,B,th,D", [(6, 3, 14.0, 5), (7, 5, 30.0, 7), (6, 2, 14.0, 1),
                                        # D > 16 with no tile chunk: the per-oct kernel's local chord tables
                                        (6, 3, 14.0, 63), (6, 3, 14.0, 65), (7, 5, 30.0, 84)])
def test_direction_counts_outside_the_tiled_set_amr(colden, Lf, B, th, D):
    """Adaptive trees with D outside the tiled set: every target walks the
    weight lists through the dense levels (a lane per direction, passes of
    64 directions above 64)."""
    tin = synth.amr_tree(synth.lognormal_field(1 << Lf, 2.0, 10.0, 60 + D), B, th, 10 * synth.PC_CM)
    dirs = _dirs(D, 200 + D)
    N, chi = _run(colden, tin, dirs)
    ref = oracle.Tree(tin).columns(dirs)
    print(f"AMR {Lf}/{B} D={D} ({tin.n_leaf} leaves): max rel {_check(N, chi, ref, tin):.3e}")


def test_zero_field_gives_zero_columns(colden):
    """n = 0 everywhere: every column is exactly 0 and chi 1 (to one unit in
    the last place of the mean), on the tiled path (D = 12) and the per-oct
    path (D = 3)."""
    tin = synth.uniform_tree(np.zeros((64, 64, 64)), 10 * synth.PC_CM)
    for dirs in (oracle.dirs_healpix(1), _dirs(3, 7)):
        N, chi = _run(colden, tin, dirs)
        assert (N == 0).all()
        assert np.abs(chi - 1.0).max() <= 1.2e-7


def test_zero_regions_beside_refined_clumps(colden):
    """Half of the box empty, refined clumps in the other half: outputs that
    see only empty cells are exactly zero, the rest meet the gate."""
    f = synth.lognormal_field(64, 2.0, 10.0, 77)
    f[:, :, :32] = 0.0
    tin = synth.amr_tree(f, 3, 14.0, 10 * synth.PC_CM)
    assert tin.max_level > tin.base_level
    for dirs in (oracle.dirs_healpix(1), oracle.dirs_axes6()):
        N, chi = _run(colden, tin, dirs)
        ref = oracle.Tree(tin).columns(dirs)
        assert (ref == 0).any()
        print(f"zero half, D={dirs.shape[0]}: max rel {_check(N, chi, ref, tin):.3e}")


def test_extreme_dynamic_range(colden):
    """sigma_ln n = 5 (densities over about 16 decades) on the tiled path."""
    tin = synth.workload_uniform(6, sigma=5.0, mean=10.0, seed=91)
    assert tin.leaf_n.max() / tin.leaf_n.min() > 1e12
    dirs = oracle.dirs_healpix(1)
    N, chi = _run(colden, tin, dirs)
    ref = oracle.Tree(tin).columns(dirs)
    print(f"sigma 5: max rel {_check(N, chi, ref, tin):.3e}")
