"""Adaptive (AMR) trees on the GPU against the FP64 oracle, through the C ABI.

Trees come from seeded log-normal fields refined where the mass-averaged
density exceeds a threshold (Sect. 3's fully threaded tree: a full base grid
plus octs).  Cases span targets at every level, base levels 1 .. 5, shells
dl >= 4 above the dense base grid (the per-axis automaton) and below it (the
coarse tables), HEALPix 1 / 2 and the six axes.  Gate: 1e-5 relative per
output, as for uniform grids."""
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


def _amr(Lf, B, th, seed, sigma=2.0):
    return synth.amr_tree(synth.lognormal_field(1 << Lf, sigma, 10.0, seed), B, th, 10 * synth.PC_CM)


def _run(colden, tin, dirs, chi=True):
    dev = torch.device("cuda:0")
    leaf = torch.from_numpy(tin.leaf_n).to(dev)
    tree = colden.Tree(tin, leaf)
    w = colden.Weights(dirs)
    N = torch.full((tin.n_leaf, dirs.shape[0]), float("nan"), dtype=torch.float32, device=dev)
    c = torch.full((tin.n_leaf,), float("nan"), dtype=torch.float32, device=dev) if chi else None
    colden.column_densities(tree, w, N, c)
    torch.cuda.synchronize()
    out = N.cpu().numpy().astype(np.float64), (c.cpu().numpy().astype(np.float64) if chi else None)
    return out, tree


def _rel(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


CASES = [
    # (fine level, base level, threshold, seed, directions)
    (6, 3, 14.0, 5, "healpix1"),   # dl >= 4 tables at level 2
    (6, 4, 20.0, 5, "healpix2"),   # D = 48
    (7, 4, 30.0, 5, "healpix1"),   # three refined levels, tables up to level 3
    (7, 2, 30.0, 6, "healpix1"),   # shells dl >= 4 at level 3 > base: automaton, then the level-2 table
    (6, 1, 14.0, 7, "axes6"),      # base 2^1, no coarse table at all
    (8, 3, 60.0, 8, "healpix1"),   # five refined levels above an 8^3 base
    (7, 5, 30.0, 7, "healpix2"),   # base 32^3: tiled shells on the active tiles of levels 5 .. 7
    (4, 2, 8.0, 9, "healpix1"),    # finest level 4: no 16^3-oct tile anywhere, every target gathered
    (5, 1, 10.0, 10, "healpix2"),  # one tile at level 5 beside gathered targets of levels 1 .. 4
    (7, 5, 30.0, 7, "mn7x12"),     # the paper's 7 x 12 set (84 directions) on the tiled path
]
DIRS = {"healpix1": oracle.dirs_healpix(1), "healpix2": oracle.dirs_healpix(2), "axes6": oracle.dirs_axes6(),
        "mn7x12": oracle.dirs_mn(7, 12)}


@pytest.mark.parametrize("Lf,B,th,seed,dname", CASES)
def test_amr_parity_all_leaves(colden, Lf, B, th, seed, dname):
    tin = _amr(Lf, B, th, seed)
    dirs = DIRS[dname]
    (N, chi), tree = _run(colden, tin, dirs)
    tr = oracle.Tree(tin)
    ref = tr.columns(dirs)
    rel = _rel(N, ref)
    print(f"AMR {Lf}/{B}/{th} {dname}: {tin.n_leaf} leaves, levels "
          f"{np.bincount(tin.leaf_level)[B:].tolist()}, max rel {rel.max():.3e}")
    assert np.isfinite(N).all()
    assert rel.max() <= REL_FP32
    assert np.abs(chi - oracle.screening(ref)).max() <= 2e-6
    lv, ijk = tree.leaf_coords()
    olv, oijk = tr.leaf_coords()
    np.testing.assert_array_equal(lv, olv)
    np.testing.assert_array_equal(ijk, oijk)


def test_c3_amr_sampled_parity(colden):
    """The AMR workload: 128^3 base + 2 refined levels (4.05M leaves from a
    512^3 field, sigma_ln n = 2), HEALPix N_side = 2 (D = 48); 30k sampled
    leaves of every level against the oracle."""
    tin = synth.workload_amr()
    dirs = oracle.dirs_healpix(2)
    (N, chi), _ = _run(colden, tin, dirs)
    assert np.isfinite(N).all() and (N > 0).all()
    rng = np.random.default_rng(1)
    tg = []
    for l in range(tin.base_level, tin.max_level + 1):
        idx = np.nonzero(tin.leaf_level == l)[0]
        tg.append(rng.choice(idx, min(10000, idx.size), replace=False))
    tg = np.concatenate(tg + [[0, tin.n_leaf - 1]])
    ref = oracle.Tree(tin).columns(dirs, tg)
    rel = _rel(N[tg], ref)
    print(f"C3 sampled: {tg.size} targets, max rel {rel.max():.3e} mean {rel.mean():.3e}")
    assert rel.max() <= REL_FP32
    assert np.abs(chi[tg] - oracle.screening(ref)).max() <= 2e-6


def test_c3b_amr_34m_leaves_sampled_all_forms(colden):
    """The same field refined above 5 cm^-3 (34M leaves, most of them at the
    finest level), D = 48, in the launch configuration the benchmark times:
    FP32 and both split forms on 3k sampled leaves of every level."""
    tin = synth.workload_amr(threshold=5.0)
    assert tin.n_leaf > 25_000_000
    dirs = oracle.dirs_healpix(2)
    rng = np.random.default_rng(2)
    tg = []
    for l in range(tin.base_level, tin.max_level + 1):
        idx = np.nonzero(tin.leaf_level == l)[0]
        tg.append(rng.choice(idx, min(3000, idx.size), replace=False))
    tg = np.concatenate(tg + [[0, tin.n_leaf - 1]])
    ref = oracle.Tree(tin).columns(dirs, tg)
    dev = torch.device("cuda:0")
    tree = colden.Tree(tin, torch.from_numpy(tin.leaf_n).to(dev))
    N = torch.empty((tin.n_leaf, 48), dtype=torch.float32, device=dev)
    chi = torch.empty((tin.n_leaf,), dtype=torch.float32, device=dev)
    idx = torch.from_numpy(tg).to(dev)
    for pname, prec in [("fp32", 0), ("bf16x2", 1), ("fp16x2", 2)]:
        w = colden.Weights(dirs, precision=prec)
        N.fill_(float("nan"))
        chi.fill_(float("nan"))
        colden.column_densities(tree, w, N, chi)
        got = N[idx].cpu().numpy().astype(np.float64)
        assert np.isfinite(got).all()
        assert bool(torch.isfinite(chi).all())
        if prec == 0:
            rel = _rel(got, ref)
            print(f"C3b {pname}: {tg.size} targets, max rel {rel.max():.3e}")
            assert rel.max() <= REL_FP32
            gchi = chi[idx].cpu().numpy().astype(np.float64)
            assert np.abs(gchi - oracle.screening(ref)).max() <= 2e-6
        else:
            err = np.abs(np.log(got) - np.log(ref))
            print(f"C3b {pname}: {tg.size} targets, max |d ln N| {err.max():.3e}")
            assert err.max() <= 1e-3
        w.close()


def test_fully_refined_amr_equals_uniform_on_gpu(colden):
    """A tree refined everywhere is the uniform grid (Sect. 3): same columns,
    leaves permuted into oct order."""
    f = synth.lognormal_field(16, 1.5, 10.0, 9)
    amr = synth.amr_tree(f, base_level=2, threshold=-1.0, box_cm=1e19)
    uni = synth.uniform_tree(f, box_cm=1e19)
    dirs = oracle.dirs_healpix(1)
    (Na, _), _ = _run(colden, amr, dirs, chi=False)
    (Nu, _), _ = _run(colden, uni, dirs, chi=False)
    idx = amr.leaf_ijk[:, 0] + 16 * (amr.leaf_ijk[:, 1] + 16 * amr.leaf_ijk[:, 2])
    assert _rel(Na, Nu[idx]).max() <= 2e-6


def test_amr_tree_update(colden):
    dev = torch.device("cuda:0")
    tin = _amr(6, 3, 14.0, 5)
    rng = np.random.default_rng(3)
    new = (tin.leaf_n * rng.uniform(0.5, 2.0, tin.n_leaf)).astype(np.float32)
    dirs = oracle.dirs_healpix(1)
    tree = colden.Tree(tin, torch.from_numpy(tin.leaf_n).to(dev))
    w = colden.Weights(dirs)
    N = torch.empty((tin.n_leaf, 12), dtype=torch.float32, device=dev)
    colden.column_densities(tree, w, N)
    tree.update(torch.from_numpy(new).to(dev))
    colden.column_densities(tree, w, N)
    torch.cuda.synchronize()
    tin.leaf_n = new
    ref = oracle.Tree(tin).columns(dirs)
    assert _rel(N.cpu().numpy().astype(np.float64), ref).max() <= REL_FP32


def test_amr_malformed_structures(colden):
    dev = torch.device("cuda:0")
    tin = _amr(5, 2, 12.0, 5)
    leaf = torch.from_numpy(tin.leaf_n).to(dev)
    # wrong leaf count
    with pytest.raises(colden.ColdenError) as e:
        colden.Tree(tin, leaf[:-1])
    assert e.value.rc == colden.CD_EINVAL
    # a cell refined twice
    bad = synth.TreeInput(box_cm=tin.box_cm, base_level=tin.base_level, max_level=tin.max_level,
                          oct_parents=[p.copy() for p in tin.oct_parents])
    bad.oct_parents[0] = np.concatenate([bad.oct_parents[0], bad.oct_parents[0][:1]])
    with pytest.raises(colden.ColdenError) as e:
        colden.Tree(bad, leaf)
    assert e.value.rc == colden.CD_EINVAL
    # an oct whose parent cell does not exist
    bad = synth.TreeInput(box_cm=tin.box_cm, base_level=tin.base_level, max_level=tin.max_level,
                          oct_parents=[p.copy() for p in tin.oct_parents])
    have = {tuple(p) for p in (bad.oct_parents[0] * 2)}
    n1 = 1 << (tin.base_level + 1)
    orphan = next((x, y, z) for z in range(n1) for y in range(n1) for x in range(n1)
                  if (x & ~1, y & ~1, z & ~1) not in have)
    bad.oct_parents[1] = np.concatenate([bad.oct_parents[1], np.array([orphan], np.int32)])
    with pytest.raises(colden.ColdenError) as e:
        colden.Tree(bad, leaf)
    assert e.value.rc == colden.CD_EINVAL
    # parent outside the grid
    bad = synth.TreeInput(box_cm=tin.box_cm, base_level=tin.base_level, max_level=tin.max_level,
                          oct_parents=[p.copy() for p in tin.oct_parents])
    bad.oct_parents[0][0, 0] = 1 << tin.base_level
    with pytest.raises(colden.ColdenError) as e:
        colden.Tree(bad, leaf)
    assert e.value.rc == colden.CD_EINVAL
