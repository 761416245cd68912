"""In-situ reference points (Sect. 4.4) against the FP64 oracle's in-situ
mode, through the C ABI (MI355X).  Every shell is seen from the centre of
the target's oct; the library computes the shells dl >= 4 per oct by walking
each ray through their cells, the shells dl = 1..3 with the tiled kernels.
Gates as for the precalculated form: 1e-5 relative (FP32), 1e-3 in ln N
(split forms)."""
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


def _run(colden, tin, dirs, mode, precision=0):
    dev = torch.device("cuda:0")
    leaf = torch.from_numpy(tin.leaf_n).to(dev)
    tree = colden.Tree(tin, leaf)
    w = colden.Weights(dirs, mode=mode, precision=precision)
    N = torch.full((tin.n_leaf, dirs.shape[0]), float("nan"), dtype=torch.float32, device=dev)
    c = torch.full((tin.n_leaf,), float("nan"), dtype=torch.float32, device=dev)
    colden.column_densities(tree, w, N, c)
    torch.cuda.synchronize()
    return N.cpu().numpy().astype(np.float64), c.cpu().numpy().astype(np.float64)


DIRS = {"healpix1": oracle.dirs_healpix(1), "healpix2": oracle.dirs_healpix(2), "axes6": oracle.dirs_axes6(),
        "mn3x8": oracle.dirs_mn(3, 8), "mn5x8": oracle.dirs_mn(5, 8)}


@pytest.mark.parametrize("L,dname,sample", [(5, "healpix1", 0), (6, "healpix1", 0), (6, "healpix2", 0),
                                            (6, "axes6", 0), (6, "mn3x8", 0), (6, "mn5x8", 0),
                                            (7, "healpix1", 60000), (8, "healpix1", 20000)])
def test_insitu_parity(colden, L, dname, sample):
    """Grids of 32^3 .. 256^3 (the C2 field at L = 8, sampled): up to five
    coarse shell levels walked per oct."""
    tin = synth.workload_uniform(L, sigma=1.5, mean=10.0, seed=20 + L)
    dirs = DIRS[dname]
    N, chi = _run(colden, tin, dirs, colden.CD_INSITU)
    tg = (np.arange(tin.n_leaf) if sample == 0 else
          np.concatenate([np.random.default_rng(L).choice(tin.n_leaf, sample, replace=False), [0, tin.n_leaf - 1]]))
    ref = oracle.Tree(tin).columns(dirs, tg, mode=oracle.INSITU)
    rel = np.abs(N[tg] - ref) / ref
    print(f"insitu L={L} {dname}: max rel {rel.max():.3e} mean {rel.mean():.3e}")
    assert np.isfinite(N).all()
    assert rel.max() <= REL_FP32
    assert np.abs(chi[tg] - oracle.screening(ref)).max() <= 2e-6


@pytest.mark.parametrize("L,D", [(2, 12), (3, 12), (4, 12), (5, 7), (6, 7), (6, 13), (7, 3)])
def test_insitu_per_oct_kernel(colden, L, D):
    """Uniform grids without the tiled kernels (2^L < 32 or D outside the
    tiled set): the per-oct kernel with the walked rows of each oct."""
    tin = synth.workload_uniform(L, sigma=1.5, mean=10.0, seed=60 + L)
    dirs = DIRS["healpix1"] if D == 12 else _rand_dirs(D, 70 + D)
    N, chi = _run(colden, tin, dirs, colden.CD_INSITU)
    ref = oracle.Tree(tin).columns(dirs, mode=oracle.INSITU)
    rel = np.abs(N - ref) / ref
    print(f"insitu per-oct L={L} D={D}: max rel {rel.max():.3e}")
    assert np.isfinite(N).all()
    assert rel.max() <= REL_FP32
    assert np.abs(chi - oracle.screening(ref)).max() <= 2e-6


def test_insitu_c4_512_sampled(colden):
    """The 512^3 workload (134M leaves) in the launch configuration the
    benchmark times, 12 and 48 directions: the walk covers six coarse shell
    levels; sampled leaves (and both corners) against the oracle."""
    tin = synth.workload_uniform(9, sigma=1.5, mean=10.0, seed=4)
    dev = torch.device("cuda:0")
    tree = colden.Tree(tin, torch.from_numpy(tin.leaf_n).to(dev))
    rng = np.random.default_rng(19)
    tr = oracle.Tree(tin)
    for dname, ns in [("healpix1", 10000), ("healpix2", 3000)]:
        dirs = DIRS[dname]
        D = dirs.shape[0]
        tg = np.concatenate([rng.choice(tin.n_leaf, ns, replace=False), [0, tin.n_leaf - 1]])
        ref = tr.columns(dirs, tg, mode=oracle.INSITU)
        w = colden.Weights(dirs, mode=colden.CD_INSITU)
        N = torch.full((tin.n_leaf, D), float("nan"), dtype=torch.float32, device=dev)
        chi = torch.full((tin.n_leaf,), float("nan"), dtype=torch.float32, device=dev)
        colden.column_densities(tree, w, N, chi)
        idx = torch.from_numpy(tg).to(dev)
        got = N[idx].cpu().numpy().astype(np.float64)
        gchi = chi[idx].cpu().numpy().astype(np.float64)
        rel = np.abs(got - ref) / ref
        print(f"insitu 512^3 {dname}: max rel {rel.max():.3e}")
        assert rel.max() <= REL_FP32
        assert np.abs(gchi - oracle.screening(ref)).max() <= 2e-6
        assert bool(torch.isfinite(N).all())
        w.close()
        del N, chi


@pytest.mark.parametrize("prec,pname", [(1, "bf16x2"), (2, "fp16x2")])
def test_insitu_split_forms(colden, prec, pname):
    tin = synth.workload_uniform(6, sigma=1.5, mean=10.0, seed=33)
    dirs = DIRS["healpix1"]
    N, _ = _run(colden, tin, dirs, colden.CD_INSITU, precision=prec)
    ref = oracle.Tree(tin).columns(dirs, mode=oracle.INSITU)
    err = np.abs(np.log(N) - np.log(ref))
    print(f"insitu {pname}: max |d ln N| {err.max():.3e}")
    assert err.max() <= 1e-3


def test_insitu_differs_from_precalc_as_the_paper_reports(colden):
    """The two schemes share the shells dl = 1..3 and differ beyond: on the
    128^3 field the mean |N_prec - N_insitu| / N_insitu is a few per cent
    (Sect. 4.4 reports 6-7 % for non-axis directions on its clouds) and the
    screening factors agree to a few 1e-3; both GPU forms equal the
    oracle's, so the difference is the method's, not the kernels'."""
    tin = synth.workload_uniform(7, sigma=1.5, mean=10.0, seed=44)
    dirs = DIRS["healpix1"]
    Np, cp = _run(colden, tin, dirs, colden.CD_PRECALC73)
    Ni, ci = _run(colden, tin, dirs, colden.CD_INSITU)
    dN = np.abs(Np - Ni) / Ni
    dchi = np.abs(cp - ci)
    print(f"prec vs insitu: mean dN {dN.mean():.3e} p99 {np.percentile(dN, 99):.3e}; mean dchi {dchi.mean():.3e}")
    assert 1e-4 < dN.mean() < 0.2
    assert dchi.mean() < 0.02


@pytest.mark.parametrize("Lf,B,th,dname", [(6, 3, 14.0, "healpix1"), (6, 2, 14.0, "axes6"), (7, 5, 30.0, "healpix2"),
                                           (7, 5, 30.0, "mn3x8"), (6, 3, 14.0, "rand7"), (6, 3, 14.0, "rand13")])
def test_insitu_amr_parity(colden, Lf, B, th, dname):
    """Adaptive trees: the walk of the shells dl >= 4 per target oct (any
    level), the shells dl = 1..3 from the tiled kernels where the target's
    level has tiles, else from the weight lists (D = 7 and 13 everywhere;
    13 directions leave a last chunk of one direction in the walk kernel)."""
    tin = synth.amr_tree(synth.lognormal_field(1 << Lf, 2.0, 10.0, 50 + B), B, th, 10 * synth.PC_CM)
    assert tin.max_level > tin.base_level
    dirs = DIRS[dname] if dname in DIRS else _rand_dirs(int(dname[4:]), 3)
    N, chi = _run(colden, tin, dirs, colden.CD_INSITU)
    ref = oracle.Tree(tin).columns(dirs, mode=oracle.INSITU)
    rel = np.abs(N - ref) / ref
    print(f"insitu AMR {Lf}/{B} {dname} ({tin.n_leaf} leaves): max rel {rel.max():.3e}")
    assert np.isfinite(N).all()
    assert rel.max() <= REL_FP32
    assert np.abs(chi - oracle.screening(ref)).max() <= 2e-6


@pytest.mark.parametrize("prec,pname", [(1, "bf16x2"), (2, "fp16x2")])
def test_insitu_amr_split_forms(colden, prec, pname):
    tin = synth.amr_tree(synth.lognormal_field(128, 2.0, 10.0, 55), 5, 30.0, 10 * synth.PC_CM)
    dirs = DIRS["healpix1"]
    N, _ = _run(colden, tin, dirs, colden.CD_INSITU, precision=prec)
    ref = oracle.Tree(tin).columns(dirs, mode=oracle.INSITU)
    err = np.abs(np.log(N) - np.log(ref))
    print(f"insitu AMR {pname}: max |d ln N| {err.max():.3e}")
    assert err.max() <= 1e-3


def test_insitu_amr_c3_sampled(colden):
    """The 128^3-base, 512^3-finest clump workload (base 7, Lmax 9), 48
    directions, sampled leaves of every level."""
    tin = synth.workload_amr(7, 9)
    dirs = DIRS["healpix2"]
    N, chi = _run(colden, tin, dirs, colden.CD_INSITU)
    rng = np.random.default_rng(9)
    lv = tin.leaf_level
    tg = np.concatenate([rng.choice(np.flatnonzero(lv == l), min(4000, int((lv == l).sum())), replace=False)
                         for l in np.unique(lv)])
    ref = oracle.Tree(tin).columns(dirs, tg, mode=oracle.INSITU)
    rel = np.abs(N[tg] - ref) / ref
    print(f"insitu C3: {tg.size} leaves, max rel {rel.max():.3e}")
    assert np.isfinite(N).all()
    assert rel.max() <= REL_FP32
    assert np.abs(chi[tg] - oracle.screening(ref)).max() <= 2e-6


def _rand_dirs(D, seed):
    u = np.random.default_rng(seed).normal(size=(D, 3))
    return u / np.linalg.norm(u, axis=1, keepdims=True)


def test_insitu_unsupported_cases(colden):
    dev = torch.device("cuda:0")
    # binary16 on an adaptive tree for a direction count outside the tiled set
    tin = synth.amr_tree(synth.lognormal_field(32, 2.0, 10.0, 5), 3, 14.0, 1e19)
    tree = colden.Tree(tin, torch.from_numpy(tin.leaf_n).to(dev))
    w = colden.Weights(_rand_dirs(7, 4), mode=colden.CD_INSITU, precision=2)
    N = torch.empty((tin.n_leaf, 7), dtype=torch.float32, device=dev)
    with pytest.raises(colden.ColdenError) as e:
        colden.column_densities(tree, w, N)
    assert e.value.rc == colden.CD_EUNSUPPORTED
    # split precision on a uniform grid below 32^3
    tin = synth.workload_uniform(4, seed=1)
    tree = colden.Tree(tin, torch.from_numpy(tin.leaf_n).to(dev))
    w = colden.Weights(DIRS["healpix1"], mode=colden.CD_INSITU, precision=1)
    N = torch.empty((tin.n_leaf, 12), dtype=torch.float32, device=dev)
    with pytest.raises(colden.ColdenError) as e:
        colden.column_densities(tree, w, N)
    assert e.value.rc == colden.CD_EUNSUPPORTED
