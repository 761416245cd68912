"""Split-precision (bf16 / fp16 hi + lo on the matrix cores) sweeps against
the FP64 oracle, through the C ABI.  Gate: max |ln N_gpu - ln N_oracle| <= 1e-3
over every checked output; the measured error is printed per case, next to
the FP32 sweep's."""
import os

import numpy as np
import pytest

import oracle
from paper_1410_0624_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LN_GATE = 1e-3


@pytest.fixture(scope="module")
def colden():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1410_0624_amd import colden as c
    c.lib()
    return c


def _run(colden, tin, dirs, precision, chi=True):
    dev = torch.device("cuda:0")
    leaf = torch.from_numpy(tin.leaf_n).to(dev)
    tree = colden.Tree(tin, leaf)
    w = colden.Weights(dirs, precision=precision)
    N = torch.full((tin.n_leaf, dirs.shape[0]), float("nan"), dtype=torch.float32, device=dev)
    c = torch.full((tin.n_leaf,), float("nan"), dtype=torch.float32, device=dev) if chi else None
    colden.column_densities(tree, w, N, c)
    torch.cuda.synchronize()
    return N.cpu().numpy().astype(np.float64), (c.cpu().numpy().astype(np.float64) if chi else None)


def _lnerr(a, b):
    return np.abs(np.log(a) - np.log(b))


PREC = {"bf16x2": 1, "fp16x2": 2}


@pytest.mark.parametrize("pname", ["bf16x2", "fp16x2"])
@pytest.mark.parametrize("L,dname", [(5, "healpix1"), (6, "healpix2"), (6, "axes6"), (7, "healpix1"), (6, "mn7x12")])
def test_split_uniform_all_leaves(colden, pname, L, dname):
    tin = synth.workload_uniform(L, sigma=1.5, mean=10.0, seed=40 + L)
    dirs = {"healpix1": oracle.dirs_healpix(1), "healpix2": oracle.dirs_healpix(2),
            "axes6": oracle.dirs_axes6(), "mn7x12": oracle.dirs_mn(7, 12)}[dname]
    N, chi = _run(colden, tin, dirs, PREC[pname])
    Nf, _ = _run(colden, tin, dirs, 0, chi=False)
    ref = oracle.Tree(tin).columns(dirs)
    assert np.isfinite(N).all() and (N > 0).all()
    err = _lnerr(N, ref)
    print(f"{pname} L={L} {dname}: max |d ln N| {err.max():.3e} mean {err.mean():.3e} "
          f"(FP32 {_lnerr(Nf, ref).max():.3e})")
    assert err.max() <= LN_GATE
    assert np.abs(chi - oracle.screening(ref)).max() <= 1e-3


@pytest.mark.parametrize("pname", ["bf16x2", "fp16x2"])
def test_split_c2_256_sampled(colden, pname):
    tin = synth.workload_uniform(8, sigma=1.5, mean=10.0, seed=2)
    dirs = oracle.dirs_healpix(1)
    N, _ = _run(colden, tin, dirs, PREC[pname], chi=False)
    assert np.isfinite(N).all() and (N > 0).all()
    tg = np.random.default_rng(5).choice(tin.n_leaf, 30000, replace=False)
    ref = oracle.Tree(tin).columns(dirs, tg)
    err = _lnerr(N[tg], ref)
    print(f"{pname} 256^3 sampled: max |d ln N| {err.max():.3e} mean {err.mean():.3e}")
    assert err.max() <= LN_GATE


@pytest.mark.parametrize("pname,Lf,B,th,seed,dname", [
    # base level < 5: targets of levels without tiles and of sparse tiles
    # gathered in FP32, dense tiles on the matrix cores
    ("bf16x2", 6, 3, 14.0, 5, "healpix1"), ("bf16x2", 7, 4, 30.0, 5, "healpix2"), ("bf16x2", 7, 2, 30.0, 6, "healpix1"),
    ("fp16x2", 6, 3, 14.0, 5, "healpix1"), ("fp16x2", 7, 4, 30.0, 5, "healpix2"),
    ("fp16x2", 4, 2, 8.0, 9, "healpix1"),  # no 16^3-oct tile: every target gathered in FP32
    # base level >= 5
    ("bf16x2", 7, 5, 30.0, 7, "healpix2"), ("fp16x2", 7, 5, 30.0, 7, "healpix2"),
    ("fp16x2", 7, 6, 14.0, 8, "healpix1"),
    # the paper's 7 x 12 set (84 directions) on the tiled path
    ("bf16x2", 7, 5, 30.0, 7, "mn7x12"), ("fp16x2", 7, 5, 30.0, 7, "mn7x12"),
    # direction counts outside the tiled set: every target on the matrix cores, grouped (bf16 only)
    ("bf16x2", 6, 3, 14.0, 5, "rand7"), ("bf16x2", 7, 5, 30.0, 7, "rand13")])
def test_split_amr_all_leaves(colden, pname, Lf, B, th, seed, dname):
    tin = synth.amr_tree(synth.lognormal_field(1 << Lf, 2.0, 10.0, seed), B, th, 10 * synth.PC_CM)
    dirs = {"healpix1": oracle.dirs_healpix(1), "healpix2": oracle.dirs_healpix(2),
            "rand7": _rand_dirs(7, 11), "rand13": _rand_dirs(13, 12), "mn7x12": oracle.dirs_mn(7, 12)}[dname]
    N, chi = _run(colden, tin, dirs, PREC[pname])
    ref = oracle.Tree(tin).columns(dirs)
    err = _lnerr(N, ref)
    print(f"{pname} AMR {Lf}/{B}/{th} {dname}: max |d ln N| {err.max():.3e} mean {err.mean():.3e}")
    assert err.max() <= LN_GATE
    assert np.abs(chi - oracle.screening(ref)).max() <= 1e-3


@pytest.mark.parametrize("pname", ["bf16x2", "fp16x2"])
def test_split_c3_amr_sampled(colden, pname):
    """The AMR workload (128^3 base + 2 levels, D = 48) in both split forms."""
    tin = synth.workload_amr()
    dirs = oracle.dirs_healpix(2)
    N, _ = _run(colden, tin, dirs, PREC[pname], chi=False)
    assert np.isfinite(N).all() and (N > 0).all()
    rng = np.random.default_rng(2)
    tg = np.concatenate([rng.choice(np.nonzero(tin.leaf_level == l)[0], 8000, replace=False)
                         for l in range(tin.base_level, tin.max_level + 1)])
    ref = oracle.Tree(tin).columns(dirs, tg)
    err = _lnerr(N[tg], ref)
    print(f"{pname} C3 sampled: max |d ln N| {err.max():.3e} mean {err.mean():.3e}")
    assert err.max() <= LN_GATE


@pytest.fixture(scope="module")
def c4(colden):
    """The 512^3 workload (134M leaves, sigma_ln n = 1.5, mean 10, seed 4) on
    the GPU, with leaves sampled in every z plane (so every z-slab boundary
    of the sweep is covered, whatever the slab count) plus the 8 corners."""
    tin = synth.workload_uniform(9, sigma=1.5, mean=10.0, seed=4)
    n = 512
    rng = np.random.default_rng(9)
    z = np.repeat(np.arange(n), 40)
    tg = (z * n + rng.integers(0, n, z.size)) * n + rng.integers(0, n, z.size)
    corners = [((k * n + j) * n + i) for k in (0, n - 1) for j in (0, n - 1) for i in (0, n - 1)]
    tg = np.unique(np.concatenate([tg, corners])).astype(np.int64)
    dev = torch.device("cuda:0")
    leaf = torch.from_numpy(tin.leaf_n).to(dev)
    tree = colden.Tree(tin, leaf, max_dirs=48)
    yield tin, leaf, tree, tg
    tree.close()


@pytest.mark.parametrize("nside", [1, 2])
def test_c4_512_all_forms_sampled(colden, c4, nside):
    """The 512^3 workload with 12 and 48 sectors in the launch configuration
    the benchmark times, all three forms against the oracle (Sect. 3.3, Eq. 11)
    on 20k leaves sampled across every z plane and the box corners; chi from
    the fused epilogue against the oracle's screening of its columns."""
    tin, leaf, tree, tg = c4
    dirs = oracle.dirs_healpix(nside)
    D = dirs.shape[0]
    ref = oracle.Tree(tin).columns(dirs, tg)
    chi_ref = oracle.screening(ref)
    dev = torch.device("cuda:0")
    N = torch.empty((tin.n_leaf, D), dtype=torch.float32, device=dev)
    chi = torch.empty(tin.n_leaf, dtype=torch.float32, device=dev)
    idx = torch.from_numpy(tg).to(dev)
    for pname, prec, gate in [("fp32", 0, None), ("bf16x2", 1, LN_GATE), ("fp16x2", 2, LN_GATE)]:
        w = colden.Weights(dirs, precision=prec)
        N.fill_(float("nan"))
        chi.fill_(float("nan"))
        colden.column_densities(tree, w, N, chi)
        got = N[idx].cpu().numpy().astype(np.float64)
        gchi = chi[idx].cpu().numpy().astype(np.float64)
        assert np.isfinite(got).all()
        err = _lnerr(got, ref)
        rel = np.abs(got - ref) / ref
        dchi = np.abs(gchi - chi_ref).max()
        print(f"512^3 D={D} {pname}: max rel {rel.max():.3e}, max |d ln N| {err.max():.3e}, max |d chi| {dchi:.2e}",
              flush=True)
        if gate is None:
            assert rel.max() <= 1e-5
            assert dchi <= 1e-5
        else:
            assert err.max() <= gate
            assert dchi <= 1e-3
        w.close()
        # every output written (the slabs tile the grid): no NaN left anywhere
        assert not torch.isnan(N).any()
        assert not torch.isnan(chi).any()
    del N, chi
    torch.cuda.empty_cache()


@pytest.mark.parametrize("m,nphi", [(3, 8), (5, 8)])
def test_c4_512_other_direction_counts(colden, c4, m, nphi):
    """The 512^3 workload with the paper's M x N sets of 24 and 40 directions
    (Sect. 3.2, Eqs. 5-6), FP32: the coarse tables of levels 4 and 5 with a
    lane per cell (216 and 64 state codes) and the matrix-core rows at these
    direction counts, on the 20k leaves sampled across every z plane and the
    corners, against the oracle (Sect. 3.3, Eq. 11) at 1e-5."""
    tin, leaf, tree, tg = c4
    dirs = oracle.dirs_mn(m, nphi)
    D = dirs.shape[0]
    ref = oracle.Tree(tin).columns(dirs, tg)
    dev = torch.device("cuda:0")
    N = torch.full((tin.n_leaf, D), float("nan"), dtype=torch.float32, device=dev)
    chi = torch.full((tin.n_leaf,), float("nan"), dtype=torch.float32, device=dev)
    w = colden.Weights(dirs)
    colden.column_densities(tree, w, N, chi)
    idx = torch.from_numpy(tg).to(dev)
    got = N[idx].cpu().numpy().astype(np.float64)
    gchi = chi[idx].cpu().numpy().astype(np.float64)
    assert not torch.isnan(N).any() and not torch.isnan(chi).any()
    w.close()
    del N, chi
    torch.cuda.empty_cache()
    rel = np.abs(got - ref) / ref
    dchi = np.abs(gchi - oracle.screening(ref)).max()
    print(f"512^3 M x N = {m} x {nphi} (D={D}) fp32: max rel {rel.max():.3e}, max |d chi| {dchi:.2e}", flush=True)
    assert rel.max() <= 1e-5
    assert dchi <= 1e-5


def test_c4_512_fp32_million_sampled(colden, c4):
    """The default benchmark's case (512^3, 48 sectors, FP32, the row kernel
    in one launch over the grid) on 2^20 leaves: 131,072 random octs with all
    8 of their leaves, every output against the oracle (Sect. 3.3, Eq. 11)
    at 1e-5, chi at 1e-5."""
    tin, leaf, tree, _ = c4
    dirs = oracle.dirs_healpix(2)
    n1 = 256
    octs = np.random.default_rng(21).choice(n1 ** 3, size=1 << 17, replace=False)
    ax, ay, az = octs % n1, (octs // n1) % n1, octs // (n1 * n1)
    tg = np.concatenate([((2 * az + (o >> 2)) * 512 + 2 * ay + ((o >> 1) & 1)) * 512 + 2 * ax + (o & 1)
                         for o in range(8)]).astype(np.int64)
    ref = oracle.Tree(tin).columns(dirs, tg, nthreads=os.cpu_count() or 1)
    dev = torch.device("cuda:0")
    N = torch.empty((tin.n_leaf, 48), dtype=torch.float32, device=dev)
    chi = torch.empty(tin.n_leaf, dtype=torch.float32, device=dev)
    w = colden.Weights(dirs)
    colden.column_densities(tree, w, N, chi)
    idx = torch.from_numpy(tg).to(dev)
    got = N[idx].cpu().numpy().astype(np.float64)
    gchi = chi[idx].cpu().numpy().astype(np.float64)
    w.close()
    del N, chi
    torch.cuda.empty_cache()
    rel = np.abs(got - ref) / ref
    dchi = np.abs(gchi - oracle.screening(ref)).max()
    print(f"512^3 D=48 fp32, {tg.size} leaves: max rel {rel.max():.3e} mean {rel.mean():.3e}, max |d chi| {dchi:.2e}")
    assert rel.max() <= 1e-5
    assert dchi <= 1e-5


def _rand_dirs(D, seed):
    u = np.random.default_rng(seed).normal(size=(D, 3))
    return u / np.linalg.norm(u, axis=1, keepdims=True)


def test_split_unsupported_cases(colden):
    dev = torch.device("cuda:0")
    # binary16 on an adaptive tree for a direction count outside the tiled set
    tin = synth.amr_tree(synth.lognormal_field(32, 2.0, 10.0, 5), 3, 14.0, 1e19)
    tree = colden.Tree(tin, torch.from_numpy(tin.leaf_n).to(dev))
    w = colden.Weights(_rand_dirs(7, 3), precision=2)
    N = torch.empty((tin.n_leaf, 7), dtype=torch.float32, device=dev)
    with pytest.raises(colden.ColdenError) as e:
        colden.column_densities(tree, w, N)
    assert e.value.rc == colden.CD_EUNSUPPORTED
    # uniform grids below 32^3 have no tiled split kernel
    tin = synth.workload_uniform(4, seed=1)
    tree = colden.Tree(tin, torch.from_numpy(tin.leaf_n).to(dev))
    w = colden.Weights(oracle.dirs_healpix(1), precision=1)
    N = torch.empty((tin.n_leaf, 12), dtype=torch.float32, device=dev)
    with pytest.raises(colden.ColdenError) as e:
        colden.column_densities(tree, w, N)
    assert e.value.rc == colden.CD_EUNSUPPORTED
