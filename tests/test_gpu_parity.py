"""Parity of the HIP path with the FP64 CPU oracle (MI355X).  Every call goes
through the C ABI; the oracle is the FP64 plain implementation in oracle/.
Gate for the FP32 sweep: <= 1e-5 relative per output N_H(t, d)."""
import ctypes

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


def _run(colden, tin, dirs, chi=True, precision=0):
    dev = torch.device("cuda:0")
    leaf = torch.from_numpy(tin.leaf_n).to(dev)
    tree = colden.Tree(tin, leaf)
    w = colden.Weights(dirs, precision=precision)
    N = torch.full((tin.n_leaf, dirs.shape[0]), float("nan"), dtype=torch.float32, device=dev)
    c = torch.full((tin.n_leaf,), float("nan"), dtype=torch.float32, device=dev) if chi else None
    colden.column_densities(tree, w, N, c)
    torch.cuda.synchronize()
    return N.cpu().numpy().astype(np.float64), (c.cpu().numpy().astype(np.float64) if chi else None)


def _rel(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def test_library_directions_match_oracle(colden):
    for args, ref in [((0, 1, 0), oracle.dirs_healpix(1)), ((0, 2, 0), oracle.dirs_healpix(2)),
                      ((1, 3, 4), oracle.dirs_mn(3, 4)), ((1, 5, 8), oracle.dirs_mn(5, 8)),
                      ((1, 7, 12), oracle.dirs_mn(7, 12)), ((2, 0, 0), oracle.dirs_axes6())]:
        np.testing.assert_allclose(colden.directions(*args), ref, atol=1e-15)


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5, 6, 7])
def test_uniform_parity_all_leaves(colden, L):
    """Every output of grids from one oct (2^3) to 128^3, D = 12: spans the
    per-oct shells (dl = 1..3), the first coarse table (L = 6) and the
    216-code coarse recursion (L = 7)."""
    tin = synth.workload_uniform(L, sigma=1.5, mean=10.0, seed=10 + L)
    dirs = oracle.dirs_healpix(1)
    N, chi = _run(colden, tin, dirs)
    tr = oracle.Tree(tin)
    if tin.n_leaf <= 300000:
        tg = np.arange(tin.n_leaf)
    else:
        tg = np.random.default_rng(L).choice(tin.n_leaf, 60000, replace=False)
    ref = tr.columns(dirs, tg)
    rel = _rel(N[tg], ref)
    print(f"L={L}: max rel {rel.max():.3e} mean {rel.mean():.3e}")
    assert np.isfinite(N).all()
    assert rel.max() <= REL_FP32
    chi_ref = oracle.screening(ref)
    assert np.abs(chi[tg] - chi_ref).max() <= 2e-6


@pytest.mark.parametrize("name,dirs", [
    ("healpix2", oracle.dirs_healpix(2)), ("axes6", oracle.dirs_axes6()),
    ("mn3x4", oracle.dirs_mn(3, 4)), ("mn3x8", oracle.dirs_mn(3, 8)), ("mn5x8", oracle.dirs_mn(5, 8)),
    ("mn7x12", oracle.dirs_mn(7, 12))])
def test_direction_families_parity(colden, name, dirs):
    tin = synth.workload_uniform(6, sigma=1.5, mean=10.0, seed=3)
    N, chi = _run(colden, tin, dirs)
    ref = oracle.Tree(tin).columns(dirs)
    rel = _rel(N, ref)
    print(f"{name} D={dirs.shape[0]}: max rel {rel.max():.3e}")
    assert rel.max() <= REL_FP32
    assert np.abs(chi - oracle.screening(ref)).max() <= 2e-6


@pytest.mark.parametrize("name,dirs", [("mn3x8", oracle.dirs_mn(3, 8)), ("mn5x8", oracle.dirs_mn(5, 8))])
def test_matrix_core_rows_one_block_per_wave(colden, name, dirs):
    """32^3 grid: 16 octs per row, so each wave of the matrix-core row kernel
    holds one 16-oct block; 24 and 40 directions (16-column tiles that
    straddle the pair of x targets).  Every output against the oracle."""
    tin = synth.workload_uniform(5, sigma=1.5, mean=10.0, seed=17)
    N, chi = _run(colden, tin, dirs)
    ref = oracle.Tree(tin).columns(dirs)
    rel = _rel(N, ref)
    print(f"{name} D={dirs.shape[0]} 32^3: max rel {rel.max():.3e}")
    assert rel.max() <= REL_FP32
    assert np.abs(chi - oracle.screening(ref)).max() <= 2e-6


def test_sweep_in_z_slabs_128(colden):
    """D = 48 on a 128^3 grid: the FP32 rows in one launch after the
    external stage, the packed rows (16-bit log codes) in 4 z-slabs whose
    row and external kernels overlap; every slab boundary is checked, the
    packed rows within their format's 2^-11 in log2 of the oracle."""
    tin = synth.workload_uniform(7, sigma=1.5, mean=10.0, seed=13)
    dirs = oracle.dirs_healpix(2)
    N, chi = _run(colden, tin, dirs)
    n = 128
    z = np.concatenate([np.arange(n)[::9], [31, 32, 63, 64, 95, 96, 127]])
    rng = np.random.default_rng(6)
    tg = np.unique(np.concatenate([(zz * n + rng.integers(0, n, 40)) * n + rng.integers(0, n, 40) for zz in z]))
    ref = oracle.Tree(tin).columns(dirs, tg)
    rel = _rel(N[tg], ref)
    print(f"slabs D=48 128^3: {tg.size} targets, max rel {rel.max():.3e}")
    assert np.isfinite(N).all()
    assert rel.max() <= REL_FP32
    assert np.abs(chi[tg] - oracle.screening(ref)).max() <= 2e-6

    dev = torch.device("cuda:0")
    leaf = torch.from_numpy(tin.leaf_n).to(dev)
    tree = colden.Tree(tin, leaf)
    w = colden.Weights(dirs)
    code = torch.full((tin.n_leaf, dirs.shape[0]), -1, dtype=torch.int16, device=dev)
    chi2 = torch.full((tin.n_leaf,), float("nan"), dtype=torch.float32, device=dev)
    colden.column_densities_log16(tree, w, code, chi2)
    torch.cuda.synchronize()
    dec = colden.decode_log16(code).cpu().numpy().astype(np.float64)
    err = np.abs(np.log(dec[tg]) - np.log(ref))
    print(f"  packed, 4 slabs: max |d ln N| {err.max():.3e}")
    assert err.max() <= np.log(2.0) * 2.0 ** -11 + REL_FP32
    assert np.abs(chi2.cpu().numpy()[tg] - oracle.screening(ref)).max() <= 2e-6


def test_c2_256_sampled_parity(colden):
    """The 256^3 workload (16.8M leaves, 9-level pyramid, D = 12), in the
    launch configuration the benchmark times: 40k sampled leaves against the
    oracle, and every output finite and positive."""
    tin = synth.workload_uniform(8, sigma=1.5, mean=10.0, seed=2)
    dirs = oracle.dirs_healpix(1)
    N, chi = _run(colden, tin, dirs)
    assert np.isfinite(N).all() and (N > 0).all()
    assert np.isfinite(chi).all() and (chi > 0).all() and (chi <= 1).all()
    tg = np.random.default_rng(0).choice(tin.n_leaf, 40000, replace=False)
    tg = np.concatenate([tg, [0, tin.n_leaf - 1, 255, 256 * 255]])
    ref = oracle.Tree(tin).columns(dirs, tg)
    rel = _rel(N[tg], ref)
    print(f"C2 sampled: max rel {rel.max():.3e} mean {rel.mean():.3e}")
    assert rel.max() <= REL_FP32
    assert np.abs(chi[tg] - oracle.screening(ref)).max() <= 2e-6


def test_uniform_density_closed_form_on_gpu(colden):
    n0 = 4.0
    L = 5
    n = 1 << L
    tin = synth.uniform_tree(np.full((n, n, n), n0), box_cm=synth.PC_CM * 10)
    dirs = oracle.dirs_healpix(2)
    N, _ = _run(colden, tin, dirs, chi=False)
    ref = oracle.Tree(tin).columns(dirs)
    assert _rel(N, ref).max() <= REL_FP32


def test_tree_update_recomputes_pyramid(colden):
    dev = torch.device("cuda:0")
    t1 = synth.workload_uniform(6, seed=31)
    t2 = synth.workload_uniform(6, seed=32)
    dirs = oracle.dirs_healpix(1)
    l1 = torch.from_numpy(t1.leaf_n).to(dev)
    l2 = torch.from_numpy(t2.leaf_n).to(dev)
    tree = colden.Tree(t1, l1)
    w = colden.Weights(dirs)
    N = torch.empty((t1.n_leaf, 12), dtype=torch.float32, device=dev)
    colden.column_densities(tree, w, N)
    tree.update(l2)
    colden.column_densities(tree, w, N)
    torch.cuda.synchronize()
    ref = oracle.Tree(t2).columns(dirs)
    assert _rel(N.cpu().numpy().astype(np.float64), ref).max() <= REL_FP32


def test_screening_factor_kernel(colden):
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(4)
    N = (10 ** rng.uniform(18, 23, size=(5000, 12))).astype(np.float32)
    Nt = torch.from_numpy(N).to(dev)
    chi = torch.empty(5000, dtype=torch.float32, device=dev)
    av = torch.empty((5000, 12), dtype=torch.float32, device=dev)
    colden.screening_factor(Nt, chi, av)
    torch.cuda.synchronize()
    ref = oracle.screening(N.astype(np.float64))
    assert np.abs(chi.cpu().numpy() - ref).max() <= 2e-6
    np.testing.assert_allclose(av.cpu().numpy(), N.astype(np.float64) / 1.87e21, rtol=1e-6)
    # empty input is a no-op
    colden.screening_factor(Nt[:0], chi[:0])


def test_invalid_densities_are_rejected(colden):
    """Negative, NaN or infinite leaf densities: cd_build_tree returns
    CD_EINVAL (uniform and AMR); cd_check_densities counts them exactly;
    -0.0 and subnormals are valid."""
    dev = torch.device("cuda:0")
    tin = synth.workload_uniform(5, seed=2)
    base = torch.from_numpy(tin.leaf_n).to(dev)
    assert colden.check_densities(base) == 0
    for bad in (float("nan"), -1e-30, float("inf"), float("-inf")):
        leaf = base.clone()
        leaf[[7, 4000, 32767]] = bad
        assert colden.check_densities(leaf) == 3
        with pytest.raises(colden.ColdenError) as e:
            colden.Tree(tin, leaf)
        assert e.value.rc == colden.CD_EINVAL
    ok = base.clone()
    ok[0] = -0.0
    ok[1] = 1e-44  # subnormal
    assert colden.check_densities(ok) == 0
    colden.Tree(tin, ok)
    assert colden.check_densities(ok[:0]) == 0
    tin = synth.amr_tree(synth.lognormal_field(32, 2.0, 10.0, 5), 3, 14.0, 1e19)
    leaf = torch.from_numpy(tin.leaf_n).to(dev)
    leaf[tin.n_leaf - 1] = float("nan")
    with pytest.raises(colden.ColdenError) as e:
        colden.Tree(tin, leaf)
    assert e.value.rc == colden.CD_EINVAL


def test_error_paths(colden):
    with pytest.raises(colden.ColdenError) as e:
        colden.Weights(np.zeros((0, 3)))
    assert e.value.rc == colden.CD_EINVAL
    with pytest.raises(colden.ColdenError) as e:
        colden.Weights(np.array([[1.0, 1.0, 0.0]]))
    assert e.value.rc == colden.CD_EINVAL
    with pytest.raises(colden.ColdenError):
        colden.directions(7, 1, 1)
    dev = torch.device("cuda:0")
    tin = synth.workload_uniform(3, seed=1)
    leaf = torch.from_numpy(tin.leaf_n[:-1].copy()).to(dev)
    with pytest.raises(colden.ColdenError) as e:  # the structure needs one leaf more
        colden.Tree(tin, leaf)
    assert e.value.rc == colden.CD_EINVAL
    # the library checks it too: cd_tree_update with a wrong leaf count
    full = torch.from_numpy(tin.leaf_n).to(dev)
    tree = colden.Tree(tin, full)
    rc = colden.lib().cd_tree_update(tree.h, ctypes.c_void_p(full.data_ptr()), tin.n_leaf - 1,
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == colden.CD_EINVAL
    with pytest.raises(ValueError):
        tree.update(leaf)
    w = colden.Weights(oracle.dirs_healpix(1))
    with pytest.raises(ValueError):  # N of the wrong shape
        colden.column_densities(tree, w, torch.empty((tin.n_leaf, 11), dtype=torch.float32, device=dev))
    with pytest.raises(ValueError):  # chi of the wrong length
        colden.column_densities(tree, w, torch.empty((tin.n_leaf, 12), dtype=torch.float32, device=dev),
                                torch.empty(tin.n_leaf - 1, dtype=torch.float32, device=dev))


def _build_raw(colden, tin, leaf, max_dirs, ws):
    """cd_build_tree through the ABI with a caller-chosen workspace tensor."""
    par = [np.ascontiguousarray(p, dtype=np.int32) for p in tin.oct_parents]
    n_octs = np.array([p.shape[0] for p in par] + [0], dtype=np.int64)
    ptrs = (ctypes.c_void_p * (len(par) + 1))(*[p.ctypes.data for p in par], None)
    h = ctypes.c_void_p()
    rc = colden.lib().cd_build_tree(float(tin.box_cm), int(tin.base_level), int(tin.max_level),
                                    n_octs.ctypes.data_as(ctypes.c_void_p) if par else None,
                                    ctypes.cast(ptrs, ctypes.c_void_p), ctypes.c_void_p(leaf.data_ptr()),
                                    int(tin.n_leaf), max_dirs, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("amr", [False, True])
def test_sweep_runs_in_the_callers_workspace(colden, amr):
    """Every device buffer of the sweep is the caller's: the tree in a torch
    workspace of exactly the queried size (one byte less is refused), the
    weights likewise; the sweep with and without the caller's second stream
    gives the oracle's columns; more directions than max_dirs are refused."""
    dev = torch.device("cuda:0")
    if amr:
        tin = synth.amr_tree(synth.lognormal_field(64, 2.0, 10.0, 7), 4, 14.0, 10 * synth.PC_CM)
    else:
        tin = synth.workload_uniform(6, seed=5)
    leaf = torch.from_numpy(tin.leaf_n).to(dev)
    dirs = oracle.dirs_healpix(1)
    ref = oracle.Tree(tin).columns(dirs)
    par = [np.ascontiguousarray(p, dtype=np.int32) for p in tin.oct_parents]
    n_octs = np.array([p.shape[0] for p in par] + [0], dtype=np.int64)
    ptrs = (ctypes.c_void_p * (len(par) + 1))(*[p.ctypes.data for p in par], None)
    nb = ctypes.c_size_t(0)
    assert colden.lib().cd_tree_workspace_bytes(int(tin.base_level), int(tin.max_level),
                                                n_octs.ctypes.data_as(ctypes.c_void_p) if par else None,
                                                ctypes.cast(ptrs, ctypes.c_void_p), int(tin.n_leaf), 12,
                                                ctypes.byref(nb)) == 0
    small = torch.empty(nb.value - 1, dtype=torch.uint8, device=dev)
    rc, _ = _build_raw(colden, tin, leaf, 12, small)
    assert rc == colden.CD_EINVAL and "too small" in colden.lib().cd_last_error().decode()
    del small
    for aux in (False, True):
        tree = colden.Tree(tin, leaf, max_dirs=12, aux_stream=aux)
        assert tree.workspace.numel() == nb.value
        w = colden.Weights(dirs)
        N = torch.empty((tin.n_leaf, 12), dtype=torch.float32, device=dev)
        chi = torch.empty(tin.n_leaf, dtype=torch.float32, device=dev)
        colden.column_densities(tree, w, N, chi)
        torch.cuda.synchronize()
        got = N.cpu().numpy().astype(np.float64)
        rel = np.abs(got - ref) / ref
        print(f"{'amr' if amr else 'uniform'} aux={aux}: max rel {rel.max():.2e}")
        assert rel.max() <= 1e-5
        w48 = colden.Weights(oracle.dirs_healpix(2))
        with pytest.raises(colden.ColdenError) as e:
            colden.column_densities(tree, w48, torch.empty((tin.n_leaf, 48), dtype=torch.float32, device=dev))
        assert e.value.rc == colden.CD_EINVAL
        tree.close()


def test_misaligned_buffers_are_rejected(colden):
    """The kernels move N in 16-byte and chi and uniform leaves in 8-byte
    vectors: views that start one float into an allocation are refused."""
    dev = torch.device("cuda:0")
    tin = synth.workload_uniform(5, seed=3)
    D = 12
    leaf_buf = torch.empty(tin.n_leaf + 1, dtype=torch.float32, device=dev)
    leaf_buf[1:] = torch.from_numpy(tin.leaf_n).to(dev)
    with pytest.raises(colden.ColdenError) as e:
        colden.Tree(tin, leaf_buf[1:])
    assert e.value.rc == colden.CD_EINVAL
    tree = colden.Tree(tin, torch.from_numpy(tin.leaf_n).to(dev))
    with pytest.raises(colden.ColdenError) as e:
        tree.update(leaf_buf[1:])
    assert e.value.rc == colden.CD_EINVAL
    w = colden.Weights(oracle.dirs_healpix(1))
    nbuf = torch.empty(tin.n_leaf * D + 4, dtype=torch.float32, device=dev)
    cbuf = torch.empty(tin.n_leaf + 1, dtype=torch.float32, device=dev)
    N_bad = nbuf[1:1 + tin.n_leaf * D].view(tin.n_leaf, D)
    with pytest.raises(colden.ColdenError) as e:
        colden.column_densities(tree, w, N_bad)
    assert e.value.rc == colden.CD_EINVAL
    N_ok = nbuf[4:].view(tin.n_leaf, D)
    with pytest.raises(colden.ColdenError) as e:
        colden.column_densities(tree, w, N_ok, cbuf[1:])
    assert e.value.rc == colden.CD_EINVAL
    # the aligned views are accepted and give the oracle's columns
    colden.column_densities(tree, w, N_ok, cbuf[:-1])
    torch.cuda.synchronize()
    ref = oracle.Tree(tin).columns(oracle.dirs_healpix(1))
    got = N_ok.cpu().numpy().astype(np.float64)
    assert (np.abs(got - ref) / ref).max() <= 1e-5
