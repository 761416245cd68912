"""Packed 16-bit output (cd_column_densities_log16): codes c with
N = 2^(40 + c / 1024), through the C ABI.

Gates: every code within 1 of the encoding, on the CPU in FP32, of the
unpacked sweep's FP32 columns on the same tree (the two sides round the
same FP32 logarithm; they may land on either side of a half step); the
decoded columns against the FP64 oracle within the format's 2^-11 in log2
(3.4e-4 in ln N) plus the FP32 sweep's 1e-5; chi identical to the unpacked
sweep's (it is taken from the FP32 columns before packing)."""
import numpy as np
import pytest

import oracle
from paper_1410_0624_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
LN_GATE = np.log(2.0) * 2.0 ** -11 + 1e-5


@pytest.fixture(scope="module")
def colden():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1410_0624_amd import colden as c
    c.lib()
    return c


def _encode(N32):
    """The format's definition, in FP32 on the CPU."""
    x = (np.log2(N32.astype(np.float32)) - np.float32(40.0)) * np.float32(1024.0)
    return np.clip(np.rint(x), 0, 65535).astype(np.int64)


def _both(colden, tin, dirs, precision=0, slab_dirs=None):
    leaf = torch.from_numpy(tin.leaf_n).to(DEV)
    tree = colden.Tree(tin, leaf)
    w = colden.Weights(dirs, precision=precision)
    N = torch.empty((tin.n_leaf, dirs.shape[0]), dtype=torch.float32, device=DEV)
    chi = torch.empty(tin.n_leaf, dtype=torch.float32, device=DEV)
    colden.column_densities(tree, w, N, chi)
    code = torch.full((tin.n_leaf, dirs.shape[0]), -1, dtype=torch.int16, device=DEV)
    chi2 = torch.full((tin.n_leaf,), float("nan"), dtype=torch.float32, device=DEV)
    colden.column_densities_log16(tree, w, code, chi2)
    torch.cuda.synchronize()
    return tree, w, N, chi, code, chi2


@pytest.mark.parametrize("L,nside,precision", [(5, 1, 0), (6, 2, 0), (6, 2, 1), (7, 1, 0)])
def test_log16_codes_every_leaf(colden, L, nside, precision):
    tin = synth.workload_uniform(L, sigma=1.5, mean=10.0, seed=60 + L)
    dirs = oracle.dirs_healpix(nside)
    _, _, N, chi, code, chi2 = _both(colden, tin, dirs, precision)
    c = code.cpu().numpy().astype(np.int64) & 0xFFFF
    want = _encode(N.cpu().numpy())
    diff = np.abs(c - want)
    print(f"L={L} D={dirs.shape[0]} precision {precision}: codes differing by 1: {np.mean(diff == 1):.2e}")
    assert diff.max() <= 1
    assert torch.equal(chi, chi2)
    ref = oracle.Tree(tin).columns(dirs)
    dec = colden.decode_log16(code).cpu().numpy()
    err = np.abs(np.log(dec) - np.log(ref))
    print(f"  decoded vs oracle: max |d ln N| {err.max():.3e} (gate {LN_GATE:.3e})")
    assert err.max() <= LN_GATE + (0 if precision == 0 else 1e-3)


@pytest.mark.parametrize("name,dirs", [("mn3x8", oracle.dirs_mn(3, 8)), ("mn5x8", oracle.dirs_mn(5, 8)),
                                       ("mn7x12", oracle.dirs_mn(7, 12))])
def test_log16_direction_families(colden, name, dirs):
    """24 and 40 directions (the matrix-core rows, whose 16-column tiles
    straddle the pair of x targets) and 84 (the multiply-add rows): every
    code of a 64^3 grid against the FP32 columns' encoding and the oracle."""
    tin = synth.workload_uniform(6, sigma=1.5, mean=10.0, seed=61)
    _, _, N, chi, code, chi2 = _both(colden, tin, dirs)
    c = code.cpu().numpy().astype(np.int64) & 0xFFFF
    assert np.abs(c - _encode(N.cpu().numpy())).max() <= 1
    assert torch.equal(chi, chi2)
    ref = oracle.Tree(tin).columns(dirs)
    err = np.abs(np.log(colden.decode_log16(code).cpu().numpy()) - np.log(ref))
    print(f"{name} D={dirs.shape[0]}: decoded vs oracle max |d ln N| {err.max():.3e}")
    assert err.max() <= LN_GATE


def test_log16_512_sampled(colden):
    """The default benchmark's case (512^3, 48 sectors, four z-slabs):
    codes of sampled leaves in every slab and the corners against the FP64
    oracle, and every code against the encoding of the FP32 columns."""
    L, n = 9, 512
    tin = synth.workload_uniform(L, sigma=1.5, mean=10.0, seed=4)
    dirs = oracle.dirs_healpix(2)
    _, _, N, chi, code, chi2 = _both(colden, tin, dirs)
    assert torch.equal(chi, chi2)
    # every code of the planes on both sides of every slab boundary against
    # the FP32 columns
    zs = [0, 127, 128, 255, 256, 383, 384, 511]
    for z in zs:
        sl = slice(z * n * n, (z + 1) * n * n)
        c = code[sl].cpu().numpy().astype(np.int64) & 0xFFFF
        assert np.abs(c - _encode(N[sl].cpu().numpy())).max() <= 1
    rng = np.random.default_rng(12)
    tg = [((z * n + rng.integers(0, n)) * n + rng.integers(0, n)) for z in zs for _ in range(40)]
    tg += [0, n - 1, n * n - 1, n ** 3 - 1, n ** 3 - n]
    tg = np.array(tg, dtype=np.int64)
    ref = oracle.Tree(tin).columns(dirs, tg, nthreads=8)
    dec = colden.decode_log16(code[torch.from_numpy(tg).to(DEV)]).cpu().numpy()
    err = np.abs(np.log(dec) - np.log(ref))
    print(f"512^3 D=48: decoded vs oracle max |d ln N| {err.max():.3e} over {tg.size} leaves")
    assert err.max() <= LN_GATE


def test_log16_errors(colden):
    tin = synth.workload_uniform(6, seed=3)
    leaf = torch.from_numpy(tin.leaf_n).to(DEV)
    tree = colden.Tree(tin, leaf)
    w6 = colden.Weights(oracle.dirs_axes6())
    with pytest.raises(colden.ColdenError) as e:
        colden.column_densities_log16(tree, w6, torch.empty((tin.n_leaf, 6), dtype=torch.int16, device=DEV))
    assert e.value.rc == colden.CD_EUNSUPPORTED
    w = colden.Weights(oracle.dirs_healpix(1))
    with pytest.raises(ValueError):
        colden.column_densities_log16(tree, w, torch.empty((tin.n_leaf, 12), dtype=torch.float32, device=DEV))
    amr = synth.workload_amr(4, 6, seed=3, threshold=30.0)
    aleaf = torch.from_numpy(amr.leaf_n).to(DEV)
    atree = colden.Tree(amr, aleaf)
    with pytest.raises(colden.ColdenError) as e:
        colden.column_densities_log16(atree, w, torch.empty((amr.n_leaf, 12), dtype=torch.int16, device=DEV))
    assert e.value.rc == colden.CD_EUNSUPPORTED
