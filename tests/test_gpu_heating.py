"""Heating rates from the screening factor (Sect. 5) on the GPU against the
FP64 oracle (oracle/heating.py), through the C ABI, on a 32^3 turbulent
field with synthetic temperature and electron density (the paper takes n_e
from a model it does not state).  Gate: 1e-5 relative (FP32 powf / expf)."""
import numpy as np
import pytest

import oracle
from oracle import heating as H
from paper_1410_0624_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def colden():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1410_0624_amd import colden as c
    c.lib()
    return c


@pytest.fixture(scope="module")
def field(colden):
    tin = synth.workload_uniform(5, sigma=1.5, mean=10.0, seed=1)
    n = tin.leaf_n.astype(np.float64)
    T = np.clip(8000.0 * n ** -0.7, 20.0, 8000.0)   # warm diffuse gas, cold dense gas
    ne = 1e-3 * n + 3e-3 * np.sqrt(n)
    leaf = torch.from_numpy(tin.leaf_n).to(DEV)
    tree = colden.Tree(tin, leaf)
    w = colden.Weights(oracle.dirs_healpix(1))
    N = torch.empty((tin.n_leaf, 12), dtype=torch.float32, device=DEV)
    chi = torch.empty(tin.n_leaf, dtype=torch.float32, device=DEV)
    colden.column_densities(tree, w, N, chi)
    torch.cuda.synchronize()
    f32 = lambda a: torch.from_numpy(np.asarray(a, np.float32)).to(DEV)
    return tin, N, chi, f32(n), f32(T), f32(ne), n, T, ne


def _rel(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def test_heating_from_chi(colden, field):
    tin, N, chi, n, T, ne, n64, T64, ne64 = field
    uv = torch.empty_like(chi)
    g = torch.empty_like(chi)
    cr = torch.empty_like(chi)
    colden.heating_rates(chi, n, T, ne, uv, g0eff=g, gamma_cr=cr)
    torch.cuda.synchronize()
    c64 = chi.cpu().numpy().astype(np.float64)
    gr, uvr, crr = H.rates(c64, n.cpu().numpy().astype(np.float64), T.cpu().numpy().astype(np.float64),
                           ne.cpu().numpy().astype(np.float64))
    e = _rel(uv.cpu().numpy().astype(np.float64), uvr)
    print(f"Gamma_UV max rel {e.max():.2e}; range {uvr.min():.2e} .. {uvr.max():.2e} erg cm^-3 s^-1")
    assert e.max() <= 1e-5
    assert _rel(g.cpu().numpy().astype(np.float64), gr).max() <= 1e-6
    assert _rel(cr.cpu().numpy().astype(np.float64), crr).max() <= 1e-6


def test_screening_heating_fused(colden, field):
    tin, N, chi, n, T, ne, *_ = field
    uv = torch.empty_like(chi)
    chi2 = torch.empty_like(chi)
    colden.screening_heating(N, n, T, ne, uv, chi=chi2)
    torch.cuda.synchronize()
    chi_ref = oracle.screening(N.cpu().numpy().astype(np.float64))
    assert np.abs(chi2.cpu().numpy() - chi_ref).max() <= 1e-6
    _, uvr, _ = H.rates(chi_ref, n.cpu().numpy().astype(np.float64), T.cpu().numpy().astype(np.float64),
                        ne.cpu().numpy().astype(np.float64))
    assert _rel(uv.cpu().numpy().astype(np.float64), uvr).max() <= 2e-5


def test_heating_limits_and_errors(colden):
    chi = torch.tensor([0.0, 1.0, 1.0, 0.5], device=DEV)
    n = torch.tensor([10.0, 10.0, 10.0, 0.0], device=DEV)
    T = torch.tensor([100.0, 100.0, 0.0, 100.0], device=DEV)
    ne = torch.tensor([0.01, 0.0, 0.01, 0.01], device=DEV)
    uv = torch.full_like(chi, float("nan"))
    colden.heating_rates(chi, n, T, ne, uv)
    torch.cuda.synchronize()
    got = uv.cpu().numpy()
    assert got[0] == 0.0          # fully screened
    assert got[1] == 0.0          # UV but no electrons: eps = 0
    np.testing.assert_allclose(got[2], 1e-24 * 4.9e-2 * 1.7 * 10.0, rtol=1e-6)  # T = 0: x = 0, second term 0
    assert got[3] == 0.0          # no gas
    colden.heating_rates(chi[:0], n[:0], T[:0], ne[:0], uv[:0])
    with pytest.raises(colden.ColdenError) as e:
        colden.heating_rates(chi, n, T, ne, uv, G0=-1.0)
    assert e.value.rc == colden.CD_EINVAL
