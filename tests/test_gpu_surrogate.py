"""The learned surrogate on the GPU, through the C ABI, against the FP64
reference in oracle/surrogate.py, the oracle's shell sums and the method
itself (networks for 256^3 grids; the 512^3 case is in
test_gpu_surrogate_512.py).

Gates: features and targets to 2e-5 (ln units); forward and gradients of
the FP32 checking path to 1e-5 against the FP64 reference; after the
sampled check and fallback, the 99th percentile of the relative chi error
<= 3 %."""
import os
import tempfile

import numpy as np
import pytest

import oracle
from oracle import surrogate as S
from paper_1410_0624_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def colden():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1410_0624_amd import colden as c
    c.lib()
    return c


DEV = "cuda:0"


def _field(seed, L=8):
    return synth.workload_uniform(L, sigma=1.5, mean=10.0, seed=seed)


def _plain(colden, tin, w):
    leaf = torch.from_numpy(tin.leaf_n).to(DEV)
    tree = colden.Tree(tin, leaf)
    N = torch.empty((tin.n_leaf, w.D), dtype=torch.float32, device=DEV)
    chi = torch.empty(tin.n_leaf, dtype=torch.float32, device=DEV)
    colden.column_densities(tree, w, N, chi)
    torch.cuda.synchronize()
    return tree, leaf, N, chi


def _blocks(flat, W, D):
    return S.unflatten(np.asarray(flat, np.float64), W, D)


def test_features_match_reference(colden):
    tin = _field(100)
    w = colden.Weights(oracle.dirs_healpix(1))
    tree, leaf, _, _ = _plain(colden, tin, w)
    n = 256
    rng = np.random.default_rng(1)
    cells = np.concatenate([[0, n ** 3 - 1, 255, n * n * 255], rng.choice(n ** 3, 600, replace=False)])
    s = colden.Surrogate(12, 64, colden.CD_SURR_FP32, 0, norm=(1.0, 2.0, 0.0, 1.0))
    X = torch.empty((cells.size, 576), dtype=torch.float32, device=DEV)
    s.features(tree, torch.from_numpy(cells).to(DEV), X)
    torch.cuda.synchronize()
    lv = S.pyramid(tin.leaf_n.reshape(n, n, n).astype(np.float64))
    ref = S.features(lv, cells, 1.0, 2.0)
    err = np.abs(X.cpu().numpy() - ref).max()
    print(f"features: max abs diff {err:.2e}")
    assert err <= 2e-5
    # an index that is not a leaf gives NaN, not an access
    bad = torch.tensor([-1, n ** 3], dtype=torch.int64, device=DEV)
    Xb = torch.zeros((2, 576), dtype=torch.float32, device=DEV)
    s.features(tree, bad, Xb)
    assert torch.isnan(Xb).all()


@pytest.mark.parametrize("prec", [0, 1])
def test_forward_and_gradients_match_reference(colden, prec):
    """Forward: the FP32 path against the FP64 reference to 1e-5; the
    bfloat16 inference path against the reference rounded where it rounds
    to 1e-2.  Gradients (both precisions: the bfloat16 network trains on
    hi + lo operand pairs) against the exact FP64 backward, element by
    element: |g - g_ref| <= tol (|g_ref| + 1e-3 max |g_ref| of the block).
    FP32: sums of up to 576 terms carry up to 576 * 2^-24 = 3.4e-5 of the
    sum of their magnitudes, which near the floor is up to ~10 times the
    element, three layers deep: tol = 1e-3.  bfloat16 pairs: about 2^-15
    per product before accumulation: tol = 1e-2."""
    W, D, n = 64, 12, 300
    s = colden.Surrogate(D, W, prec, 7)
    p = _blocks(s.get_params(), W, D)
    rng = np.random.default_rng(2)
    X = rng.normal(0, 1, (n, 576))
    T = rng.normal(0, 1, (n, D))
    Xd = torch.from_numpy(X.astype(np.float32)).to(DEV)
    Td = torch.from_numpy(T.astype(np.float32)).to(DEV)
    Y = torch.empty((n, D), dtype=torch.float32, device=DEV)
    s.forward(Xd, Y)
    torch.cuda.synchronize()
    Xr = X.astype(np.float32).astype(np.float64)
    Yref, cache = S.forward(p, Xr)
    if prec == 1:
        yerr = np.abs(Y.cpu().numpy() - S.forward_bf16(p, Xr)).max() / np.abs(Yref).max()
    else:
        yerr = np.abs(Y.cpu().numpy() - Yref).max() / np.abs(Yref).max()
    g, loss = s.gradients(Xd, Td)
    Tr = T.astype(np.float32).astype(np.float64)
    gexact = S.backward(p, cache, Yref, Tr)
    lref = S.mse(Yref, Tr)
    got = _blocks(g, W, D)
    tol = 1e-3 if prec == 0 else 1e-2
    elem = [float((np.abs(a - b) / (np.abs(b) + 1e-3 * np.abs(b).max())).max()) for a, b in zip(got, gexact)]
    norm = [float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(got, gexact)]
    diag = ""
    if prec == 1:  # what single bfloat16 operands would give (not a gate)
        gb = S.backward_bf16(p, Xr, Tr)
        diag = f"; single-bf16 reference vs exact {np.round([float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(gb, gexact)], 4)}"
    print(f"prec {prec}: forward {yerr:.2e}, loss {loss:.7f} vs {lref:.7f}, gradient vs exact FP64 per element "
          f"{np.round(elem, 6)}, per block norm {np.round(norm, 7)}{diag}")
    assert yerr <= (1e-5 if prec == 0 else 1e-2)
    assert abs(loss - lref) <= 1e-5 * lref
    assert max(elem) <= tol


def test_adam_step_matches_reference(colden):
    """One training step of the FP32 path: features, targets (the method's
    near shells dl = 1..3 against the oracle's), gradient and the Adam
    update against the reference."""
    tin = _field(101)
    w = colden.Weights(oracle.dirs_healpix(1))
    tree, leaf, N, _ = _plain(colden, tin, w)
    W, D, lr = 32, 12, 1e-3
    norm = (1.2, 1.5, 46.0, 1.0)
    s = colden.Surrogate(D, W, colden.CD_SURR_FP32, 3, norm=norm)
    p0 = s.get_params().astype(np.float64)
    cells = np.random.default_rng(3).choice(tin.n_leaf, 512, replace=False)
    dcells = torch.from_numpy(cells).to(DEV)
    Tg = torch.empty((cells.size, D), dtype=torch.float32, device=DEV)
    s.targets(tree, w, dcells, Tg)
    s.train_step(tree, w, dcells, lr)
    p1 = s.get_params().astype(np.float64)
    n = 256
    lv = S.pyramid(tin.leaf_n.reshape(n, n, n).astype(np.float64))
    X = S.features(lv, cells, norm[0], norm[1])
    T = S.targets(oracle.Tree(tin).external(oracle.dirs_healpix(1), cells, 1, 3), norm[2], norm[3])
    terr = np.abs(Tg.cpu().numpy() - T).max()
    print(f"targets: max abs diff {terr:.2e}")
    assert terr <= 2e-5
    params = S.unflatten(p0, W, D)
    Y, cache = S.forward(params, X)
    g = S.flatten(S.backward(params, cache, Y, T))
    pref, _, _ = S.adam_step(p0, g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    d = np.abs(p1 - pref)
    # first Adam step is -lr sign(g) (up to eps): only gradients within
    # rounding of zero may differ, by at most 2 lr
    close = d <= 1e-6 * np.abs(p0) + 1e-3 * lr
    print(f"Adam step: {np.mean(~close):.2e} of parameters differ, max diff {d.max():.2e}")
    assert np.mean(~close) <= 1e-3 and d.max() <= 2.001 * lr


@pytest.fixture(scope="module")
def trained(colden):
    """A bfloat16 network for 256^3 grids trained on two seeded 256^3 fields."""
    from paper_1410_0624_amd import surrogate_train
    w = colden.Weights(oracle.dirs_healpix(1))
    runs = [_plain(colden, _field(sd), w) for sd in (110, 111)]
    fields = [surrogate_train.label_field(_field(sd), w, 8, DEV) for sd in (110, 111)]
    nrm = surrogate_train.norms(fields)
    s = colden.Surrogate(12, 256, colden.CD_SURR_BF16, 11, norm=nrm)
    untrained = s.get_params()
    log = surrogate_train.fit(s, fields, steps=2000, batch=4096, lr=2e-3, lr_final=1e-4, seed=5, log_every=250)
    del fields
    print("training log:", [(k, round(l, 4)) for k, l in log])
    return s, w, nrm, untrained, log, runs


def _chi_err(a, b):
    return np.abs(a - b) / b


def test_training_lowers_the_loss_and_beats_baselines(colden, trained):
    """What the network gains: on an unseen field its chi error is far below
    that of the same network untrained and of the best constant column."""
    s, w, nrm, untrained, log, _ = trained
    assert log[-1][1] < 0.2 * log[0][1]
    tin = _field(120)
    tree, leaf, N, chi = _plain(colden, tin, w)
    Ns = torch.empty_like(N)
    chis = torch.empty_like(chi)
    s.infer(tree, w, Ns, chis)
    torch.cuda.synchronize()
    ref = chi.cpu().numpy()
    e_tr = _chi_err(chis.cpu().numpy(), ref)
    trained_params = s.get_params()
    s.set_params(untrained)
    s.infer(tree, w, Ns, chis)
    torch.cuda.synchronize()
    e_un = _chi_err(chis.cpu().numpy(), ref)
    # best constant near-shell column: every direction at exp(out_shift),
    # plus the method's internal + local part and shells dl >= 4 (the same
    # split as the network's)
    s.set_params(np.concatenate([np.zeros(s.n_params() - 12, np.float32), np.zeros(12, np.float32)]))
    s.infer(tree, w, Ns, chis)
    torch.cuda.synchronize()
    e_cst = _chi_err(chis.cpu().numpy(), ref)
    s.set_params(trained_params)
    q = lambda e: (float(np.mean(e)), float(np.percentile(e, 99)))
    print(f"chi error mean/p99: trained {q(e_tr)}, untrained {q(e_un)}, constant {q(e_cst)}")
    assert np.percentile(e_tr, 99) < 0.5 * np.percentile(e_un, 99)
    assert np.percentile(e_tr, 99) < 0.5 * np.percentile(e_cst, 99)


def test_infer_matches_features_and_forward(colden, trained):
    """Inference (network once per level-7 cell on the logarithms taken once
    per pyramid cell, then each leaf's output) equals, at sampled leaves,
    the same network run row by row on cd_surrogate_features, plus the
    oracle's internal + local part and shells dl >= 4 (Sect. 3.2)."""
    s, w, nrm, _, _, _ = trained
    tin = _field(122)
    tree, leaf, N, chi = _plain(colden, tin, w)
    Ns = torch.empty_like(N)
    s.infer(tree, w, Ns)
    tg = np.random.default_rng(8).choice(tin.n_leaf, 3000, replace=False)
    cells = torch.from_numpy(tg).to(DEV)
    X = torch.empty((tg.size, 576), dtype=torch.float32, device=DEV)
    s.features(tree, cells, X)
    Y = torch.empty((tg.size, w.D), dtype=torch.float32, device=DEV)
    s.forward(X, Y)
    torch.cuda.synchronize()
    tr = oracle.Tree(tin)
    exact = tr.internal_local(oracle.dirs_healpix(1), tg) + tr.external(oracle.dirs_healpix(1), tg, 4)
    ref = S.columns_from_output(Y.cpu().numpy().astype(np.float64), exact, nrm[2], nrm[3])
    got = Ns.cpu().numpy().astype(np.float64)[tg]
    err = np.abs(np.log(got) - np.log(ref))
    print(f"infer vs features + forward: max |d ln N| {err.max():.3e} mean {err.mean():.3e}")
    assert err.max() <= 2e-3


def test_check_and_fallback_meet_the_chi_gate(colden, trained):
    s, w, nrm, _, _, _ = trained
    tin = _field(121)
    tree, leaf, N, chi = _plain(colden, tin, w)
    Ns = torch.empty_like(N)
    chis = torch.empty_like(chi)
    s.infer(tree, w, Ns, chis)
    nf, nt, emax = s.check_fallback(tree, w, Ns, chis, frac=0.01, tol_chi=0.03, seed=9)
    torch.cuda.synchronize()
    e = _chi_err(chis.cpu().numpy(), chi.cpu().numpy())
    print(f"fallback {nf}/{nt} tiles, max sampled err {emax:.3e}; chi error mean {e.mean():.3e} "
          f"p99 {np.percentile(e, 99):.3e} max {e.max():.3e}")
    assert np.percentile(e, 99) <= 0.03
    # against the oracle on a sample
    tg = np.random.default_rng(4).choice(tin.n_leaf, 2000, replace=False)
    ref = oracle.screening(oracle.Tree(tin).columns(oracle.dirs_healpix(1), tg))
    eo = _chi_err(chis.cpu().numpy()[tg], ref)
    print(f"vs oracle: p99 {np.percentile(eo, 99):.3e}")
    assert np.percentile(eo, 99) <= 0.03


def test_zero_tolerance_falls_back_everywhere(colden, trained):
    """tol = 0: every tile is recomputed by the method, so N equals the
    tiled sweep's to FP32 parity."""
    s, w, _, _, _, runs = trained
    tree, leaf, N, chi = runs[0]
    Ns = torch.empty_like(N)
    chis = torch.empty_like(chi)
    s.infer(tree, w, Ns, chis)
    nf, nt, _ = s.check_fallback(tree, w, Ns, chis, frac=0.01, tol_chi=0.0, seed=1)
    torch.cuda.synchronize()
    assert nf == nt
    rel = (torch.abs(Ns - N) / N).max().item()
    assert rel <= 1e-5


def test_many_failing_tiles_take_the_whole_grid_route(colden, trained):
    """An untrained network fails the check on most tiles: the method then
    sweeps the whole grid into N and chi, which equal the plain sweep's."""
    _, w, nrm, _, _, runs = trained
    tree, leaf, N, chi = runs[0]
    s = colden.Surrogate(w.D, 256, colden.CD_SURR_BF16, 5, norm=nrm)
    Ns = torch.empty_like(N)
    chis = torch.empty_like(chi)
    s.infer(tree, w, Ns, chis)
    nf, nt, _ = s.check_fallback(tree, w, Ns, chis, frac=0.01, tol_chi=0.03, seed=3)
    torch.cuda.synchronize()
    print(f"untrained: fallback {nf}/{nt} tiles")
    assert 4 * nf > nt
    assert (torch.abs(Ns - N) / N).max().item() <= 1e-5
    assert (torch.abs(chis - chi) / chi).max().item() <= 1e-5
    s.close()


def test_few_failing_tiles_take_the_per_tile_route(colden, trained):
    """A loose tolerance leaves at most a quarter of the tiles failing: each
    failing 8^3 tile is recomputed by the method (equal to the plain sweep),
    every other tile keeps the network's values, and the counts agree."""
    s, w, _, _, _, runs = trained
    tree, leaf, N, chi = runs[1]
    Ns0 = torch.empty_like(N)
    chis0 = torch.empty_like(chi)
    s.infer(tree, w, Ns0, chis0)
    for tol in (0.01, 0.02, 0.03, 0.05, 0.1, 0.3, 0.5, 1.0, 2.0, 5.0):
        Ns, chis = Ns0.clone(), chis0.clone()
        nf, nt, _ = s.check_fallback(tree, w, Ns, chis, frac=0.01, tol_chi=tol, seed=4)
        if 0 < 4 * nf <= nt:
            break
    torch.cuda.synchronize()
    print(f"tol {tol}: fallback {nf}/{nt} tiles")
    assert 0 < 4 * nf <= nt
    n = round(N.shape[0] ** (1 / 3))
    t = n // 8

    def tiles(a):  # [tiles][512 leaves][...]
        a = a.reshape(t, 8, t, 8, t, 8, -1).permute(0, 2, 4, 1, 3, 5, 6)
        return a.reshape(t ** 3, 512, -1)
    new, old, plain = tiles(Ns), tiles(Ns0), tiles(N)
    kept = (new == old).all(dim=2).all(dim=1)
    redone = (torch.abs(new - plain) <= 1e-5 * plain).all(dim=2).all(dim=1)
    assert bool((kept | redone).all())
    assert int((~kept).sum()) <= nf <= int(redone.sum())
    cn, cp = tiles(chis[:, None]), tiles(chi[:, None])
    assert bool((torch.abs(cn - cp)[~kept] <= 1e-5 * cp[~kept]).all())


def test_save_load_round_trip(colden, trained):
    s = trained[0]
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "net.bin")
        s.save(path)
        s2 = colden.Surrogate.load(path)
        assert np.array_equal(s2.get_params(), s.get_params())
        X = torch.randn((100, 576), device=DEV)
        Y1 = torch.empty((100, 12), device=DEV)
        Y2 = torch.empty((100, 12), device=DEV)
        s.forward(X, Y1)
        s2.forward(X, Y2)
        torch.cuda.synchronize()
        assert torch.equal(Y1, Y2)


def test_surrogate_errors(colden):
    with pytest.raises(colden.ColdenError):
        colden.Surrogate(12, 100)  # width not a multiple of 16
    with pytest.raises(colden.ColdenError):
        colden.Surrogate(12, 32, leaf_level=10)
    # a network for 512^3 grids on a 256^3 tree, and weights of another D
    tin8 = _field(100)
    leaf8 = torch.from_numpy(tin8.leaf_n).to(DEV)
    tree8 = colden.Tree(tin8, leaf8)
    N8 = torch.empty((tin8.n_leaf, 12), device=DEV)
    s9 = colden.Surrogate(12, 32, leaf_level=9)
    assert s9.Dout == 96
    with pytest.raises(colden.ColdenError) as e:
        s9.infer(tree8, colden.Weights(oracle.dirs_healpix(1)), N8)
    assert e.value.rc == colden.CD_EINVAL
    N6 = torch.empty((tin8.n_leaf, 6), device=DEV)
    with pytest.raises(colden.ColdenError):
        colden.Surrogate(12, 32).infer(tree8, colden.Weights(oracle.dirs_axes6()), N6)
    tin = synth.workload_uniform(5, seed=1)
    leaf = torch.from_numpy(tin.leaf_n).to(DEV)
    tree = colden.Tree(tin, leaf)
    s = colden.Surrogate(12, 32)
    w = colden.Weights(oracle.dirs_healpix(1))
    N = torch.empty((tin.n_leaf, 12), device=DEV)
    with pytest.raises(colden.ColdenError) as e:
        s.infer(tree, w, N)
    assert e.value.rc == colden.CD_EINVAL
