"""The learned surrogate on 512^3 grids (a network of leaf level 9): targets
and row tables against the oracle's near-shell sums, inference against the
network run row by row, and the end-to-end case: trained on 16 seeded 256^3
fields (seeds 100-115, each refined into 2^9 equal leaves for its labels),
run on the unseen 512^3 field of seed 999 (sigma_ln n = 1.5, mean 10 cm^-3)
with the 1 % sampled check and the method as fallback.

Gates: targets to 2e-5 (ln units); inference against features + forward to
2e-3 in ln N; after check + fallback, the 99th percentile of the relative
chi error <= 3 % against the plain FP32 sweep (every leaf) and against the
FP64 oracle (a sample); the network alone passes the check on at least
half of the 8^3 tiles.  Printed: the network-alone chi error distribution,
the fallback fraction and the time of inference + check + fallback against
the plain sweep of the same field."""
import numpy as np
import pytest

import oracle
from oracle import surrogate as S
from paper_1410_0624_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
L = 9
D = 12


@pytest.fixture(scope="module")
def colden():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1410_0624_amd import colden as c
    c.lib()
    return c


@pytest.fixture(scope="module")
def field(colden):
    """The unseen 512^3 field, its tree and the plain FP32 sweep."""
    tin = synth.workload_uniform(L, sigma=1.5, mean=10.0, seed=999)
    w = colden.Weights(oracle.dirs_healpix(1))
    leaf = torch.from_numpy(tin.leaf_n).to(DEV)
    tree = colden.Tree(tin, leaf, max_dirs=D)
    N = torch.empty((tin.n_leaf, D), dtype=torch.float32, device=DEV)
    chi = torch.empty(tin.n_leaf, dtype=torch.float32, device=DEV)
    colden.column_densities(tree, w, N, chi)
    torch.cuda.synchronize()
    return tin, w, tree, leaf, N, chi


@pytest.fixture(scope="module")
def orc(field):
    return oracle.Tree(field[0])


@pytest.fixture(scope="module")
def trained(colden):
    from paper_1410_0624_amd import surrogate_train
    w = colden.Weights(oracle.dirs_healpix(1))
    tins = synth.workloads_uniform(8, list(range(100, 116)), sigma=1.5, mean=10.0)
    fields = [surrogate_train.label_field(t, w, L, DEV) for t in tins]
    del tins
    nrm = surrogate_train.norms(fields)
    s = colden.Surrogate(D, 256, colden.CD_SURR_BF16, 1, norm=nrm, leaf_level=L)
    log = surrogate_train.fit(s, fields, steps=6000, batch=8192, lr=2e-3, lr_final=5e-5, seed=2, log_every=1000)
    print("training log:", [(k, round(l, 4)) for k, l in log])
    del fields
    torch.cuda.empty_cache()
    return s, nrm, log


def _first_leaf_of_blocks(cells, n):
    """[len(cells), 8]: the first leaf of each of the 8 octs (blocks j) of
    every listed leaf's level-7 cell."""
    x, y, z = cells % n, (cells // n) % n, cells // (n * n)
    out = np.empty((cells.size, 8), np.int64)
    for j in range(8):
        xj = (x >> 2 << 2) + 2 * (j & 1)
        yj = (y >> 2 << 2) + 2 * ((j >> 1) & 1)
        zj = (z >> 2 << 2) + 2 * (j >> 2)
        out[:, j] = (zj * n + yj) * n + xj
    return out


def test_targets_and_row_table_against_the_oracle(colden, field, orc):
    tin, w, tree, _, _, _ = field
    n = 1 << L
    probe = colden.Surrogate(D, 16, colden.CD_SURR_FP32, 0, norm=(0.0, 1.0, 0.0, 1.0), leaf_level=L)
    rng = np.random.default_rng(3)
    cells = np.concatenate([[0, n ** 3 - 1, n - 1, n * n * (n - 1)], rng.choice(n ** 3, 250, replace=False)])
    T = torch.empty((cells.size, 8 * D), dtype=torch.float32, device=DEV)
    probe.targets(tree, w, torch.from_numpy(cells).to(DEV), T)
    rows = torch.empty((colden.Surrogate.ROWS, 8 * D), dtype=torch.float32, device=DEV)
    probe.row_targets(tree, w, rows)
    torch.cuda.synchronize()
    got = T.cpu().numpy().reshape(cells.size, 8, D).astype(np.float64)
    leaves = _first_leaf_of_blocks(cells, n)
    E = orc.external(oracle.dirs_healpix(1), leaves.ravel(), 1, 3, nthreads=8).reshape(cells.size, 8, D)
    want = S.targets(E, 0.0, 1.0)
    err = np.abs(got - want).max()
    print(f"targets at 512^3 vs oracle near shells: max |d ln| {err:.2e}")
    assert err <= 2e-5
    # the row table holds the same values at each cell's level-7 row
    x, y, z = cells % n, (cells // n) % n, cells // (n * n)
    r7 = ((z >> 2) * 128 + (y >> 2)) * 128 + (x >> 2)
    assert torch.equal(rows[torch.from_numpy(r7).to(DEV)], T)
    probe.close()


def test_infer_matches_features_and_forward(colden, field, orc, trained):
    """Each leaf's N is its oct's block of the network row of its level-7
    cell plus the oracle's internal + local part and shells dl >= 4."""
    tin, w, tree, _, N, _ = field
    s, nrm, _ = trained
    Ns = torch.empty_like(N)
    s.infer(tree, w, Ns)
    tg = np.random.default_rng(8).choice(tin.n_leaf, 2000, replace=False)
    cells = torch.from_numpy(tg).to(DEV)
    X = torch.empty((tg.size, 576), dtype=torch.float32, device=DEV)
    s.features(tree, cells, X)
    Y = torch.empty((tg.size, 8 * D), dtype=torch.float32, device=DEV)
    s.forward(X, Y)
    torch.cuda.synchronize()
    j = S.block_of(tg, L)
    Yb = Y.cpu().numpy().reshape(tg.size, 8, D)[np.arange(tg.size), j].astype(np.float64)
    dirs = oracle.dirs_healpix(1)
    exact = orc.internal_local(dirs, tg) + orc.external(dirs, tg, 4, nthreads=8)
    ref = S.columns_from_output(Yb, exact, nrm[2], nrm[3])
    got = Ns.cpu().numpy().astype(np.float64)[tg]
    err = np.abs(np.log(got) - np.log(ref))
    print(f"infer vs features + forward at 512^3: max |d ln N| {err.max():.3e} mean {err.mean():.3e}")
    assert err.max() <= 2e-3


def test_unseen_512_field_end_to_end(colden, field, orc, trained):
    tin, w, tree, leaf, N, chi = field
    s, _, log = trained
    assert log[-1][1] < 0.05 * log[0][1]
    Ns = torch.empty_like(N)
    chis = torch.empty_like(chi)
    stream = torch.cuda.current_stream()

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    Np, chip = torch.empty_like(N), torch.empty_like(chi)
    ms_plain = timed(lambda: colden.column_densities(tree, w, Np, chip))
    ms_net = timed(lambda: s.infer(tree, w, Ns, chis))
    ref = chi.cpu().numpy().astype(np.float64)
    e_net = np.abs(chis.cpu().numpy() - ref) / ref
    n, t = 1 << L, (1 << L) // 8
    tile_max = e_net.reshape(t, 8, t, 8, t, 8).max(axis=(1, 3, 5))
    fb = {}

    def surrogate():
        s.infer(tree, w, Ns, chis)
        fb["r"] = s.check_fallback(tree, w, Ns, chis, frac=0.01, tol_chi=0.03, seed=7)

    ms_surr = timed(surrogate)
    nf, nt, emax = fb["r"]
    e = np.abs(chis.cpu().numpy().astype(np.float64) - ref) / ref
    tg = np.random.default_rng(4).choice(tin.n_leaf, 2000, replace=False)
    chi_o = oracle.screening(orc.columns(oracle.dirs_healpix(1), tg, nthreads=8))
    eo = np.abs(chis.cpu().numpy().astype(np.float64)[tg] - chi_o) / chi_o
    q = lambda a: f"mean {a.mean():.4f} p50 {np.median(a):.4f} p99 {np.percentile(a, 99):.4f} max {a.max():.3f}"
    print(f"network alone: chi error {q(e_net)}; tiles with every leaf within 3 %: {np.mean(tile_max <= 0.03):.3f}")
    print(f"check + fallback: {nf}/{nt} tiles recomputed ({nf / nt:.3f}), largest sampled error {emax:.3f}; "
          f"chi error after: {q(e)}; vs oracle sample: {q(eo)}")
    print(f"time: plain FP32 sweep {ms_plain:.3f} ms, network inference {ms_net:.3f} ms, inference + check + "
          f"fallback {ms_surr:.3f} ms (surrogate / plain = {ms_surr / ms_plain:.2f})")
    assert np.percentile(e, 99) <= 0.03
    assert np.percentile(eo, 99) <= 0.03
    assert 2 * nf <= nt
