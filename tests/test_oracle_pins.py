"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix
(no GPU).  Each test names the passage it checks and is built so that a
plausible slip in the oracle (wrong origin, dropped shell, wrong sign, wrong
index, sum instead of mean, wrong reference point) fails at least one of them.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1410_0624_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    return np.array(rows)


# ---------------------------------------------------------------- helpers ---
def exit_distance(lo, hi, o, u):
    """Distance from a point o inside the box [lo, hi] to its boundary along
    unit u (closed form: the nearest face crossing)."""
    t = np.inf
    for k in range(3):
        if u[k] > 0:
            t = min(t, (hi[k] - o[k]) / u[k])
        elif u[k] < 0:
            t = min(t, (lo[k] - o[k]) / u[k])
    return t


def chord_by_sorting(lo, hi, o, u):
    """Length of {o + t u, t >= 0} inside the box, by sorting every plane
    crossing and testing the midpoint of each interval (independent of the
    oracle's slab clipping)."""
    ts = [0.0]
    for k in range(3):
        if u[k] != 0:
            for b in (lo[k], hi[k]):
                tb = (b - o[k]) / u[k]
                if tb > 0:
                    ts.append(tb)
    ts = sorted(ts)
    ts.append(ts[-1] + 1.0)
    tot = 0.0
    for a, b in zip(ts[:-1], ts[1:]):
        m = 0.5 * (a + b)
        p = o + m * u
        if np.all(p > lo) and np.all(p < hi):
            tot += b - a
    return tot


# ------------------------------------------------------------ directions ---
def test_theta_pin_from_precalc_caption():
    """Sect. 4.4 figure caption: theta = 0.841, 0.644, 0.541 rad at phi = 0 are
    theta_1 = arccos(1 - 1/M) of Eqs. 5-6 for M = 3, 5, 7, and phi_1 = 0."""
    g = _gold("theta_caption.txt")
    for M, theta in g:
        M = int(M)
        N = {3: 4, 5: 8, 7: 12}[M]
        u = oracle.dirs_mn(M, N)
        assert u.shape == (M * N, 3)
        th1 = np.arccos(u[0, 2])
        assert abs(th1 - theta) < 6e-4
        assert u[0, 1] == 0.0 and u[0, 0] > 0  # phi_1 = 0
    # equal solid angles: cos(theta_m) are the centres of M equal bins
    u = oracle.dirs_mn(5, 8)
    cz = np.unique(np.round(u[:, 2], 12))[::-1]
    assert np.allclose(cz, 1 - (2 * np.arange(1, 6) - 1) / 5.0)


def test_healpix_rings_match_gorski():
    g = _gold("healpix_rings.txt")
    for ns in (1, 2):
        u = oracle.dirs_healpix(ns)
        assert u.shape == (12 * ns * ns, 3)
        assert np.allclose(np.linalg.norm(u, axis=1), 1.0, atol=1e-14)
        rows = g[g[:, 0] == ns]
        start = 0
        for _, ring, zn, zd, npix, pn, pd in rows:
            npix = int(npix)
            blk = u[start:start + npix]
            start += npix
            assert np.allclose(blk[:, 2], zn / zd, atol=1e-14)
            phi = np.sort(np.mod(np.arctan2(blk[:, 1], blk[:, 0]), 2 * np.pi))
            phi = np.where(phi > 2 * np.pi - 1e-9, 0.0, phi)
            phi = np.sort(phi)
            want = np.pi * pn / pd + 2 * np.pi * np.arange(npix) / npix
            assert np.allclose(phi, np.sort(np.mod(want, 2 * np.pi)), atol=1e-12)
        assert start == 12 * ns * ns
        assert np.allclose(u.sum(axis=0), 0.0, atol=1e-12)


def test_healpix_nside1_shares_paper_3x4_rings():
    a = np.unique(np.round(oracle.dirs_healpix(1)[:, 2], 12))
    b = np.unique(np.round(oracle.dirs_mn(3, 4)[:, 2], 12))
    assert np.allclose(a, b)


def test_axes6():
    u = oracle.dirs_axes6()
    assert np.allclose(np.abs(u).sum(axis=1), 1.0)
    assert np.allclose(u.sum(axis=0), 0.0)


# ------------------------------------------------------------------ chord ---
def test_chord_against_plane_sorting():
    rng = np.random.default_rng(7)
    for _ in range(400):
        lo = rng.uniform(-2, 1, 3)
        hi = lo + rng.uniform(0.1, 2, 3)
        o = rng.uniform(-3, 3, 3)
        u = rng.normal(size=3)
        if rng.random() < 0.3:
            u[rng.integers(3)] = 0.0
        u /= np.linalg.norm(u)
        assert abs(oracle.chord(lo, hi, o, u) - chord_by_sorting(lo, hi, o, u)) < 1e-12


def test_chord_half_line_only():
    lo, hi = np.zeros(3), np.ones(3)
    assert oracle.chord(lo, hi, np.array([2.0, 0.5, 0.5]), np.array([1.0, 0, 0])) == 0.0
    assert abs(oracle.chord(lo, hi, np.array([2.0, 0.5, 0.5]), np.array([-1.0, 0, 0])) - 1.0) < 1e-15
    assert abs(oracle.chord(lo, hi, np.array([0.25, 0.5, 0.5]), np.array([1.0, 0, 0])) - 0.75) < 1e-15


# ------------------------------------------------------- uniform closed form ---
def _uniform_closed_form(L, T, u):
    """Uniform density, reference point fixed at the oct centre: the shells
    tile the box outside the oct, so their chords telescope to the exit
    distance of the box minus that of the oct (Eqs. 9-10 with every cell of
    density n0), plus the internal+local chord from the target centre."""
    dx = 0.5 ** L
    A = T // 2
    olo, ohi = A * 2 * dx, (A + 1) * 2 * dx
    ct = (T + 0.5) * dx
    co = (A + 0.5) * 2 * dx
    return (exit_distance(olo, ohi, ct, u) + exit_distance(np.zeros(3), np.ones(3), co, u)
            - exit_distance(olo, ohi, co, u))


@pytest.mark.parametrize("L,mode", [(2, 0), (3, 0), (4, 0), (5, 0), (6, 1), (7, 1)])
def test_uniform_density_closed_form(L, mode):
    """For L <= 5 the two-level approximation never moves the reference point
    (it only moves for dl >= 4, whose shells are empty on a 2^L <= 32 grid),
    so the precalculated mode must telescope exactly; the in-situ mode must
    telescope at any size."""
    n0 = 7.5
    n = 1 << L
    tin = synth.uniform_tree(np.full((n, n, n), n0), box_cm=1.0)
    tr = oracle.Tree(tin)
    U = np.concatenate([oracle.dirs_healpix(2), oracle.dirs_axes6(), oracle.dirs_mn(5, 8)])
    rng = np.random.default_rng(L)
    tg = np.unique(np.concatenate([[0, n - 1, tin.n_leaf - 1],
                                   rng.integers(0, tin.n_leaf, 64)]))
    N = tr.columns(U, tg, mode=mode)
    for r, t in enumerate(tg):
        T = np.array([t % n, (t // n) % n, t // (n * n)])
        want = np.array([_uniform_closed_form(L, T, u) for u in U]) * n0
        np.testing.assert_allclose(N[r], want, rtol=1e-12, atol=1e-12)


def test_precalc_moves_reference_only_beyond_three_levels():
    """L = 6 and 7: precalculated and in-situ agree on every direction where no
    shell of dl >= 4 is crossed, and differ only by a few per cent overall
    (the paper reports mean column differences of 6-7 %)."""
    L = 7
    n = 1 << L
    tin = synth.uniform_tree(np.full((n, n, n), 1.0), box_cm=1.0)
    tr = oracle.Tree(tin)
    U = oracle.dirs_healpix(1)
    tg = np.random.default_rng(1).integers(0, tin.n_leaf, 200)
    a = tr.columns(U, tg, mode=oracle.PRECALC73)
    b = tr.columns(U, tg, mode=oracle.INSITU)
    rel = np.abs(a - b) / b
    assert rel.max() > 1e-6          # the approximation does act
    assert rel.mean() < 0.05


# ------------------------------------------------------------ shell rules ---
def _shell_table(L, n_targets=400, seed=0):
    n = 1 << L
    tin = synth.uniform_tree(np.ones((n, n, n)), box_cm=1.0)
    tr = oracle.Tree(tin)
    rng = np.random.default_rng(seed)
    tg = rng.integers(0, tin.n_leaf, n_targets)
    return tr, tin, tg


def test_shell_construction_rules():
    """Sect. 3.2 shell rules: the inner limit is the previous outer limit; the
    outer limit adds two or three level-l cells per side so that it covers
    whole parent cells; Sect. 3.3: every shell lies within 5 cells of the
    level-l ancestor (the 11^3 standard cube), and 5 is reached."""
    L = 9
    tr, tin, tg = _shell_table(L, 300)
    n = 1 << L
    maxoff = 0
    for t in tg:
        T = np.array([t % n, (t // n) % n, t // (n * n)])
        sh, ref = tr.shells(int(t))
        assert sh.shape[0] == L
        prev = None
        for q, row in enumerate(sh):
            l = row[0]
            olo, ohi, ilo, ihi = row[1:4], row[4:7], row[7:10], row[10:13]
            assert l == L - 1 - q
            A = T >> (L - l)
            if q == 0:
                assert np.all(ilo == A) and np.all(ihi == A)
            else:
                # inner = previous outer, in this level's cells
                po, ph = prev
                assert np.all(2 * ilo == po) and np.all(2 * (ihi + 1) == ph + 1)
            ext_lo, ext_hi = ilo - olo, ohi - ihi
            assert np.all((ext_lo == 2) | (ext_lo == 3))
            assert np.all((ext_hi == 2) | (ext_hi == 3))
            assert np.all(olo % 2 == 0) and np.all((ohi + 1) % 2 == 0)
            maxoff = max(maxoff, np.abs(olo - A).max(), np.abs(ohi - A).max())
            prev = (olo, ohi)
    assert maxoff == 5


def test_reference_points_73_configurations():
    """Sect. 3.3: one configuration at dl = 1, eight at dl = 2 (octant of the
    level l+1 ancestor), 64 at dl >= 3 (octants at l+1 and l+2): 73 in all,
    seen as positions relative to the level-l ancestor in dx_l units."""
    L = 8
    n = 1 << L
    tr, tin, tg = _shell_table(L, 2000, seed=3)
    seen = {1: set(), 2: set(), 3: set()}
    for t in tg:
        T = np.array([t % n, (t // n) % n, t // (n * n)])
        sh, ref = tr.shells(int(t))
        for row, r in zip(sh, ref):
            l = row[0]
            dl = L - l
            A = T >> (L - l)
            rel = tuple(np.round(r * (1 << l) - (A + 0.5), 9))
            seen[min(dl, 3)].add(rel)
            allowed = {1: {0.0}, 2: {-0.25, 0.25}, 3: {-0.375, -0.125, 0.125, 0.375}}[min(dl, 3)]
            assert all(x in allowed for x in rel)
    assert (len(seen[1]), len(seen[2]), len(seen[3])) == (1, 8, 64)


def test_shells_tile_the_box_exactly_once():
    """Sect. 3.2: every cell of the box is counted at exactly one resolution
    (the target's oct at l0, else exactly one shell)."""
    L = 5
    n = 1 << L
    tin = synth.uniform_tree(np.ones((n, n, n)), box_cm=1.0)
    tr = oracle.Tree(tin)
    for t in np.random.default_rng(5).integers(0, tin.n_leaf, 60):
        T = np.array([t % n, (t // n) % n, t // (n * n)])
        cover = np.zeros((n, n, n), np.int32)  # [x, y, z]
        A = T >> 1
        cover[2 * A[0]:2 * A[0] + 2, 2 * A[1]:2 * A[1] + 2, 2 * A[2]:2 * A[2] + 2] += 1
        sh, _ = tr.shells(int(t))
        for row in sh:
            l = row[0]
            f = 1 << (L - l)
            olo, ohi, ilo, ihi = row[1:4], row[4:7], row[7:10], row[10:13]
            m = np.zeros((n, n, n), bool)
            lo = np.clip(olo * f, 0, n)
            hi = np.clip((ohi + 1) * f, 0, n)
            m[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = True
            lo = np.clip(ilo * f, 0, n)
            hi = np.clip((ihi + 1) * f, 0, n)
            m[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = False
            cover += m
        assert cover.min() == 1 and cover.max() == 1


# ------------------------------------------------------------- point mass ---
def test_point_mass_seen_once_with_pyramid_dilution():
    """A single dense leaf cell P: the tree method sees it exactly once, either
    at the target's resolution (its oct) or at the shell level l that holds
    the level-l cell containing P, where its density is diluted by 8^-(L-l)
    (coarse cell = mean of children, Sect. 3.2) and weighted by the chord
    from the shell's reference point."""
    L = 5
    n = 1 << L
    P = np.array([20, 9, 13])
    nd = 1000.0
    tin = synth.uniform_tree(synth.point_mass_field(L, P, nd), box_cm=1.0)
    tr = oracle.Tree(tin)
    U = np.concatenate([oracle.dirs_healpix(1), oracle.dirs_mn(5, 8)])
    rng = np.random.default_rng(11)
    tg = np.unique(np.concatenate([rng.integers(0, tin.n_leaf, 150),
                                   [P[0] + n * (P[1] + n * P[2]), P[0] + 1 + n * (P[1] + n * P[2])]]))
    N = tr.columns(U, tg)
    nonzero = 0
    for r, t in enumerate(tg):
        T = np.array([t % n, (t // n) % n, t // (n * n)])
        want = np.zeros(len(U))
        if np.all(T >> 1 == P >> 1):
            dx = 1.0 / n
            c = (T + 0.5) * dx
            for d, u in enumerate(U):
                want[d] = nd * chord_by_sorting(P * dx, (P + 1) * dx, c, u)
            hits = 1
        else:
            sh, ref = tr.shells(int(t))
            hits = 0
            for row, rp in zip(sh, ref):
                l = row[0]
                cP = P >> (L - l)
                olo, ohi, ilo, ihi = row[1:4], row[4:7], row[7:10], row[10:13]
                inside_outer = np.all(cP >= olo) and np.all(cP <= ohi)
                inside_inner = np.all(cP >= ilo) and np.all(cP <= ihi)
                if inside_outer and not inside_inner:
                    hits += 1
                    dx = 0.5 ** l
                    dens = nd * 8.0 ** (-(L - l))
                    for d, u in enumerate(U):
                        want[d] = dens * chord_by_sorting(cP * dx, (cP + 1) * dx, rp, u)
        assert hits == 1
        np.testing.assert_allclose(N[r], want, rtol=1e-11, atol=1e-14)
        nonzero += int(np.any(want > 0))
    assert nonzero > 20


def test_six_directions_need_no_geometric_factor():
    """Sect. 4.4: with the six axis directions every crossed cell is crossed
    over its full width, so every weight is 0 or 1 cell width: the column
    along +x is a sum of densities x dx along the target's row at each level
    (a prefix sum of the pyramid along index rows)."""
    L = 5
    n = 1 << L
    f = synth.lognormal_field(n, 1.5, 10.0, 21).astype(np.float32).astype(np.float64)
    tin = synth.uniform_tree(f, box_cm=1.0)
    tr = oracle.Tree(tin)
    U = oracle.dirs_axes6()
    pyr = {L: f}
    for l in range(L - 1, -1, -1):
        pyr[l] = synth.block_mean(pyr[l + 1], 2)
    for t in np.random.default_rng(2).integers(0, tin.n_leaf, 40):
        T = np.array([t % n, (t // n) % n, t // (n * n)])
        got = tr.columns(U, [t])[0]
        dx0 = 1.0 / n
        # +x: own half cell, then the sibling if the target is the low-x child
        want = f[T[2], T[1], T[0]] * 0.5 * dx0
        if T[0] % 2 == 0:
            want += f[T[2], T[1], T[0] + 1] * dx0
        sh, _ = tr.shells(int(t))
        for row in sh:
            l = row[0]
            A = T >> (L - l)
            ihi, ohi = row[10], row[4]
            for i in range(ihi + 1, min(ohi, (1 << l) - 1) + 1):
                want += pyr[l][A[2], A[1], i] * 0.5 ** l
        assert abs(got[0] - want) <= 1e-12 * want


# ---------------------------------------------------- pyramid and injection ---
def test_pyramid_and_injection_are_block_means():
    """Coarse cells hold the mean of their children (equal volumes, so the
    mass average), and a position with no cell at the requested level reads
    the coarser leaf that covers it: both equal block means of the fine field
    that generated the AMR leaves."""
    fine = synth.lognormal_field(32, 2.0, 10.0, 4)
    tin = synth.amr_tree(fine, base_level=3, threshold=14.0, box_cm=1.0)
    fine = fine.astype(np.float32).astype(np.float64)  # leaves are stored float32
    assert len(tin.oct_parents) == 2 and all(p.shape[0] > 0 for p in tin.oct_parents)
    tr = oracle.Tree(tin)
    assert tr.n_leaf == tin.n_leaf
    lv, ijk = tr.leaf_coords()
    assert np.array_equal(lv, tin.leaf_level) and np.array_equal(ijk, tin.leaf_ijk)
    means = {5: fine}
    for l in range(4, -1, -1):
        means[l] = synth.block_mean(means[l + 1], 2)
    # leaf level of every finest position
    leaf_at = np.full((32, 32, 32), -1)
    for q in range(tin.n_leaf):
        l = tin.leaf_level[q]
        f = 1 << (5 - l)
        x, y, z = tin.leaf_ijk[q] * f
        leaf_at[z:z + f, y:y + f, x:x + f] = l
    assert leaf_at.min() >= 3
    rng = np.random.default_rng(0)
    for _ in range(300):
        l = int(rng.integers(0, 6))
        i, j, k = rng.integers(0, 1 << l, 3)
        f = 1 << (5 - l)
        leaf_levels = leaf_at[k * f:(k + 1) * f, j * f:(j + 1) * f, i * f:(i + 1) * f]
        if leaf_levels.min() >= l:
            want = means[l][k, j, i]            # the cell exists: subtree mean
        else:
            ll = int(leaf_levels.max())         # inside one coarser leaf
            g = 1 << (l - ll)
            want = means[ll][k // g, j // g, i // g]
        # leaves are float32 roundings of block means: compare at that level
        assert abs(tr.density(l, int(i), int(j), int(k)) - want) <= 3e-7 * want
    assert tr.density(3, -1, 0, 0) == 0.0 and tr.density(3, 8, 0, 0) == 0.0


def test_amr_uniform_density_closed_form():
    """Uniform density on an AMR tree: every target, at any level, telescopes
    as on a uniform grid (in-situ reference point)."""
    fine = synth.lognormal_field(32, 2.0, 10.0, 4)
    tin = synth.amr_tree(fine, base_level=3, threshold=14.0, box_cm=1.0)
    tin.leaf_n = np.full(tin.n_leaf, 3.0, np.float32)
    tr = oracle.Tree(tin)
    U = oracle.dirs_healpix(1)
    tg = np.random.default_rng(8).integers(0, tin.n_leaf, 120)
    N = tr.columns(U, tg, mode=oracle.INSITU)
    for r, t in enumerate(tg):
        l = tin.leaf_level[t]
        T = tin.leaf_ijk[t].astype(np.int64)
        want = np.array([_uniform_closed_form(l, T, u) for u in U]) * 3.0
        np.testing.assert_allclose(N[r], want, rtol=1e-12)


def test_fully_refined_amr_equals_uniform_grid():
    f = synth.lognormal_field(16, 1.5, 10.0, 9)
    uni = synth.uniform_tree(f, box_cm=1.0)
    amr = synth.amr_tree(f, base_level=2, threshold=-1.0, box_cm=1.0)
    assert amr.n_leaf == uni.n_leaf
    U = oracle.dirs_healpix(1)
    a = oracle.Tree(amr).columns(U)
    b = oracle.Tree(uni).columns(U)
    # match leaves by coordinates
    idx = amr.leaf_ijk[:, 0] + 16 * (amr.leaf_ijk[:, 1] + 16 * amr.leaf_ijk[:, 2])
    np.testing.assert_allclose(a, b[idx], rtol=1e-13)


def test_linearity_in_density():
    L = 4
    n = 1 << L
    f1 = synth.lognormal_field(n, 1.5, 10.0, 1)
    f2 = synth.lognormal_field(n, 1.0, 3.0, 2)
    U = oracle.dirs_healpix(1)
    a = oracle.Tree(synth.uniform_tree(f1, 1.0)).columns(U)
    b = oracle.Tree(synth.uniform_tree(f2, 1.0)).columns(U)
    c = oracle.Tree(synth.uniform_tree(2 * f1 + 0.5 * f2, 1.0)).columns(U)
    # float32 leaf storage: compare at float32 input rounding
    np.testing.assert_allclose(c, 2 * a + 0.5 * b, rtol=2e-7)


# -------------------------------------------------------------- screening ---
def test_screening_factor_reading():
    """chi = (1/D) sum exp(-gamma A_V), A_V = N/1.87e21 with gamma = 3.74, is
    the paper's chi = (1/MN) sum exp(-sigma N) with sigma = 2e-21 cm^2 (Eq. 7)."""
    N = np.array([[0.0, 0.0, 0.0], [1e21, 1e21, 1e21], [0.0, 5e20, 3e21]])
    chi = oracle.screening(N)
    assert chi[0] == 1.0
    assert abs(chi[1] - np.exp(-2e-21 * 1e21)) < 1e-15
    assert abs(chi[2] - np.mean(np.exp(-2e-21 * N[2]))) < 1e-15


# ---------------------------------------------- accuracy vs brute force rays ---
@pytest.mark.parametrize("mean,D", [(10.0, 12), (100.0, 12), (100.0, 48)])
def test_extinction_accuracy_against_cone_raymarching(mean, D):
    """Abstract and Sect. 6: the extinction of the tree method is accurate to
    better than 10 %.  Reference: 768 exact rays per target (HEALPix Nside=8
    centres) through every finest cell, chi_ref = mean exp(-sigma N_ray);
    gate on the mean |chi_tree - chi_ref| (Eq. 13) over all targets of a 16^3
    turbulent log-normal cloud."""
    L = 4
    tin = synth.workload_uniform(L, sigma=1.5, mean=mean, seed=5)
    tr = oracle.Tree(tin)
    U = oracle.dirs_healpix(1 if D == 12 else 2)
    tg = np.arange(tin.n_leaf)
    chi_tree = oracle.screening(tr.columns(U, tg))
    rays = oracle.dirs_healpix(8)
    chi_ref = oracle.screening(tr.raymarch(rays, tg))
    dchi = np.abs(chi_tree - chi_ref)
    print(f"mean={mean} D={D}: mean dchi={dchi.mean():.4f} max={dchi.max():.4f} "
          f"chi_ref range=({chi_ref.min():.3f},{chi_ref.max():.3f})")
    assert dchi.mean() <= 0.10
    assert dchi.max() <= 0.35


def test_raymarch_uniform_is_distance_to_edge():
    """The brute-force reference itself: uniform density gives n x distance to
    the box edge along every ray."""
    L = 3
    n = 1 << L
    tin = synth.uniform_tree(np.full((n, n, n), 2.0), box_cm=1.0)
    tr = oracle.Tree(tin)
    rays = oracle.dirs_healpix(2)
    tg = np.arange(tin.n_leaf)
    R = tr.raymarch(rays, tg)
    for q in tg[::37]:
        T = np.array([q % n, (q // n) % n, q // (n * n)])
        c = (T + 0.5) / n
        for r, u in enumerate(rays):
            assert abs(R[q, r] - 2.0 * exit_distance(np.zeros(3), np.ones(3), c, u)) < 1e-12


def test_internal_local_of_uniform_density_is_the_exit_distance_from_the_oct():
    """Sect. 3.2: the internal + local part of a target is the sum over its
    oct's 8 cells of n x chord from the target centre; for uniform n0 that is
    n0 times the distance from the target centre to the oct's boundary along
    u (written out here per axis, no chord routine)."""
    L, n0, box = 4, 3.0, 2.0
    n = 1 << L
    tin = synth.uniform_tree(np.full((n, n, n), n0), box_cm=box)
    tr = oracle.Tree(tin)
    dirs = oracle.dirs_healpix(2)
    rng = np.random.default_rng(8)
    tg = rng.choice(tin.n_leaf, 50, replace=False)
    got = tr.internal_local(dirs, tg)
    dx = 1.0 / n
    for q, t in enumerate(tg):
        T = np.array([t % n, (t // n) % n, t // (n * n)])
        c = (T + 0.5) * dx
        lo, hi = (T // 2) * 2 * dx, (T // 2) * 2 * dx + 2 * dx
        for d, u in enumerate(dirs):
            dist = min(((hi[k] - c[k]) / u[k]) if u[k] > 0 else ((lo[k] - c[k]) / u[k])
                       for k in range(3) if u[k] != 0)
            assert abs(got[q, d] - n0 * box * dist) <= 1e-12 * n0 * box


def test_raymarch_axis_rays_sum_distinct_densities():
    """The brute-force reference along the six axes of a grid of distinct
    densities: from a cell centre a ray along +x crosses half of its own cell
    and then every later cell of its row, so the column is dx (n_own / 2 +
    sum of the densities beyond); the other five axes likewise.  A lookup of
    the wrong cell of a segment (its start instead of its middle) breaks the
    negative directions."""
    L = 3
    n = 1 << L
    rng = np.random.default_rng(21)
    f = rng.permutation(n ** 3).reshape(n, n, n).astype(np.float64) + 1.0  # f[z, y, x], all distinct
    box = 3.0
    tin = synth.uniform_tree(f, box_cm=box)
    tr = oracle.Tree(tin)
    rays = oracle.dirs_axes6()
    tg = np.arange(tin.n_leaf)
    R = tr.raymarch(rays, tg)
    dx = box / n
    for q in tg:
        i, j, k = q % n, (q // n) % n, q // (n * n)
        own = 0.5 * f[k, j, i]
        want = [own + f[k, j, i + 1:].sum(), own + f[k, j, :i].sum(),
                own + f[k, j + 1:, i].sum(), own + f[k, :j, i].sum(),
                own + f[k + 1:, j, i].sum(), own + f[:k, j, i].sum()]
        np.testing.assert_allclose(R[q], dx * np.array(want), rtol=1e-13)


def test_raymarch_single_dense_cell_gives_its_chord():
    """Only one finest cell holds matter: every ray's column is that density
    times the ray's chord through that one cell (the chord found by sorting
    plane crossings here), for oblique rays of every sign pattern."""
    L = 3
    n = 1 << L
    f = np.zeros((n, n, n))
    c = np.array([5, 2, 3])  # x, y, z of the dense cell
    f[c[2], c[1], c[0]] = 7.0
    tin = synth.uniform_tree(f, box_cm=1.0)
    tr = oracle.Tree(tin)
    rays = oracle.dirs_healpix(4)
    tg = np.arange(tin.n_leaf)
    R = tr.raymarch(rays, tg)
    lo, hi = c / n, (c + 1) / n
    hits = 0
    for q in tg:
        T = np.array([q % n, (q // n) % n, q // (n * n)])
        o = (T + 0.5) / n
        for r, u in enumerate(rays):
            want = 7.0 * chord_by_sorting(lo, hi, o, u)
            hits += want > 0
            assert abs(R[q, r] - want) <= 1e-13
    assert hits > 500


def test_mn_azimuths_step_two_pi_over_n():
    """Sect. 3.2: the azimuths of a ring are phi_n = 2 pi (n - 1) / N, N equal
    steps round the full circle starting at 0: each ring is closed under a
    rotation by 2 pi / N about z, its unit vectors sum to zero (N >= 2), and
    the first direction lies in the x-z half-plane x > 0."""
    for M, N in [(3, 4), (5, 8), (7, 12), (2, 5), (3, 7)]:
        u = oracle.dirs_mn(M, N)
        rot = np.array([[np.cos(2 * np.pi / N), -np.sin(2 * np.pi / N), 0],
                        [np.sin(2 * np.pi / N), np.cos(2 * np.pi / N), 0], [0, 0, 1]])
        for m in range(M):
            ring = u[m * N:(m + 1) * N]
            assert abs(ring[0, 1]) == 0.0 and ring[0, 0] > 0
            np.testing.assert_allclose(ring.sum(axis=0)[:2], 0.0, atol=1e-13)
            # the ring rotated by one step is the next direction of the ring
            np.testing.assert_allclose(ring @ rot.T, np.roll(ring, -1, axis=0), atol=1e-13)


def _slab_chords(lo, hi, o, u):
    """Length of the half-line o + t u (t >= 0) inside each box [lo, hi]
    (rows), by the slab method: a second chord routine, independent of the
    oracle's."""
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (lo - o) / u
        t2 = (hi - o) / u
    inside = (o >= lo) & (o <= hi)
    tmin = np.where(u == 0, np.where(inside, -np.inf, np.inf), np.minimum(t1, t2))
    tmax = np.where(u == 0, np.where(inside, np.inf, -np.inf), np.maximum(t1, t2))
    return np.maximum(tmax.min(-1) - np.maximum(tmin.max(-1), 0.0), 0.0)


@pytest.mark.parametrize("lo,hi", [(1, 1), (2, 3), (1, 3), (4, 6)])
def test_external_shell_ranges_against_a_direct_sum(lo, hi):
    """Eqs. 9-10 shell by shell: the oracle's external sum restricted to
    dl = lo..hi equals a direct numpy sum over the same shells (cells of the
    outer box minus the inner box, inside the grid, density from the
    pyramid, chord from the shell's reference point by a second chord
    routine)."""
    L = 6
    n = 1 << L
    tin = synth.workload_uniform(L, seed=11)
    tr = oracle.Tree(tin)
    dirs = oracle.dirs_healpix(1)
    f = tin.leaf_n.reshape(n, n, n).astype(np.float64)
    lv = [f]
    while lv[0].shape[0] > 1:
        a = lv[0]
        m = a.shape[0] // 2
        lv.insert(0, a.reshape(m, 2, m, 2, m, 2).mean(axis=(1, 3, 5)))
    tg = np.random.default_rng(5).choice(tin.n_leaf, 12, replace=False)
    got = tr.external(dirs, tg, lo, hi)
    for i, q in enumerate(tg):
        sh, ref = tr.shells(int(q))
        want = np.zeros(dirs.shape[0])
        for s, r in zip(sh, ref):
            l = int(s[0])
            if not lo <= L - l <= hi:
                continue
            olo, ohi, ilo, ihi = s[1:4], s[4:7], s[7:10], s[10:13]
            g = np.stack(np.meshgrid(*[np.arange(olo[a], ohi[a] + 1) for a in range(3)], indexing="ij"), -1)
            g = g.reshape(-1, 3)
            keep = ~np.all((g >= ilo) & (g <= ihi), 1) & np.all((g >= 0) & (g < (1 << l)), 1)
            g = g[keep]
            dn = lv[l][g[:, 2], g[:, 1], g[:, 0]]
            dx = 1.0 / (1 << l)
            for d in range(dirs.shape[0]):
                want[d] += (dn * _slab_chords(g * dx, (g + 1) * dx, r, dirs[d])).sum()
        want *= tin.box_cm
        assert np.allclose(got[i], want, rtol=1e-12, atol=1e-9 * want.max())


def test_external_shell_ranges_partition_the_column():
    """Internal + local plus the external sums over dl = 1, 2, 3 and >= 4
    give the method's column exactly, on a uniform grid and an AMR tree."""
    dirs = oracle.dirs_healpix(1)
    for tin in (synth.workload_uniform(6, seed=2), synth.workload_amr(4, 6, seed=3, threshold=30.0)):
        tr = oracle.Tree(tin)
        tg = np.random.default_rng(1).choice(tin.n_leaf, 200, replace=False)
        parts = tr.internal_local(dirs, tg) + sum(tr.external(dirs, tg, k, k) for k in (1, 2, 3)) + \
            tr.external(dirs, tg, 4)
        full = tr.columns(dirs, tg)
        assert np.allclose(parts, full, rtol=1e-13, atol=0)
        with pytest.raises(ValueError):
            tr.external(dirs, tg, 0, 3)
        with pytest.raises(ValueError):
            tr.external(dirs, tg, 3, 2)
