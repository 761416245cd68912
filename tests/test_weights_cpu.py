"""Pins of the library's precalculated geometric factors K (Sect. 3.3,
Eqs. 10-11) through the host-only query cd_weight_lists (no GPU): the FP64
lists that cd_precompute_weights rounds and uploads.  None of these checks
uses the oracle; each is a fact of the geometry:

* every listed cell lies in its shell (the outer box minus the inner box) and
  inside the 11^3 standard cube, and every weight is a chord of a unit cell
  (0 < K <= sqrt 3);
* the weights of one (configuration, direction) add up to the ray's length
  between leaving the inner box and leaving the outer box, both exit
  distances written out here per axis (the shell telescopes);
* the lists are mirror symmetric: the x-mirror of a configuration with the
  x-mirrored direction has the x-mirrored cells with the same weights
  (HEALPix sets are closed under x -> -x);
* along the six axes (Sect. 4.4) every weight is exactly 1 (whole cells);
* internal + local (Sect. 3.2): the 8 chords from a target centre through
  its oct's cells add up to the distance to the oct's boundary.
"""
import os

import numpy as np
import pytest

from paper_1410_0624_amd import colden

pytestmark = pytest.mark.skipif(not os.path.exists(colden.LIB_PATH), reason="libcolden.so not built")


def exit_distance(lo, hi, o, u):
    """Distance from o (inside [lo, hi]) to the box boundary along unit u."""
    t = np.inf
    for k in range(3):
        if u[k] > 0:
            t = min(t, (hi[k] - o[k]) / u[k])
        elif u[k] < 0:
            t = min(t, (lo[k] - o[k]) / u[k])
    return t


def _dirs(scheme, p1, p2=0):
    return colden.directions(scheme, p1, p2)


DIR_SETS = {
    "healpix1": (colden.CD_DIR_HEALPIX, 1, 0),
    "healpix2": (colden.CD_DIR_HEALPIX, 2, 0),
    "mn5x8": (colden.CD_DIR_PAPER_MN, 5, 8),
}


@pytest.mark.parametrize("kind", [1, 2, 3, 4])
@pytest.mark.parametrize("dset", ["healpix1", "healpix2", "mn5x8"])
def test_shell_weights_telescope_to_the_exit_distances(kind, dset):
    U = _dirs(*DIR_SETS[dset])
    t = colden.weight_lists(U, kind)
    off, w, cnt, ref, box = t["off"], t["w"], t["cnt"], t["ref"], t["box"]
    nc, D, ln = w.shape
    assert nc == {1: 8, 2: 64, 3: 512, 4: 1728}[kind]
    assert D == U.shape[0]
    worst = 0.0
    for c in range(nc):
        ilo, ihi, olo, ohi = (box[c, :, k].astype(float) for k in range(4))
        assert np.all(olo >= -5) and np.all(ohi <= 5)  # the 11^3 standard cube
        for d in range(D):
            k = cnt[c, d]
            assert np.all(w[c, d, k:] == 0)
            e = off[c, d, :k]
            inner = np.all((e >= ilo) & (e <= ihi), axis=1)
            outer = np.all((e >= olo) & (e <= ohi), axis=1)
            assert not inner.any() and outer.all()
            assert len({tuple(x) for x in e}) == k  # no cell twice
            assert np.all(w[c, d, :k] > 0) and np.all(w[c, d, :k] <= np.sqrt(3) + 1e-12)
            want = exit_distance(olo - 0.5, ohi + 0.5, ref[c], U[d]) - exit_distance(ilo - 0.5, ihi + 0.5, ref[c], U[d])
            worst = max(worst, abs(w[c, d, :k].sum() - want))
    assert worst <= 1e-12, worst


def _mirror_x(t, U):
    """Index maps of the x-mirror: configuration c -> c', direction d -> d'."""
    ref, box = t["ref"], t["box"]
    key = {}
    for c in range(ref.shape[0]):
        key[(tuple(np.round(ref[c], 12)), tuple(box[c].ravel()))] = c
    cmap = []
    for c in range(ref.shape[0]):
        r = ref[c].copy()
        r[0] = -r[0]
        b = box[c].copy()
        b[0] = [-box[c, 0, 1], -box[c, 0, 0], -box[c, 0, 3], -box[c, 0, 2]]
        cmap.append(key[(tuple(np.round(r, 12)), tuple(b.ravel()))])
    Um = U.copy()
    Um[:, 0] = -Um[:, 0]
    dmap = [int(np.argmin(np.linalg.norm(U - um, axis=1))) for um in Um]
    assert np.allclose(U[dmap], Um, atol=1e-14)
    return cmap, dmap


@pytest.mark.parametrize("kind", [1, 2, 3, 4])
def test_shell_weights_are_mirror_symmetric(kind):
    U = _dirs(colden.CD_DIR_HEALPIX, 2)
    t = colden.weight_lists(U, kind)
    off, w, cnt = t["off"], t["w"], t["cnt"]
    cmap, dmap = _mirror_x(t, U)
    for c in range(w.shape[0]):
        for d in range(w.shape[1]):
            cm, dm = cmap[c], dmap[d]
            assert cnt[c, d] == cnt[cm, dm]
            a = {(x, y, z): v for (x, y, z), v in zip(off[c, d, :cnt[c, d]], w[c, d, :cnt[c, d]])}
            b = {(-x, y, z): v for (x, y, z), v in zip(off[cm, dm, :cnt[cm, dm]], w[cm, dm, :cnt[cm, dm]])}
            assert a.keys() == b.keys()
            for k in a:
                assert abs(a[k] - b[k]) <= 1e-13


@pytest.mark.parametrize("kind", [1, 2, 3, 4])
def test_axis_directions_cross_whole_cells(kind):
    U = _dirs(colden.CD_DIR_AXES6, 0)
    t = colden.weight_lists(U, kind)
    w, cnt, box = t["w"], t["cnt"], t["box"]
    for c in range(w.shape[0]):
        for d in range(6):
            k = cnt[c, d]
            assert np.all(w[c, d, :k] == 1.0)
            # the number of cells crossed is the shell's thickness on that side
            a, s = d // 2, d % 2
            want = box[c, a, 3] - box[c, a, 1] if s == 0 else box[c, a, 0] - box[c, a, 2]
            assert k == want


@pytest.mark.parametrize("dset", ["healpix1", "healpix2", "mn5x8"])
def test_internal_local_chords_reach_the_oct_boundary(dset):
    U = _dirs(*DIR_SETS[dset])
    t = colden.weight_lists(U, 0)
    w, ref = t["w"], t["ref"]
    assert w.shape == (8, U.shape[0], 8)
    for a in range(8):
        # the target's own cell is crossed for half a cell width at most
        own = a
        assert np.all(w[a, :, own] > 0) and np.all(w[a, :, own] <= np.sqrt(3) / 2 + 1e-12)
        for d, u in enumerate(U):
            want = exit_distance(np.zeros(3), np.full(3, 2.0), ref[a], u)
            assert abs(w[a, d].sum() - want) <= 1e-13


def test_weight_lists_reject_bad_arguments():
    U = _dirs(colden.CD_DIR_HEALPIX, 1)
    with pytest.raises(colden.ColdenError):
        colden.weight_lists(U, 5)
    with pytest.raises(colden.ColdenError):
        colden.weight_lists(2 * U, 1)  # not unit vectors
