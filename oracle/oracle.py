"""ctypes front end of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  Every
function cites the part of the paper it follows in oracle.c.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PRECALC73 = 0
INSITU = 1
AV_PER_NH = 1.0 / 1.87e21
GAMMA = 3.74


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_DEFAULT_SOURCE", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.orc_dirs_mn.argtypes = [C.c_int, C.c_int, P]
        L.orc_dirs_healpix.argtypes = [C.c_int, P]
        L.orc_dirs_axes6.argtypes = [P]
        L.orc_chord.argtypes = [P, P, P, P]
        L.orc_chord.restype = C.c_double
        L.orc_tree_new.argtypes = [C.c_double, C.c_int, C.c_int, P, P, P, C.c_int64]
        L.orc_tree_new.restype = P
        L.orc_tree_free.argtypes = [P]
        L.orc_tree_n_leaf.argtypes = [P]
        L.orc_tree_n_leaf.restype = C.c_int64
        L.orc_leaf_coords.argtypes = [P, P, P]
        L.orc_density.argtypes = [P, C.c_int, C.c_int64, C.c_int64, C.c_int64]
        L.orc_density.restype = C.c_double
        L.orc_columns.argtypes = [P, P, C.c_int, C.c_int, P, C.c_int64, P, C.c_int]
        L.orc_shells.argtypes = [P, C.c_int64, C.c_int, P, P]
        L.orc_internal_local.argtypes = [P, P, C.c_int, P, C.c_int64, P]
        L.orc_external_shells.argtypes = [P, P, C.c_int, C.c_int, P, C.c_int64, C.c_int, C.c_int, P, C.c_int]
        L.orc_screening.argtypes = [P, C.c_int64, C.c_int, C.c_double, C.c_double, P]
        L.orc_raymarch.argtypes = [P, P, C.c_int, P, C.c_int64, P, C.c_int]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# --------------------------------------------------------------------------
# directions (Sect. 3.2 Eqs. 5-6; HEALPix centres; six axes)
# --------------------------------------------------------------------------

def dirs_mn(M: int, N: int) -> np.ndarray:
    out = np.zeros((M * N, 3))
    d = lib().orc_dirs_mn(M, N, _p(out))
    assert d == M * N
    return out


def dirs_healpix(nside: int) -> np.ndarray:
    out = np.zeros((12 * nside * nside, 3))
    d = lib().orc_dirs_healpix(nside, _p(out))
    assert d == 12 * nside * nside
    return out


def dirs_axes6() -> np.ndarray:
    out = np.zeros((6, 3))
    lib().orc_dirs_axes6(_p(out))
    return out


def chord(lo, hi, o, u) -> float:
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (lo, hi, o, u)]
    return float(lib().orc_chord(*[_p(x) for x in a]))


# --------------------------------------------------------------------------
# tree
# --------------------------------------------------------------------------

class Tree:
    """Oracle-side tree (pyramid of means, injection of coarser leaves)."""

    def __init__(self, tin):
        self.tin = tin
        self._keep = [np.ascontiguousarray(p, dtype=np.int32) for p in tin.oct_parents]
        n_octs = np.array([p.shape[0] for p in self._keep] + [0], dtype=np.int64)
        ptrs = (C.c_void_p * (len(self._keep) + 1))(*[p.ctypes.data for p in self._keep], None)
        self._leaf = np.ascontiguousarray(tin.leaf_n, dtype=np.float32)
        h = lib().orc_tree_new(float(tin.box_cm), int(tin.base_level), int(tin.max_level),
                               _p(n_octs), C.cast(ptrs, C.c_void_p), _p(self._leaf),
                               int(self._leaf.shape[0]))
        if not h:
            raise ValueError("oracle: malformed tree description")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_tree_free(self.h)
            self.h = None

    @property
    def n_leaf(self) -> int:
        return int(lib().orc_tree_n_leaf(self.h))

    def leaf_coords(self):
        n = self.n_leaf
        lv = np.zeros(n, np.int8)
        ijk = np.zeros((n, 3), np.int32)
        lib().orc_leaf_coords(self.h, _p(lv), _p(ijk))
        return lv, ijk

    def density(self, level: int, i: int, j: int, k: int) -> float:
        return float(lib().orc_density(self.h, level, i, j, k))

    def columns(self, dirs: np.ndarray, targets=None, mode: int = PRECALC73,
                nthreads: int = 0) -> np.ndarray:
        """N[n_targets, D] in cm^-2 (FP64)."""
        dirs = np.ascontiguousarray(dirs, dtype=np.float64)
        D = dirs.shape[0]
        if targets is None:
            targets = np.arange(self.n_leaf, dtype=np.int64)
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        out = np.zeros((targets.shape[0], D))
        rc = lib().orc_columns(self.h, _p(dirs), D, mode, _p(targets), targets.shape[0],
                               _p(out), nthreads)
        if rc != 0:
            raise ValueError("oracle: bad arguments")
        return out

    def internal_local(self, dirs: np.ndarray, targets) -> np.ndarray:
        """Internal + local part alone (Sect. 3.2), [n_targets, D] cm^-2."""
        dirs = np.ascontiguousarray(dirs, dtype=np.float64)
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        out = np.zeros((targets.shape[0], dirs.shape[0]))
        if lib().orc_internal_local(self.h, _p(dirs), dirs.shape[0], _p(targets), targets.shape[0], _p(out)) != 0:
            raise ValueError("oracle: bad arguments")
        return out

    def external(self, dirs: np.ndarray, targets, dl_lo: int = 1, dl_hi: int = 1 << 20, mode: int = PRECALC73,
                 nthreads: int = 0) -> np.ndarray:
        """External sum of the targets' octs over the shells dl_lo <= dl <=
        dl_hi only (Sect. 3.2, Eqs. 9-10), [n_targets, D] cm^-2."""
        dirs = np.ascontiguousarray(dirs, dtype=np.float64)
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        out = np.zeros((targets.shape[0], dirs.shape[0]))
        if lib().orc_external_shells(self.h, _p(dirs), dirs.shape[0], mode, _p(targets), targets.shape[0],
                                     int(dl_lo), int(min(dl_hi, 1 << 30)), _p(out), nthreads) != 0:
            raise ValueError("oracle: bad arguments")
        return out

    def shells(self, target: int, mode: int = PRECALC73):
        out = np.zeros((32, 16), np.int64)
        ref = np.zeros((32, 3))
        ns = lib().orc_shells(self.h, int(target), mode, _p(out), _p(ref))
        return out[:ns], ref[:ns]

    def raymarch(self, rays: np.ndarray, targets, nthreads: int = 0) -> np.ndarray:
        rays = np.ascontiguousarray(rays, dtype=np.float64)
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        out = np.zeros((targets.shape[0], rays.shape[0]))
        rc = lib().orc_raymarch(self.h, _p(rays), rays.shape[0], _p(targets),
                                targets.shape[0], _p(out), nthreads)
        assert rc == 0
        return out


def screening(N: np.ndarray, av_per_nh: float = AV_PER_NH, gamma: float = GAMMA) -> np.ndarray:
    """chi = (1/D) sum_d exp(-gamma A_V,d), A_V = N av_per_nh (Eq. 7)."""
    N = np.ascontiguousarray(N, dtype=np.float64)
    n, D = N.shape
    chi = np.zeros(n)
    lib().orc_screening(_p(N), n, D, av_per_nh, gamma, _p(chi))
    return chi
