"""Seeded synthetic inputs: turbulent log-normal density fields and the AMR
tree structure built on them.

This module prepares inputs only. It holds none of the column-density
arithmetic (no pyramid, no shells, no chords, no screening): both the HIP path
and the CPU oracle receive the arrays it returns.

Fields follow the statistics of the paper's turbulent clouds (Sect. 4.2): a
Gaussian random field g with power spectrum P(k) ~ k^-11/3 (Kolmogorov), turned
into a log-normal density n = exp(sigma g) rescaled to a prescribed mean.

Conventions
-----------
* Leaf densities are in cm^-3, stored float32.
* Every 3D array is indexed [z, y, x] in C order, so x varies fastest.
* A tree is described by a base level B (a full 2^B grid), a maximum level
  Lmax and, for each level l in (B, Lmax], the list of refined parent cells at
  level l-1 (integer coordinates, one oct of 8 children each).
* Leaf order: base cells in row-major order (x fastest) skipping refined ones,
  then for l = B+1 .. Lmax every oct in list order, its children c = i + 2j + 4k
  (i, j, k the x, y, z child bits) skipping refined ones.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

PC_CM = 3.0857e18  # one parsec in cm


def gaussian_random_field(n: int, seed: int, slope: float = -11.0 / 3.0) -> np.ndarray:
    """Real white noise N(0,1) from PCG64(seed), coloured in Fourier space by
    |k|^(slope/2) (k = 0 removed), standardised to sample mean 0, variance 1.
    Returns float64 [n, n, n] indexed [z, y, x]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal((n, n, n))
    W = np.fft.rfftn(w)
    del w
    kz = np.fft.fftfreq(n)[:, None, None]
    ky = np.fft.fftfreq(n)[None, :, None]
    kx = np.fft.rfftfreq(n)[None, None, :]
    k2 = kz * kz + ky * ky + kx * kx
    k2[0, 0, 0] = 1.0
    amp = k2 ** (slope / 4.0)
    amp[0, 0, 0] = 0.0
    W *= amp
    del amp, k2
    g = np.fft.irfftn(W, s=(n, n, n), axes=(0, 1, 2))
    del W
    g -= g.mean()
    g /= g.std()
    return g


def lognormal_field(n: int, sigma: float, mean: float, seed: int) -> np.ndarray:
    """n = exp(sigma g), rescaled so that the sample mean equals `mean`.
    float64 [n, n, n], [z, y, x]."""
    g = gaussian_random_field(n, seed)
    g *= sigma
    np.exp(g, out=g)
    g *= mean / g.mean()
    return g


def block_mean(a: np.ndarray, f: int) -> np.ndarray:
    """Average a cubic [z, y, x] array over f^3 blocks (input preparation:
    the leaf density of a coarse leaf is the mass average of the fine field)."""
    n = a.shape[0] // f
    return a.reshape(n, f, n, f, n, f).mean(axis=(1, 3, 5))


@dataclass
class TreeInput:
    """Structure and leaf densities of a fully threaded octree."""
    box_cm: float
    base_level: int
    max_level: int
    # oct_parents[l - base_level - 1]: int32 [n_octs_l, 3] (x, y, z) of the
    # refined parent cells at level l - 1, for l in base_level+1 .. max_level.
    oct_parents: List[np.ndarray] = field(default_factory=list)
    leaf_n: np.ndarray = None          # float32 [n_leaf]
    leaf_level: np.ndarray = None      # int8 [n_leaf]
    leaf_ijk: np.ndarray = None        # int32 [n_leaf, 3] (x, y, z) at leaf level

    @property
    def n_leaf(self) -> int:
        return int(self.leaf_n.shape[0])

    @property
    def is_uniform(self) -> bool:
        return self.base_level == self.max_level

    def n_octs(self) -> List[int]:
        return [int(p.shape[0]) for p in self.oct_parents]


def uniform_tree(density_zyx: np.ndarray, box_cm: float) -> TreeInput:
    """Uniform grid of side 2^L: every cell is a leaf, row-major order."""
    n = density_zyx.shape[0]
    L = int(round(np.log2(n)))
    assert 1 << L == n and density_zyx.shape == (n, n, n)
    leaf_n = np.ascontiguousarray(density_zyx, dtype=np.float32).reshape(-1)
    t = TreeInput(box_cm=box_cm, base_level=L, max_level=L)
    t.leaf_n = leaf_n
    t.leaf_level = np.full(leaf_n.shape[0], L, dtype=np.int8)
    t.leaf_ijk = None  # implied by row-major order
    return t


def refine_uniform(tin: TreeInput) -> TreeInput:
    """The same uniform field one level finer: every leaf split into 8
    equal children (2^(L+1) per axis, same box).  Levels 0 .. L of its
    pyramid are the original field's."""
    assert tin.is_uniform
    n = 1 << tin.max_level
    a = tin.leaf_n.reshape(n, n, n)
    a = np.repeat(np.repeat(np.repeat(a, 2, axis=0), 2, axis=1), 2, axis=2)
    return uniform_tree(a, tin.box_cm)


def amr_tree(fine_zyx: np.ndarray, base_level: int, threshold: float,
             box_cm: float) -> TreeInput:
    """AMR tree on a field sampled at the finest level: a full 2^base grid,
    and every cell at level l < Lmax whose mass-averaged density exceeds
    `threshold` (and which exists) is split into an oct at level l + 1."""
    nf = fine_zyx.shape[0]
    Lmax = int(round(np.log2(nf)))
    assert 1 << Lmax == nf and base_level <= Lmax
    # mass averages at every level from base to Lmax
    avg = {Lmax: fine_zyx}
    for l in range(Lmax - 1, base_level - 1, -1):
        avg[l] = block_mean(avg[l + 1], 2)
    # existence / refinement flags
    exists = {base_level: np.ones((1 << base_level,) * 3, dtype=bool)}
    refined = {}
    for l in range(base_level, Lmax):
        refined[l] = exists[l] & (avg[l] > threshold)
        exists[l + 1] = np.repeat(np.repeat(np.repeat(refined[l], 2, 0), 2, 1), 2, 2)
    refined[Lmax] = np.zeros((1 << Lmax,) * 3, dtype=bool)

    oct_parents = []
    for l in range(base_level + 1, Lmax + 1):
        z, y, x = np.nonzero(refined[l - 1])  # C order: sorted by z, then y, then x
        oct_parents.append(np.stack([x, y, z], axis=1).astype(np.int32))

    leaves_n, leaves_lvl, leaves_ijk = [], [], []
    # base level, row-major
    z, y, x = np.nonzero(~refined[base_level])
    leaves_n.append(avg[base_level][z, y, x])
    leaves_lvl.append(np.full(z.shape[0], base_level, np.int8))
    leaves_ijk.append(np.stack([x, y, z], axis=1))
    for l in range(base_level + 1, Lmax + 1):
        par = oct_parents[l - base_level - 1]
        if par.shape[0] == 0:
            continue
        c = np.arange(8)
        ci, cj, ck = c & 1, (c >> 1) & 1, (c >> 2) & 1
        cx = (2 * par[:, 0:1] + ci[None, :]).reshape(-1)
        cy = (2 * par[:, 1:2] + cj[None, :]).reshape(-1)
        cz = (2 * par[:, 2:3] + ck[None, :]).reshape(-1)
        keep = ~refined[l][cz, cy, cx]
        cx, cy, cz = cx[keep], cy[keep], cz[keep]
        leaves_n.append(avg[l][cz, cy, cx])
        leaves_lvl.append(np.full(cx.shape[0], l, np.int8))
        leaves_ijk.append(np.stack([cx, cy, cz], axis=1))

    t = TreeInput(box_cm=box_cm, base_level=base_level, max_level=Lmax,
                  oct_parents=oct_parents)
    t.leaf_n = np.concatenate(leaves_n).astype(np.float32)
    t.leaf_level = np.concatenate(leaves_lvl)
    t.leaf_ijk = np.concatenate(leaves_ijk).astype(np.int32)
    return t


# ---------------------------------------------------------------------------
# The named workloads (sizes and statistics of the turbulent-cloud runs).
# ---------------------------------------------------------------------------

def workload_uniform(L: int, sigma: float = 1.5, mean: float = 10.0, seed: int = 1,
                     box_pc: float = 10.0) -> TreeInput:
    return uniform_tree(lognormal_field(1 << L, sigma, mean, seed), box_pc * PC_CM)


def workloads_uniform(L: int, seeds, sigma: float = 1.5, mean: float = 10.0, box_pc: float = 10.0,
                      threads: int = 8) -> List[TreeInput]:
    """workload_uniform for several seeds, generated side by side in threads
    (each field depends on its own seed only)."""
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(max(1, min(threads, len(seeds)))) as ex:
        return list(ex.map(lambda sd: workload_uniform(L, sigma, mean, sd, box_pc), seeds))


def workload_amr(base_level: int = 7, max_level: int = 9, sigma: float = 2.0,
                 mean: float = 10.0, seed: int = 3, threshold: float = 100.0,
                 box_pc: float = 20.0) -> TreeInput:
    fine = lognormal_field(1 << max_level, sigma, mean, seed)
    return amr_tree(fine, base_level, threshold, box_pc * PC_CM)


def point_mass_field(L: int, pos_xyz, value: float, background: float = 0.0) -> np.ndarray:
    n = 1 << L
    a = np.full((n, n, n), background, dtype=np.float64)
    x, y, z = pos_xyz
    a[z, y, x] = value
    return a


def sphere_field(L: int, radius_frac: float = 0.25, n_in: float = 1000.0,
                 n_out: float = 10.0) -> np.ndarray:
    """Uniform sphere at the box centre (the paper's first verification
    cloud: R = L/4, 1000 cm^-3 inside, 10 cm^-3 outside), cell-centre test."""
    n = 1 << L
    c = (np.arange(n) + 0.5) / n - 0.5
    r2 = c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2
    return np.where(r2 <= radius_frac ** 2, n_in, n_out).astype(np.float64)


def workload_sphere(base_level: int = 7, max_level: int = 9, box_pc: float = 50.0, radius_pc: float = 12.5,
                    n_in: float = 1000.0, n_out: float = 10.0) -> TreeInput:
    """The paper's sphere test cloud: a uniform sphere (n_in inside radius R,
    n_out outside) at the centre of the box, a full base grid and every cell
    that holds sphere matter refined down to max_level (the sphere resolved
    at 2^max_level effective)."""
    f = sphere_field(max_level, radius_pc / box_pc, n_in, n_out)
    # refine every cell whose mean density exceeds the ambient value
    return amr_tree(f, base_level, n_out * 1.0000001, box_pc * PC_CM)


def midplane_leaves(tin: TreeInput) -> np.ndarray:
    """Leaves whose cell lies just below the z = box / 2 plane (every level
    has a cell face there)."""
    lv = tin.leaf_level.astype(np.int64)
    kz = tin.leaf_ijk[:, 2].astype(np.int64)
    return np.nonzero(kz == (np.int64(1) << lv) // 2 - 1)[0]

