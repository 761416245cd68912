"""Host-side behaviour of the binding and of the C ABI's host-only queries
(no GPU): buffer checks raise ValueError before any pointer reaches the
library, and the workspace sizes follow the documented layout."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1410_0624_amd import colden, synth

pytestmark = pytest.mark.skipif(not os.path.exists(colden.LIB_PATH), reason="libcolden.so not built")


def test_buffer_checks_raise_before_the_call():
    f32 = torch.float32
    with pytest.raises(ValueError, match="torch tensor"):
        colden._dev_f32(np.zeros(4, np.float32), "N")
    with pytest.raises(ValueError, match="float32"):
        colden._dev_f32(torch.zeros(4, dtype=torch.float64), "N")
    with pytest.raises(ValueError, match="contiguous"):
        colden._dev_f32(torch.zeros(4, 4, dtype=f32).t(), "N")
    with pytest.raises(ValueError, match="shape"):
        colden._dev_f32(torch.zeros(8, 12, dtype=f32), "N", shape=(8, 48))
    with pytest.raises(ValueError, match="elements"):
        colden._dev_f32(torch.zeros(7, dtype=f32), "chi", numel=8)
    with pytest.raises(ValueError, match="CUDA"):
        colden._dev_f32(torch.zeros(8, dtype=f32), "chi", numel=8)
    with pytest.raises(ValueError, match="1-D"):
        colden._dev_i64(torch.zeros(2, 2, dtype=torch.int64))
    with pytest.raises(ValueError, match="int64"):
        colden._dev_i64(torch.zeros(2, dtype=torch.int32))


def test_tree_rejects_bad_leaf_arrays():
    tin = synth.workload_uniform(3, seed=1)
    with pytest.raises(ValueError, match="1-D"):
        colden.Tree(tin, torch.zeros((tin.n_leaf, 1), dtype=torch.float32))
    with pytest.raises(ValueError, match="float32"):
        colden.Tree(tin, torch.zeros(tin.n_leaf, dtype=torch.float64))


def _ws_tree(tin, max_dirs):
    par = [np.ascontiguousarray(p, dtype=np.int32) for p in tin.oct_parents]
    import ctypes as C
    n_octs = np.array([p.shape[0] for p in par] + [0], dtype=np.int64)
    ptrs = (C.c_void_p * (len(par) + 1))(*[p.ctypes.data for p in par], None)
    nb = C.c_size_t(0)
    rc = colden.lib().cd_tree_workspace_bytes(int(tin.base_level), int(tin.max_level),
                                              n_octs.ctypes.data_as(C.c_void_p) if par else None,
                                              C.cast(ptrs, C.c_void_p), int(tin.n_leaf), max_dirs, C.byref(nb))
    return rc, nb.value


def _al(b):
    return (b + 255) // 256 * 256


def test_uniform_tree_workspace_follows_the_layout():
    """A uniform 2^L grid: padded levels 0 .. L-1 (side 2^l + 10), coarse
    tables of levels 2 .. L-4 (216 codes, 64 at L-4) and one row per oct,
    for max_dirs directions, and an 8-byte counter; each piece 256-aligned."""
    for L, D in [(6, 12), (8, 48), (9, 48)]:
        n_leaf = 1 << (3 * L)

        class T:  # structure only: a uniform grid has no oct lists
            base_level = max_level = L
            oct_parents = []
        T.n_leaf = n_leaf
        rc, got = _ws_tree(T, D)
        assert rc == 0
        want = 0
        for l in range(L):
            want = _al(want) + ((1 << l) + 10) ** 3 * 4
        for l in range(2, L - 3):
            want = _al(want) + 8 ** l * (64 if l == L - 4 else 216) * D * 4
        want = _al(want) + 8 ** (L - 1) * D * 4
        want = _al(want) + 8
        assert got == want, (L, D, got, want)


def test_adaptive_tree_workspace_and_bad_structures():
    fine = synth.lognormal_field(32, 2.0, 10.0, 4)
    tin = synth.amr_tree(fine, base_level=3, threshold=14.0, box_cm=1.0)
    rc, b12 = _ws_tree(tin, 12)
    assert rc == 0 and b12 > 0
    rc, b48 = _ws_tree(tin, 48)
    assert rc == 0 and b48 > b12  # the sweep buffers grow with max_dirs
    # a wrong leaf count and max_dirs outside 1 .. 128 are rejected
    class Wrong:
        base_level, max_level, oct_parents = tin.base_level, tin.max_level, tin.oct_parents
        n_leaf = tin.n_leaf + 1
    assert _ws_tree(Wrong, 12)[0] == colden.CD_EINVAL
    assert _ws_tree(tin, 0)[0] == colden.CD_EINVAL
    assert _ws_tree(tin, colden.CD_MAX_DIRS + 1)[0] == colden.CD_EINVAL


def test_weights_workspace_query_is_host_only():
    import ctypes as C
    U = colden.directions(colden.CD_DIR_HEALPIX, 2)
    sizes = {}
    for prec in (colden.CD_FP32, colden.CD_BF16X2, colden.CD_FP16X2):
        nb = C.c_size_t(0)
        rc = colden.lib().cd_weights_workspace_bytes(U.ctypes.data_as(C.c_void_p), U.shape[0], colden.CD_PRECALC73,
                                                     prec, C.byref(nb))
        assert rc == 0
        sizes[prec] = nb.value
    assert sizes[colden.CD_BF16X2] > sizes[colden.CD_FP32] > 0  # split banks come on top
    nb = C.c_size_t(0)
    assert colden.lib().cd_weights_workspace_bytes(U.ctypes.data_as(C.c_void_p), 0, 0, 0, C.byref(nb)) == \
        colden.CD_EINVAL
