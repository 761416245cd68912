"""Python binding of the colden C ABI (include/colden.h): argument marshalling
only.  Every step of the column-density path runs in the HIP library; torch
tensors provide device memory (the handles' workspaces, inputs and outputs)
and streams.  Missing library = hard error.  Buffer shapes, dtypes and
devices are checked here (ValueError) before any pointer crosses the ABI."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcolden.so")

CD_OK, CD_EINVAL, CD_ENOMEM, CD_EDEVICE, CD_EUNSUPPORTED = 0, -1, -2, -3, -4
CD_DIR_HEALPIX, CD_DIR_PAPER_MN, CD_DIR_AXES6 = 0, 1, 2
CD_PRECALC73, CD_INSITU = 0, 1
CD_FP32, CD_BF16X2, CD_FP16X2 = 0, 1, 2
CD_MAX_DIRS = 128
AV_PER_NH = 1.0 / 1.87e21
GAMMA = 3.74

EXPORTS = [
    "cd_last_error", "cd_version", "cd_directions", "cd_build_tree", "cd_tree_update",
    "cd_tree_n_leaf", "cd_tree_leaf_coords", "cd_tree_destroy", "cd_precompute_weights",
    "cd_weights_n_dirs", "cd_weights_split_steps", "cd_weights_destroy", "cd_column_densities", "cd_column_densities_log16",
    "cd_screening_factor",
    "cd_profile_enable", "cd_profile_read", "cd_check_densities", "cd_heating_rates", "cd_screening_heating",
    "cd_weight_lists", "cd_tree_workspace_bytes", "cd_weights_workspace_bytes", "cd_tree_set_aux_stream",
]
G0_DRAINE = 1.7
STAGES = ["pyramid", "coarse", "external", "rows", "sweep"]


class ColdenError(RuntimeError):
    def __init__(self, rc: int, msg: str):
        super().__init__(f"colden error {rc}: {msg}")
        self.rc = rc


_lib = None


def lib():
    """Load libcolden.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        P, I, I64, D = C.c_void_p, C.c_int, C.c_int64, C.c_double
        L.cd_last_error.restype = C.c_char_p
        L.cd_version.restype = I
        L.cd_directions.argtypes = [I, I, I, P, I, P]
        L.cd_build_tree.argtypes = [D, I, I, P, P, P, I64, I, P, C.c_size_t, P, P]
        L.cd_tree_workspace_bytes.argtypes = [I, I, P, P, I64, I, P]
        L.cd_tree_set_aux_stream.argtypes = [P, P]
        L.cd_tree_update.argtypes = [P, P, I64, P]
        L.cd_tree_n_leaf.argtypes = [P, P]
        L.cd_tree_leaf_coords.argtypes = [P, P, P]
        L.cd_tree_destroy.argtypes = [P]
        L.cd_tree_destroy.restype = None
        L.cd_precompute_weights.argtypes = [P, I, I, I, P, C.c_size_t, P, P]
        L.cd_weights_workspace_bytes.argtypes = [P, I, I, I, P]
        L.cd_weights_n_dirs.argtypes = [P, P]
        L.cd_weights_split_steps.argtypes = [P, P]
        L.cd_weights_destroy.argtypes = [P]
        L.cd_weights_destroy.restype = None
        L.cd_column_densities.argtypes = [P, P, P, P, D, D, P]
        L.cd_column_densities_log16.argtypes = [P, P, P, P, D, D, P]
        L.cd_screening_factor.argtypes = [P, I64, I, D, D, P, P, P]
        L.cd_profile_enable.argtypes = [P, I]
        L.cd_profile_read.argtypes = [P, P]
        L.cd_check_densities.argtypes = [P, I64, P, P, P]
        L.cd_heating_rates.argtypes = [P, P, P, P, I64, D, P, P, P, P]
        L.cd_screening_heating.argtypes = [P, I64, I, D, D, P, P, P, D, P, P, P, P, P]
        L.cd_weight_lists.argtypes = [P, I, I, P, P, P, P, P, P, P]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != CD_OK:
        raise ColdenError(rc, lib().cd_last_error().decode())


def _np(a):
    return a.ctypes.data_as(C.c_void_p)


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def directions(scheme: int, p1: int, p2: int = 0) -> np.ndarray:
    cap = 4096
    out = np.zeros((cap, 3))
    D = C.c_int(0)
    _check(lib().cd_directions(scheme, p1, p2, _np(out), cap, C.byref(D)))
    return out[:D.value].copy()


def weight_lists(dirs: np.ndarray, kind: int) -> dict:
    """The library's FP64 geometric factors K of one shell kind (1..4: dl = 1,
    2, 3, >= 4; 0: internal + local), as cd_weight_lists returns them (host
    only, no device): off [c][d][e][3], w [c][d][e], cnt [c][d], ref [c][3],
    box [c][3][4]."""
    dirs = np.ascontiguousarray(dirs, dtype=np.float64)
    D = dirs.shape[0]
    nc, ln = C.c_int(0), C.c_int(0)
    _check(lib().cd_weight_lists(_np(dirs), D, kind, C.byref(nc), C.byref(ln), None, None, None, None, None))
    nc, ln = nc.value, ln.value
    off = np.zeros((nc, D, ln, 3), np.int32)
    w = np.zeros((nc, D, ln))
    cnt = np.zeros((nc, D), np.int32)
    ref = np.zeros((nc, 3))
    box = np.zeros((nc, 3, 4), np.int32)
    _check(lib().cd_weight_lists(_np(dirs), D, kind, C.byref(C.c_int(0)), C.byref(C.c_int(0)), _np(off), _np(w),
                                 _np(cnt), _np(ref), _np(box)))
    return {"off": off, "w": w, "cnt": cnt, "ref": ref, "box": box}


def _dev(t, dtype, name: str, shape=None, numel=None):
    """Device pointer of a contiguous CUDA tensor of the given dtype, shape
    and element count (ValueError otherwise)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")
    if not t.is_cuda:
        raise ValueError(f"{name}: expected a CUDA tensor, got one on {t.device}")
    return C.c_void_p(t.data_ptr())


def _dev_f32(t, name: str = "buffer", shape=None, numel=None):
    import torch
    return _dev(t, torch.float32, name, shape, numel)


def _workspace(nbytes: int, device):
    """A torch-allocated device workspace (the caching allocator's blocks are
    at least 512-byte aligned)."""
    import torch
    ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    if ws.data_ptr() % 256:
        raise RuntimeError("torch returned a workspace that is not 256-byte aligned")
    return ws


class Tree:
    """cd_tree handle.  `leaf_n` is a float32 CUDA tensor in leaf order; for
    uniform grids the tree keeps reading it until the next update (keep it
    alive and unchanged).  The tree's device memory is a torch uint8 tensor
    (`workspace`) sized by cd_tree_workspace_bytes for sweeps of up to
    `max_dirs` directions; with `aux_stream` the sweep runs its side-by-side
    stages on a second torch stream (default priority)."""

    def __init__(self, tin, leaf_n, stream=None, max_dirs: int = CD_MAX_DIRS, aux_stream: bool = True):
        import torch
        # the leaf count is the array's; the library checks it against the structure
        if isinstance(leaf_n, torch.Tensor) and leaf_n.dim() != 1:
            raise ValueError(f"leaf_n: expected a 1-D tensor, got {tuple(leaf_n.shape)}")
        leaf_p = _dev_f32(leaf_n, "leaf_n")
        n_leaf = int(leaf_n.numel())
        self._keep_leaf = leaf_n
        self._par = [np.ascontiguousarray(p, dtype=np.int32) for p in tin.oct_parents]
        for p in self._par:
            if p.ndim != 2 or p.shape[1] != 3:
                raise ValueError(f"oct_parents: expected [n_octs, 3] arrays, got {p.shape}")
        n_octs = np.array([p.shape[0] for p in self._par] + [0], dtype=np.int64)
        ptrs = (C.c_void_p * (len(self._par) + 1))(*[p.ctypes.data for p in self._par], None)
        args = (int(tin.base_level), int(tin.max_level), _np(n_octs) if self._par else None,
                C.cast(ptrs, C.c_void_p), n_leaf, int(max_dirs))
        nbytes = C.c_size_t(0)
        _check(lib().cd_tree_workspace_bytes(*args, C.byref(nbytes)))
        self.workspace = _workspace(nbytes.value, leaf_n.device)
        h = C.c_void_p()
        _check(lib().cd_build_tree(float(tin.box_cm), int(tin.base_level), int(tin.max_level), args[2], args[3],
                                   leaf_p, n_leaf, int(max_dirs), C.c_void_p(self.workspace.data_ptr()),
                                   self.workspace.numel(), _stream(stream), C.byref(h)))
        self.h = h
        self.n_leaf = n_leaf
        self.max_level = int(tin.max_level)
        self.max_dirs = int(max_dirs)
        self.aux = None
        if aux_stream:
            self.aux = torch.cuda.Stream(device=leaf_n.device)
            _check(lib().cd_tree_set_aux_stream(self.h, C.c_void_p(self.aux.cuda_stream)))

    def update(self, leaf_n, stream=None):
        p = _dev_f32(leaf_n, "leaf_n", numel=self.n_leaf)
        self._keep_leaf = leaf_n
        _check(lib().cd_tree_update(self.h, p, self.n_leaf, _stream(stream)))

    def profile(self, on: bool = True):
        """Record HIP events around each stage of later calls on this tree."""
        _check(lib().cd_profile_enable(self.h, 1 if on else 0))

    def stage_ms(self) -> dict:
        """Stage durations (ms) of the last profiled calls."""
        ms = np.zeros(len(STAGES), np.float32)
        _check(lib().cd_profile_read(self.h, _np(ms)))
        return dict(zip(STAGES, ms.tolist()))

    def leaf_coords(self):
        lv = np.zeros(self.n_leaf, np.int8)
        ijk = np.zeros((self.n_leaf, 3), np.int32)
        _check(lib().cd_tree_leaf_coords(self.h, _np(lv), _np(ijk)))
        return lv, ijk

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            import torch
            torch.cuda.synchronize()  # the workspace is released with the handle
            lib().cd_tree_destroy(self.h)
        self.h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Weights:
    """cd_weights handle (precalculated geometric factors, uploaded once)."""

    def __init__(self, dirs: np.ndarray, mode: int = CD_PRECALC73, precision: int = CD_FP32,
                 stream=None, device=None):
        import torch
        dirs = np.ascontiguousarray(dirs, dtype=np.float64)
        if dirs.ndim != 2 or dirs.shape[1] != 3:
            raise ValueError(f"dirs: expected [D, 3], got {dirs.shape}")
        nbytes = C.c_size_t(0)
        _check(lib().cd_weights_workspace_bytes(_np(dirs), dirs.shape[0], mode, precision, C.byref(nbytes)))
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.workspace = _workspace(nbytes.value, dev)
        h = C.c_void_p()
        _check(lib().cd_precompute_weights(_np(dirs), dirs.shape[0], mode, precision,
                                           C.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                           _stream(stream), C.byref(h)))
        self.h = h
        self.D = dirs.shape[0]
        self.precision = precision

    def split_steps(self) -> int:
        """32-offset steps of the split contraction summed over classes,
        shells dl = 1..3 and direction tiles (0 for FP32 weights)."""
        n = C.c_int64(0)
        _check(lib().cd_weights_split_steps(self.h, C.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            import torch
            torch.cuda.synchronize()  # the workspace is released with the handle
            lib().cd_weights_destroy(self.h)
        self.h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def column_densities(tree: Tree, w: Weights, N, chi=None, av_per_nh: float = AV_PER_NH,
                     gamma: float = GAMMA, stream=None):
    """N: float32 CUDA tensor [n_leaf, D]; chi: optional float32 [n_leaf]."""
    Np = _dev_f32(N, "N", shape=(tree.n_leaf, w.D))
    chip = _dev_f32(chi, "chi", numel=tree.n_leaf) if chi is not None else None
    _check(lib().cd_column_densities(tree.h, w.h, Np, chip, av_per_nh, gamma, _stream(stream)))
    return N


def column_densities_log16(tree: Tree, w: Weights, Ncode, chi=None, av_per_nh: float = AV_PER_NH,
                           gamma: float = GAMMA, stream=None):
    """Ncode: int16 CUDA tensor [n_leaf, D] receiving the packed columns
    (16-bit codes c, N = 2^(40 + c / 1024), c read as unsigned; see
    decode_log16); chi: optional float32 [n_leaf]."""
    import torch
    Cp = _dev(Ncode, torch.int16, "Ncode", shape=(tree.n_leaf, w.D))
    chip = _dev_f32(chi, "chi", numel=tree.n_leaf) if chi is not None else None
    _check(lib().cd_column_densities_log16(tree.h, w.h, Cp, chip, av_per_nh, gamma, _stream(stream)))
    return Ncode


def decode_log16(Ncode):
    """Columns (cm^-2, float64) from the packed codes of column_densities_log16."""
    import torch
    c = Ncode.to(torch.int32) & 0xFFFF
    return torch.exp2(40.0 + c.to(torch.float64) / 1024.0)


def check_densities(leaf_n, stream=None) -> int:
    """Number of entries of a float32 CUDA tensor that are negative, NaN or
    infinite (synchronises the stream)."""
    import torch
    p = _dev_f32(leaf_n, "leaf_n")
    scratch = torch.empty(1, dtype=torch.int64, device=leaf_n.device)
    bad = C.c_int64(0)
    _check(lib().cd_check_densities(p, int(leaf_n.numel()), C.c_void_p(scratch.data_ptr()), C.byref(bad),
                                    _stream(stream)))
    return bad.value


def heating_rates(chi, n, T, ne, gamma_uv, g0eff=None, gamma_cr=None, G0: float = G0_DRAINE, stream=None):
    """Photoelectric and cosmic-ray heating rates (Sect. 5) from chi."""
    m = int(chi.numel())
    ck = lambda t, nm: _dev_f32(t, nm, numel=m)
    _check(lib().cd_heating_rates(ck(chi, "chi"), ck(n, "n"), ck(T, "T"), ck(ne, "ne"), m, G0,
                                  ck(g0eff, "g0eff") if g0eff is not None else None, ck(gamma_uv, "gamma_uv"),
                                  ck(gamma_cr, "gamma_cr") if gamma_cr is not None else None, _stream(stream)))
    return gamma_uv


def screening_heating(N, n, T, ne, gamma_uv, chi=None, g0eff=None, gamma_cr=None, G0: float = G0_DRAINE,
                      av_per_nh: float = AV_PER_NH, gamma: float = GAMMA, stream=None):
    """chi (Eq. 7) from N and the heating rates in one pass."""
    if N.dim() != 2:
        raise ValueError(f"N: expected [n_cells, D], got {tuple(N.shape)}")
    cells, D = N.shape
    ck = lambda t, nm: _dev_f32(t, nm, numel=cells) if t is not None else None
    _check(lib().cd_screening_heating(_dev_f32(N, "N"), cells, D, av_per_nh, gamma, ck(n, "n"), ck(T, "T"),
                                      ck(ne, "ne"), G0, ck(chi, "chi"), ck(g0eff, "g0eff"), ck(gamma_uv, "gamma_uv"),
                                      ck(gamma_cr, "gamma_cr"), _stream(stream)))
    return gamma_uv


def screening_factor(N, chi, av=None, av_per_nh: float = AV_PER_NH, gamma: float = GAMMA, stream=None):
    if N.dim() != 2:
        raise ValueError(f"N: expected [n_leaf, D], got {tuple(N.shape)}")
    n, D = N.shape
    _check(lib().cd_screening_factor(_dev_f32(N, "N"), n, D, av_per_nh, gamma, _dev_f32(chi, "chi", numel=n),
                                     _dev_f32(av, "av", shape=(n, D)) if av is not None else None,
                                     _stream(stream)))
    return chi


# ------------------------------------------------------------- surrogate --
CD_SURR_FP32, CD_SURR_BF16 = 0, 1
SURROGATE_EXPORTS = [
    "cd_surrogate_create", "cd_surrogate_destroy", "cd_surrogate_n_params", "cd_surrogate_get_params",
    "cd_surrogate_set_params", "cd_surrogate_features", "cd_surrogate_targets", "cd_surrogate_forward", "cd_surrogate_gradients",
    "cd_surrogate_train_step", "cd_surrogate_infer", "cd_surrogate_check_fallback", "cd_surrogate_save",
    "cd_surrogate_load", "cd_surrogate_info", "cd_surrogate_row_targets", "cd_surrogate_train_step_rows",
]
EXPORTS += SURROGATE_EXPORTS
N_FEAT = 576


def _surr_types():
    L = lib()
    if getattr(L, "_surr_typed", False):
        return L
    P, I, I64, D, F = C.c_void_p, C.c_int, C.c_int64, C.c_double, C.c_float
    L.cd_surrogate_create.argtypes = [I, I, I, I, C.c_uint64, P, P]
    L.cd_surrogate_info.argtypes = [P, P]
    L.cd_surrogate_row_targets.argtypes = [P, P, P, P, P]
    L.cd_surrogate_train_step_rows.argtypes = [P, P, P, P, I64, F, P, P]
    L.cd_surrogate_destroy.argtypes = [P]
    L.cd_surrogate_destroy.restype = None
    L.cd_surrogate_n_params.argtypes = [P, P]
    L.cd_surrogate_get_params.argtypes = [P, P]
    L.cd_surrogate_set_params.argtypes = [P, P]
    L.cd_surrogate_features.argtypes = [P, P, P, I64, P, P]
    L.cd_surrogate_targets.argtypes = [P, P, P, P, I64, P, P]
    L.cd_surrogate_forward.argtypes = [P, P, I64, P, P]
    L.cd_surrogate_gradients.argtypes = [P, P, P, I64, P, P, P]
    L.cd_surrogate_train_step.argtypes = [P, P, P, P, I64, F, P, P]
    L.cd_surrogate_infer.argtypes = [P, P, P, P, P, D, D, P]
    L.cd_surrogate_check_fallback.argtypes = [P, P, P, D, D, C.c_uint64, P, P, D, D, P, P, P, P]
    L.cd_surrogate_save.argtypes = [P, C.c_char_p]
    L.cd_surrogate_load.argtypes = [C.c_char_p, P]
    L._surr_typed = True
    return L


def _dev_i64(t, name: str = "cells", numel=None):
    import torch
    if isinstance(t, torch.Tensor) and t.dim() != 1:
        raise ValueError(f"{name}: expected a 1-D index tensor, got {tuple(t.shape)}")
    return _dev(t, torch.int64, name, numel=numel)


class Surrogate:
    """cd_surrogate handle: ReLU MLP 576 -> width -> width -> Dout on the
    pyramid features of a level-7 cell, Dout = D for each of the
    8^(leaf_level - 8) octs inside it; trained and run by the library's
    kernels."""

    ROWS = 1 << 21  # level-7 cells

    def __init__(self, D: int = 12, width: int = 256, precision: int = CD_SURR_BF16, seed: int = 0,
                 norm=(0.0, 1.0, 0.0, 1.0), leaf_level: int = 8, _handle=None):
        L = _surr_types()
        if _handle is None:
            nrm = np.asarray(norm, dtype=np.float32)
            h = C.c_void_p()
            _check(L.cd_surrogate_create(D, leaf_level, width, precision, seed, _np(nrm), C.byref(h)))
            _handle = h
        self.h = _handle
        info = np.zeros(5, np.int32)
        _check(L.cd_surrogate_info(self.h, _np(info)))
        self.D, self.leaf_level, self.width, self.precision, self.Dout = (int(v) for v in info)

    @classmethod
    def load(cls, path: str) -> "Surrogate":
        L = _surr_types()
        h = C.c_void_p()
        _check(L.cd_surrogate_load(path.encode(), C.byref(h)))
        return cls(_handle=h)

    def save(self, path: str):
        _check(_surr_types().cd_surrogate_save(self.h, path.encode()))

    def n_params(self) -> int:
        n = C.c_int64(0)
        _check(_surr_types().cd_surrogate_n_params(self.h, C.byref(n)))
        return n.value

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.n_params(), np.float32)
        _check(_surr_types().cd_surrogate_get_params(self.h, _np(p)))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(_surr_types().cd_surrogate_set_params(self.h, _np(p)))

    def _rows(self, t, name: str, n: int, cols):
        """Pointer of a float32 [n, cols] tensor (cols None: any 2-D width)."""
        if t.dim() != 2 or t.shape[0] != n or (cols is not None and t.shape[1] != cols):
            raise ValueError(f"{name}: expected shape ({n}, {cols if cols is not None else 'D'}), "
                             f"got {tuple(t.shape)}")
        return _dev_f32(t, name)

    def features(self, tree: Tree, cells, X, stream=None):
        n = int(cells.numel())
        _check(_surr_types().cd_surrogate_features(self.h, tree.h, _dev_i64(cells), n,
                                                   self._rows(X, "X", n, N_FEAT), _stream(stream)))
        return X

    def targets(self, tree: Tree, w: Weights, cells, T, stream=None):
        """Scaled near-shell targets of the level-7 cells of `cells` into T [n, Dout]."""
        n = int(cells.numel())
        _check(_surr_types().cd_surrogate_targets(self.h, tree.h, w.h, _dev_i64(cells), n,
                                                  self._rows(T, "T", n, self.Dout), _stream(stream)))
        return T

    def row_targets(self, tree: Tree, w: Weights, T_rows, stream=None):
        """Unscaled near-shell targets of every level-7 cell into T_rows [2^21, Dout]."""
        _check(_surr_types().cd_surrogate_row_targets(self.h, tree.h, w.h,
                                                      self._rows(T_rows, "T_rows", self.ROWS, self.Dout),
                                                      _stream(stream)))
        return T_rows

    def forward(self, X, Y, stream=None):
        n = int(X.shape[0]) if X.dim() == 2 else -1
        _check(_surr_types().cd_surrogate_forward(self.h, self._rows(X, "X", n, N_FEAT), n,
                                                  self._rows(Y, "Y", n, self.Dout), _stream(stream)))
        return Y

    def gradients(self, X, T, stream=None):
        g = np.zeros(self.n_params(), np.float32)
        loss = C.c_float(0)
        n = int(X.shape[0]) if X.dim() == 2 else -1
        _check(_surr_types().cd_surrogate_gradients(self.h, self._rows(X, "X", n, N_FEAT),
                                                    self._rows(T, "T", n, self.Dout), n, _np(g),
                                                    C.byref(loss), _stream(stream)))
        return g, loss.value

    def train_step(self, tree: Tree, w: Weights, cells, lr: float, want_loss: bool = False, stream=None):
        loss = C.c_float(0)
        _check(_surr_types().cd_surrogate_train_step(self.h, tree.h, w.h, _dev_i64(cells),
                                                     int(cells.numel()), float(lr),
                                                     C.byref(loss) if want_loss else None, _stream(stream)))
        return loss.value if want_loss else None

    def train_step_rows(self, tree: Tree, T_rows, rows, lr: float, want_loss: bool = False, stream=None):
        """Adam step on level-7 cells `rows` (int64), features from `tree`,
        targets from a row_targets table."""
        loss = C.c_float(0)
        _check(_surr_types().cd_surrogate_train_step_rows(self.h, tree.h,
                                                          self._rows(T_rows, "T_rows", self.ROWS, self.Dout),
                                                          _dev_i64(rows), int(rows.numel()), float(lr),
                                                          C.byref(loss) if want_loss else None, _stream(stream)))
        return loss.value if want_loss else None

    def infer(self, tree: Tree, w: Weights, N, chi=None, av_per_nh: float = AV_PER_NH, gamma: float = GAMMA,
              stream=None):
        _check(_surr_types().cd_surrogate_infer(self.h, tree.h, w.h, _dev_f32(N, "N", shape=(tree.n_leaf, w.D)),
                                                _dev_f32(chi, "chi", numel=tree.n_leaf) if chi is not None else None,
                                                av_per_nh, gamma, _stream(stream)))
        return N

    def check_fallback(self, tree: Tree, w: Weights, N, chi, frac: float = 0.01, tol_chi: float = 0.03,
                       seed: int = 0, av_per_nh: float = AV_PER_NH, gamma: float = GAMMA, stream=None):
        nf, nt, emax = C.c_int64(0), C.c_int64(0), C.c_float(0)
        _check(_surr_types().cd_surrogate_check_fallback(self.h, tree.h, w.h, frac, tol_chi, seed,
                                                         _dev_f32(N, "N", shape=(tree.n_leaf, w.D)),
                                                         _dev_f32(chi, "chi", numel=tree.n_leaf), av_per_nh, gamma,
                                                         C.byref(nf), C.byref(nt), C.byref(emax), _stream(stream)))
        return nf.value, nt.value, emax.value

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            _surr_types().cd_surrogate_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
