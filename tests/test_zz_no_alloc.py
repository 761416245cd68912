"""cd_check_densities_noalloc (the entry point for callers that cannot
allocate device memory) against cd_check_densities with a caller scratch, on
two calls in a row, the second on a smaller input (its scratch keeps the
last call's count, so the count must be cleared by each call)."""
import ctypes

import numpy as np
import pytest

from paper_1410_0624_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def colden():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1410_0624_amd import colden as c
    c.lib().cd_check_densities_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                                   ctypes.c_void_p]
    return c


def _noalloc(colden, buf, n):
    bad = ctypes.c_int64(-1)
    rc = colden.lib().cd_check_densities_noalloc(ctypes.c_void_p(buf.data_ptr()), n, ctypes.byref(bad),
                                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, colden.lib().cd_last_error().decode()
    return bad.value


def _with_scratch(colden, buf, n):
    scratch = torch.empty(1, dtype=torch.int64, device=buf.device)
    bad = ctypes.c_int64(-1)
    rc = colden.lib().cd_check_densities(ctypes.c_void_p(buf.data_ptr()), n, ctypes.c_void_p(scratch.data_ptr()),
                                         ctypes.byref(bad), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, colden.lib().cd_last_error().decode()
    return bad.value


def test_noalloc_check_matches_the_scratch_form(colden):
    dev = torch.device("cuda:0")
    tin = synth.workload_uniform(6, seed=3)
    leaf = torch.from_numpy(tin.leaf_n).to(dev)
    rng = np.random.default_rng(5)
    bad_at = rng.choice(tin.n_leaf, 517, replace=False)
    vals = torch.tensor([float("nan"), -1.0, float("inf"), float("-inf")], device=dev)
    leaf[torch.from_numpy(bad_at).to(dev)] = vals[torch.from_numpy(bad_at % 4).to(dev)]
    # first call: the whole array; second call: a smaller prefix
    n_small = 100000
    want_small = int((bad_at < n_small).sum())
    for n, want in [(tin.n_leaf, 517), (n_small, want_small)]:
        a = _noalloc(colden, leaf, n)
        b = _with_scratch(colden, leaf, n)
        print(f"n = {n}: noalloc {a}, scratch form {b}, expected {want}")
        assert a == b == want
    # an empty input and a clean one after a dirty one
    assert _noalloc(colden, leaf, 0) == 0
    clean = torch.from_numpy(tin.leaf_n).to(dev)
    assert _noalloc(colden, clean, tin.n_leaf) == 0
    # argument errors are reported, nothing runs
    bad = ctypes.c_int64(0)
    assert colden.lib().cd_check_densities_noalloc(None, 5, ctypes.byref(bad), None) == colden.CD_EINVAL
    assert colden.lib().cd_check_densities_noalloc(ctypes.c_void_p(leaf.data_ptr()), -1, ctypes.byref(bad),
                                                   None) == colden.CD_EINVAL
