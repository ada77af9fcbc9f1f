"""CPU checks of libspm: exported symbols, the host-side construction (tree,
cluster ranges, block pattern) bit-exact against the oracle, and the pattern
validation errors that fire before any device call."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import pattern, samplets, tree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2211_11681_amd import _lib
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "spm.h")).read()
    names = set(re.findall(r"\b(spm_[a-z0-9_]+)\s*\(", hdr))
    assert len(names) >= 25
    for n in sorted(names):
        assert hasattr(lib, n), n
    from paper_2211_11681_amd import _lib
    assert set(_lib.SIGNATURES) | {"spm_status_string", "spm_last_error"} == names


def test_binding_arity_matches_header():
    """Every ctypes signature has as many arguments as the header's declaration."""
    hdr = open(os.path.join(ROOT, "include", "spm.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    from paper_2211_11681_amd import _lib
    for name, args in _lib.SIGNATURES.items():
        m = re.search(r"\b" + name + r"\s*\(([^)]*)\)\s*;", hdr)
        assert m, name
        params = [x for x in m.group(1).split(",") if x.strip() and x.strip() != "void"]
        assert len(params) == len(args), (name, len(params), len(args))


CASES = [("cube2", 2048, 16, 1, 1.6, 1), ("cube3", 4096, 32, 1, 1.0, 2), ("cube2", 4096, 32, 2, 1.6, 3),
         ("sphere", 4096, 32, 1, 1.0, 5), ("cube3", 3000, 32, 1, 1.0, 4), ("cube2", 777, 16, 1, 0.7, 8)]


@pytest.mark.parametrize("kind,n,leaf,q,eta,seed", CASES)
def test_tree_and_pattern_bit_exact(lib, kind, n, leaf, q, eta, seed):
    from paper_2211_11681_amd.spm import Tree
    pts = synth.workload_points(kind, n, seed)
    t = Tree(pts, leaf, q)
    arr = t.arrays()
    ot = tree.build_tree(pts, leaf)
    ob = samplets.build_samplets(ot, q)
    assert t.n_clusters == ot.n_clusters and t.depth == ot.depth and t.m == ob.m
    assert np.array_equal(arr["perm"], ot.perm)
    assert np.array_equal(arr["pt_start"], ot.start) and np.array_equal(arr["pt_size"], ot.size)
    assert np.array_equal(arr["level"], ot.level)
    assert np.array_equal(arr["cluster_start"], ob.cluster_start)
    rp, col = t.block_pattern(eta)
    orp, ocol = pattern.block_csr(pattern.block_pattern(ot, eta))
    assert np.array_equal(rp, orp) and np.array_equal(col, ocol)


def _upload_csr(lib, n, rp, col, cs):
    rp = np.ascontiguousarray(rp, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    cs = np.ascontiguousarray(cs, np.int64)
    h = ctypes.c_void_p()
    st = lib.spm_compress_pattern_upload(n, rp.ctypes.data_as(ctypes.c_void_p), col.ctypes.data_as(ctypes.c_void_p),
                                         len(cs) - 1, cs.ctypes.data_as(ctypes.c_void_p), None, ctypes.byref(h))
    return st, lib.spm_last_error().decode()


def _dense_csr(mask):
    rp = np.zeros(mask.shape[0] + 1, np.int64)
    rp[1:] = np.cumsum(mask.sum(1))
    return rp, np.nonzero(mask)[1].astype(np.int32)


def test_pattern_validation_errors(lib):
    n = 8
    cs = np.array([0, 2, 4, 6, 8])
    full = np.ones((n, n), bool)
    rp, col = _dense_csr(full)
    # unsorted columns
    c2 = col.copy(); c2[[0, 1]] = c2[[1, 0]]
    assert _upload_csr(lib, n, rp, c2, cs)[0] == -2
    # duplicate column
    c3 = col.copy(); c3[1] = c3[0]
    assert _upload_csr(lib, n, rp, c3, cs)[0] == -2
    # out of range
    c4 = col.copy(); c4[-1] = n
    assert _upload_csr(lib, n, rp, c4, cs)[0] == -2
    # not symmetric
    m = full.copy(); m[0, 7] = False
    st, msg = _upload_csr(lib, n, *_dense_csr(m), cs)
    assert st == -2 and "symmetric" in msg
    # missing diagonal
    m = full.copy(); m[3, 3] = False
    st, msg = _upload_csr(lib, n, *_dense_csr(m), cs)
    assert st == -2 and "diagonal" in msg
    # cluster ranges that do not tile [0, n)
    assert _upload_csr(lib, n, rp, col, np.array([0, 2, 4, 6, 7]))[0] == -2
    assert _upload_csr(lib, n, rp, col, np.array([1, 2, 4, 6, 8]))[0] == -2
    # more than 32 functions in one cluster
    big = 40
    rpb, colb = _dense_csr(np.ones((big, big), bool))
    assert _upload_csr(lib, big, rpb, colb, np.array([0, big]))[0] == -6
    # null pointers and bad sizes
    h = ctypes.c_void_p()
    assert lib.spm_compress_pattern_upload(n, None, None, 4, None, None, ctypes.byref(h)) == -1
    assert lib.spm_block_pattern_upload(0, 1, None, None, None, None, ctypes.byref(h)) == -1
    pts = np.zeros((4, 2))
    assert lib.spm_tree_build(pts.ctypes.data_as(ctypes.c_void_p), 4, 5, 16, 1, ctypes.byref(h)) == -1
    assert lib.spm_masked_gemm(None, 0, None, 0, None, 0, None, None) == -1
    assert lib.spm_status_string(-2) == b"invalid pattern"


def test_block_pattern_validation(lib):
    cs = np.array([0, 3, 6, 9], np.int64)
    rp = np.array([0, 2, 4, 6], np.int64)
    col = np.array([0, 1, 0, 1, 1, 2], np.int32)     # (2,2) present, (2,1) present but (1,2) missing
    h = ctypes.c_void_p()
    P = ctypes.c_void_p
    st = lib.spm_block_pattern_upload(9, 3, cs.ctypes.data_as(P), rp.ctypes.data_as(P), col.ctypes.data_as(P),
                                      None, ctypes.byref(h))
    assert st == -2


def test_tree_rejects_too_many_functions(lib):
    from paper_2211_11681_amd._lib import SpmError
    from paper_2211_11681_amd.spm import Tree
    with pytest.raises(SpmError) as e:
        Tree(synth.points_cube(512, 2, 1), 64, 1)       # leaves of 64 points own 61 samplets
    assert e.value.status == -6


@pytest.mark.parametrize("lo,hi,nodes,rtol", [(1e-2, 1.01, 7, 1e-12), (1e-4, 1.0, 12, 1e-12), (0.5, 2.0, 3, 1e-12),
                                              (1.0, 1.0, 4, 1e-12), (1e-8, 10.0, 20, 2e-11), (0.3, 0.3, 5, 1e-12)])
def test_contour_rule_matches_oracle(lib, lo, hi, nodes, rtol):
    """Host-side shifts and weights of the contour quadrature (Section 4.4) against the
    oracle's rule, which evaluates the Jacobi functions with scipy.  At a spectral ratio
    of 1e-9 the parameter sits 1e-9 below 1, where the two evaluations (descending
    Landen here, scipy's own there) part by a few 1e-12."""
    from oracle import ops
    from paper_2211_11681_amd import spm
    w2, c = spm.contour_rule(lo, hi, nodes)
    ow2, oc = ops.contour_invsqrt_rule(lo, hi, nodes)
    np.testing.assert_allclose(w2, ow2, rtol=rtol, atol=0)
    np.testing.assert_allclose(c, oc, rtol=rtol, atol=0)
    if lo == hi:   # parameter 0: the rule is exact at lam = lo (closed form)
        assert np.sum(c / (lo + w2)) == pytest.approx(lo ** -0.5, rel=1e-14)


def test_contour_rule_errors(lib):
    w = np.empty(4)
    for lo, hi, k in [(0.0, 1.0, 4), (2.0, 1.0, 4), (1.0, 2.0, 0), (float("nan"), 1.0, 4), (1.0, float("inf"), 4)]:
        st = lib.spm_contour_rule(lo, hi, k, w.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p))
        assert st == -1, (lo, hi, k)   # SPM_EINVAL
