"""The allocation-free product (spm_masked_gemm_noalloc, workspace in the library's
fixed device array) against the allocating spm_masked_gemm, through the C ABI.

Same kernels, so the results must agree bit for bit: in every precision and
transpose combination, on two calls in a row where the second product is smaller
than the first (the array keeps the first call's contents, which the second must
not read).  A product needing more workspace than the array holds is refused
before any work.
"""
import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def _problem(S, kind, n, leaf, q, eta, seed):
    pts = synth.workload_points(kind, n, seed)
    t = S.Tree(pts, leaf, q)
    pat = S.Pattern.from_tree(t, eta)
    nst = pat.n_stored
    a = torch.from_numpy(2.0 * synth.uniform(seed * 10 + 1, np.arange(nst)) - 1.0).cuda()
    b = torch.from_numpy(2.0 * synth.uniform(seed * 10 + 2, np.arange(nst)) - 1.0).cuda()
    return t, pat, a, b


def test_noalloc_matches_allocating_product():
    from paper_2211_11681_amd import _lib
    from paper_2211_11681_amd import spm as S
    lib = _lib.load()
    assert torch.cuda.is_available()
    cap = ctypes.c_size_t()
    assert lib.spm_masked_gemm_noalloc_max_bytes(ctypes.byref(cap)) == 0
    assert cap.value == 64 << 20
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # products of decreasing size on three patterns (ragged leaves, all unit classes)
    cases = [("cube2", 3000, 32, 2, 1.6, 3), ("cube3", 2048, 32, 1, 1.0, 2), ("cube2", 1024, 16, 1, 1.6, 1)]
    sizes = []
    for kind, n, leaf, q, eta, seed in cases:
        print(f"case: noalloc product {kind} n={n} leaf={leaf} q={q} eta={eta}", flush=True)
        t, pat, a, b = _problem(S, kind, n, leaf, q, eta, seed)
        sizes.append(pat.n_stored)
        for prec in ("f64", "f32acc", "f32split"):
            pc = S.prec_code(prec)
            A = a if prec == "f64" else S.convert(pat, a, "f64", prec)
            B = b if prec == "f64" else S.convert(pat, b, "f64", prec)
            for ta, tb in [(0, 0), (1, 0), (0, 1), (1, 1)]:
                need = S.gemm_workspace_bytes(pat, prec, bool(ta), bool(tb))
                assert need <= cap.value
                C1, C2 = pat.empty(prec), pat.empty(prec)
                C2.fill_(float("nan"))
                assert lib.spm_masked_gemm(pat._h, pc, _vp(A), ta, _vp(B), tb, _vp(C1), stream) == 0
                st = lib.spm_masked_gemm_noalloc(pat._h, pc, _vp(A), ta, _vp(B), tb, _vp(C2), stream)
                assert st == 0, lib.spm_last_error()
                torch.cuda.synchronize()
                assert torch.equal(C1, C2), (kind, prec, ta, tb)
        del pat, t
    assert sizes[2] < sizes[1] < sizes[0]


def test_noalloc_refuses_oversized_workspace():
    from paper_2211_11681_amd import _lib
    from paper_2211_11681_amd import spm as S
    lib = _lib.load()
    print("case: noalloc refusal n=16384 cube3", flush=True)
    t, pat, a, b = _problem(S, "cube3", 16384, 32, 1, 1.0, 4)
    cap = ctypes.c_size_t()
    lib.spm_masked_gemm_noalloc_max_bytes(ctypes.byref(cap))
    assert S.gemm_workspace_bytes(pat, "f64", False, False) > cap.value
    C = pat.empty("f64")
    C.fill_(1.5)
    st = lib.spm_masked_gemm_noalloc(pat._h, 0, _vp(a), 0, _vp(b), 0, _vp(C), None)
    assert st == -1 and b"above the fixed" in lib.spm_last_error()
    torch.cuda.synchronize()
    assert bool(torch.all(C == 1.5))                       # nothing was launched
    # with the transpose of B not needed (op(B) = B^T) the same product fits only if
    # its workspace does: P_S(A B^T) needs none in FP64
    assert S.gemm_workspace_bytes(pat, "f64", False, True) == 0
    C2 = pat.empty("f64")
    st = lib.spm_masked_gemm_noalloc(pat._h, 0, _vp(a), 0, _vp(b), 1, _vp(C2), None)
    assert st == 0, lib.spm_last_error()
    C3 = S.masked_gemm(pat, a, b, transB=True)
    torch.cuda.synchronize()
    assert torch.equal(C2, C3)
