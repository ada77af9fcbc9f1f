"""Python binding of libspm: the same operations as include/spm.h, on torch tensors.

Argument marshalling only: every step runs in libspm (host C++ or HIP kernels);
torch provides device memory and the current HIP stream.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import call

F64, F32SPLIT, F32ACC = 0, 1, 2
_PREC = {"f64": F64, "f32split": F32SPLIT, "f32acc": F32ACC}


def prec_code(prec) -> int:
    return _PREC[prec] if isinstance(prec, str) else int(prec)


def _ptr(a) -> ctypes.c_void_p:
    if a is None:
        return ctypes.c_void_p(0)
    if isinstance(a, torch.Tensor):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _host(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _check_vals(pat: "Pattern", t, prec, name: str, what: str = "operand"):
    """A value array of `pat` in precision `prec`: device tensor of the right dtype and
    length, contiguous (the library reads and writes n_stored values through it)."""
    p = prec_code(prec)
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: {what} must be a torch tensor")
    want = torch.float64 if p == F64 else torch.float32
    n = pat.n_stored * (2 if p == F32SPLIT else 1)
    if t.dtype != want or t.numel() != n or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name}: {what} must be a contiguous CUDA {want} tensor of {n} values "
                         f"(got {t.dtype}, {t.numel()} values, device {t.device}, "
                         f"contiguous={t.is_contiguous()})")


def _workspace(nbytes: int, device) -> torch.Tensor | None:
    """Device workspace from torch's allocator (256-byte aligned blocks)."""
    if nbytes == 0:
        return None
    return torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=device)


class Tree:
    """Cluster tree and samplet basis of a point set (library construction)."""

    def __init__(self, points: np.ndarray, leaf_size: int, q: int):
        pts = _host(points, np.float64)
        n, d = pts.shape
        h = ctypes.c_void_p()
        call("spm_tree_build", _ptr(pts), n, d, leaf_size, q, ctypes.byref(h))
        self._h = h
        self.n, self.d = n, d
        nc, depth, m = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        call("spm_tree_info", h, ctypes.byref(nc), ctypes.byref(depth), ctypes.byref(m))
        self.n_clusters, self.depth, self.m = nc.value, depth.value, m.value

    def arrays(self):
        nc = self.n_clusters
        perm = np.empty(self.n, np.int64)
        cs = np.empty(nc + 1, np.int64)
        lev = np.empty(nc, np.int32)
        ps = np.empty(nc, np.int64)
        pz = np.empty(nc, np.int64)
        call("spm_tree_arrays", self._h, _ptr(perm), _ptr(cs), _ptr(lev), _ptr(ps), _ptr(pz))
        return dict(perm=perm, cluster_start=cs, level=lev, pt_start=ps, pt_size=pz)

    def block_pattern(self, eta: float):
        rp = np.empty(self.n_clusters + 1, np.int64)
        nb = ctypes.c_int64()
        call("spm_tree_block_pattern", self._h, eta, _ptr(rp), None, ctypes.byref(nb))
        col = np.empty(nb.value, np.int32)
        call("spm_tree_block_pattern", self._h, eta, _ptr(rp), _ptr(col), ctypes.byref(nb))
        return rp, col

    def __del__(self):
        try:
            if getattr(self, "_h", None) and _lib._lib is not None:
                _lib._lib.spm_tree_destroy(self._h)
                self._h = None
        except Exception:
            pass


class Pattern:
    """Device-resident tiled compression pattern."""

    def __init__(self, handle, n: int, n_clusters: int):
        self._h = handle
        self.n, self.n_clusters = n, n_clusters
        nnz, ns, nt, macs = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        call("spm_pattern_info", handle, ctypes.byref(nnz), ctypes.byref(ns), ctypes.byref(nt), ctypes.byref(macs))
        self.nnz, self.n_stored, self.n_tiles, self.macs = nnz.value, ns.value, nt.value, macs.value

    @classmethod
    def from_blocks(cls, n, cluster_start, blk_row_ptr, blk_col):
        cs = _host(cluster_start, np.int64)
        rp = _host(blk_row_ptr, np.int64)
        col = _host(blk_col, np.int32)
        h = ctypes.c_void_p()
        call("spm_block_pattern_upload", n, len(cs) - 1, _ptr(cs), _ptr(rp), _ptr(col), _stream(), ctypes.byref(h))
        return cls(h, n, len(cs) - 1)

    @classmethod
    def from_csr(cls, n, row_ptr, col_idx, cluster_start):
        rp = _host(row_ptr, np.int64)
        col = _host(col_idx, np.int32)
        cs = _host(cluster_start, np.int64)
        h = ctypes.c_void_p()
        call("spm_compress_pattern_upload", n, _ptr(rp), _ptr(col), len(cs) - 1, _ptr(cs), _stream(), ctypes.byref(h))
        return cls(h, n, len(cs) - 1)

    @classmethod
    def from_tree(cls, tree: Tree, eta: float):
        """Block pattern of the tree, planned with the clusters' levels and uploaded."""
        rp, col = tree.block_pattern(eta)
        arr = tree.arrays()
        pat = cls.plan_blocks(tree.n, arr["cluster_start"], rp, col, levels=arr["level"])
        pat.upload()
        return pat

    @classmethod
    def plan_blocks(cls, n, cluster_start, blk_row_ptr, blk_col, levels=None):
        """Host-only planning (no device memory); upload with upload() or upload_workspace()."""
        cs = _host(cluster_start, np.int64)
        rp = _host(blk_row_ptr, np.int64)
        col = _host(blk_col, np.int32)
        lev = None if levels is None else _host(levels, np.int32)
        h = ctypes.c_void_p()
        call("spm_block_pattern_plan", n, len(cs) - 1, _ptr(cs), _ptr(rp), _ptr(col), _ptr(lev), ctypes.byref(h))
        return cls(h, n, len(cs) - 1)

    @classmethod
    def plan_csr(cls, n, row_ptr, col_idx, cluster_start, levels=None):
        rp = _host(row_ptr, np.int64)
        col = _host(col_idx, np.int32)
        cs = _host(cluster_start, np.int64)
        lev = None if levels is None else _host(levels, np.int32)
        h = ctypes.c_void_p()
        call("spm_compress_pattern_plan", n, _ptr(rp), _ptr(col), len(cs) - 1, _ptr(cs), _ptr(lev), ctypes.byref(h))
        return cls(h, n, len(cs) - 1)

    def upload(self):
        """Uploads the device tables into a block the library allocates."""
        call("spm_pattern_upload", self._h, _stream())
        return self

    def workspace_bytes(self) -> int:
        b = ctypes.c_size_t()
        call("spm_pattern_workspace_bytes", self._h, ctypes.byref(b))
        return b.value

    def upload_workspace(self, device="cuda") -> torch.Tensor:
        """Uploads the device tables into a torch-owned buffer, kept by the pattern."""
        ws = torch.empty((self.workspace_bytes() + 7) // 8, dtype=torch.float64, device=device)
        call("spm_pattern_upload_workspace", self._h, _ptr(ws), ws.numel() * 8, _stream())
        self._ws = ws
        return ws

    def classes(self):
        """Launch classes of the product schedule: list of dicts (row_blocks, col_blocks,
        units, out_tiles, exact_macs, padded_macs)."""
        n = ctypes.c_int32(0)
        call("spm_pattern_classes", self._h, ctypes.byref(n), None, None, None, None, None, None)
        k = n.value
        rb, cb = np.empty(k, np.int32), np.empty(k, np.int32)
        un, ot = np.empty(k, np.int64), np.empty(k, np.int64)
        ex, pd = np.empty(k, np.float64), np.empty(k, np.float64)
        call("spm_pattern_classes", self._h, ctypes.byref(n), _ptr(rb), _ptr(cb), _ptr(un), _ptr(ot), _ptr(ex),
             _ptr(pd))
        return [dict(row_blocks=int(rb[i]), col_blocks=int(cb[i]), units=int(un[i]), out_tiles=int(ot[i]),
                     exact_macs=float(ex[i]), padded_macs=float(pd[i])) for i in range(k)]

    def tiles(self):
        tr = np.empty(self.n_tiles, np.int32)
        tc = np.empty(self.n_tiles, np.int32)
        to = np.empty(self.n_tiles, np.int64)
        call("spm_pattern_tiles", self._h, _ptr(tr), _ptr(tc), _ptr(to))
        return tr, tc, to

    def download_csr(self):
        rp = np.empty(self.n + 1, np.int64)
        col = np.empty(self.nnz, np.int32)
        call("spm_pattern_download_csr", self._h, _ptr(rp), _ptr(col))
        return rp, col

    def empty(self, prec="f64", device="cuda") -> torch.Tensor:
        p = prec_code(prec)
        if p == F64:
            return torch.empty(self.n_stored, dtype=torch.float64, device=device)
        return torch.empty(self.n_stored * (2 if p == F32SPLIT else 1), dtype=torch.float32, device=device)

    def values_from_csr(self, csr_vals: torch.Tensor) -> torch.Tensor:
        if not (isinstance(csr_vals, torch.Tensor) and csr_vals.dtype == torch.float64 and csr_vals.is_cuda
                and csr_vals.numel() == self.nnz and csr_vals.is_contiguous()):
            raise ValueError(f"values_from_csr: need a contiguous CUDA float64 tensor of {self.nnz} values")
        out = self.empty("f64", device=csr_vals.device)
        call("spm_values_from_csr", self._h, _ptr(csr_vals), _ptr(out), _stream())
        return out

    def values_to_csr(self, vals: torch.Tensor) -> torch.Tensor:
        _check_vals(self, vals, "f64", "values_to_csr", "vals")
        out = torch.zeros(self.nnz, dtype=torch.float64, device=vals.device)
        call("spm_values_to_csr", self._h, _ptr(vals), _ptr(out), _stream())
        return out

    def __del__(self):
        try:
            if getattr(self, "_h", None) and _lib._lib is not None:
                _lib._lib.spm_pattern_destroy(self._h)
                self._h = None
        except Exception:
            pass


def kernel_compress(pat: Pattern, tree: Tree, matern_p: int, ell: float, scale: float, deriv: bool = False,
                    out: torch.Tensor | None = None) -> torch.Tensor:
    out = pat.empty("f64") if out is None else out
    _check_vals(pat, out, "f64", "kernel_compress", "out")
    call("spm_kernel_compress", pat._h, tree._h, matern_p, ell, scale, int(deriv), _ptr(out), _stream())
    return out


def gemm_workspace_bytes(pat: Pattern, prec="f64", transA=False, transB=False) -> int:
    need = ctypes.c_size_t()
    call("spm_masked_gemm_workspace", pat._h, prec_code(prec), int(transA), int(transB), ctypes.byref(need))
    return need.value


def gemm_workspace(pat: Pattern, prec="f64", transA=False, transB=False, device="cuda") -> torch.Tensor | None:
    """A reusable workspace for masked_gemm with these arguments (None if none is needed)."""
    return _workspace(gemm_workspace_bytes(pat, prec, transA, transB), device)


def masked_gemm(pat: Pattern, A, B, transA=False, transB=False, prec="f64", out=None,
                workspace: torch.Tensor | None = None) -> torch.Tensor:
    """C = P_S(op(A) op(B)); the workspace is the given one (from gemm_workspace) or
    comes from torch's allocator."""
    p = prec_code(prec)
    _check_vals(pat, A, p, "masked_gemm", "A")
    _check_vals(pat, B, p, "masked_gemm", "B")
    out = pat.empty(p, device=A.device) if out is None else out
    _check_vals(pat, out, p, "masked_gemm", "out")
    need = gemm_workspace_bytes(pat, p, transA, transB)
    if workspace is None:
        workspace = _workspace(need, A.device)
    elif workspace.numel() * workspace.element_size() < need or not workspace.is_cuda:
        raise ValueError(f"masked_gemm: workspace needs {need} bytes on the device")
    call("spm_masked_gemm_ws", pat._h, p, _ptr(A), int(transA), _ptr(B), int(transB), _ptr(out), _ptr(workspace),
         need, _stream())
    return out


def masked_gemm_backward(pat: Pattern, dC, A, B, need_a=True, need_b=True, prec="f64"):
    p = prec_code(prec)
    for t, nm in ((dC, "dC"), (A, "A"), (B, "B")):
        _check_vals(pat, t, p, "masked_gemm_backward", nm)
    dA = pat.empty(p, device=dC.device) if need_a else None
    dB = pat.empty(p, device=dC.device) if need_b else None
    need = ctypes.c_size_t()
    call("spm_masked_gemm_backward_workspace", pat._h, p, ctypes.byref(need))
    ws = _workspace(need.value, dC.device)
    call("spm_masked_gemm_backward_ws", pat._h, p, _ptr(dC), _ptr(A), _ptr(B), _ptr(dA), _ptr(dB), _ptr(ws),
         need.value, _stream())
    return dA, dB


def axpy(pat: Pattern, alpha: float, X, beta: float, Y: torch.Tensor, prec="f64") -> torch.Tensor:
    """Y <- alpha X + beta Y in place (X = None: the identity)."""
    if X is not None:
        _check_vals(pat, X, prec, "axpy", "X")
    _check_vals(pat, Y, prec, "axpy", "Y")
    call("spm_axpy", pat._h, prec_code(prec), alpha, _ptr(X), beta, _ptr(Y), _stream())
    return Y


def convert(pat: Pattern, X, prec_from, prec_to) -> torch.Tensor:
    _check_vals(pat, X, prec_from, "convert", "X")
    out = pat.empty(prec_to, device=X.device)
    call("spm_convert", pat._h, prec_code(prec_from), _ptr(X), prec_code(prec_to), _ptr(out), _stream())
    return out


def _scalar(dev) -> torch.Tensor:
    return torch.empty(1, dtype=torch.float64, device=dev)


def sqdist(pat: Pattern, X, Y=None, prec="f64") -> torch.Tensor:
    _check_vals(pat, X, prec, "sqdist", "X")
    if Y is not None:
        _check_vals(pat, Y, prec, "sqdist", "Y")
    out = _scalar(X.device)
    call("spm_sqdist", pat._h, prec_code(prec), _ptr(X), _ptr(Y), _ptr(out), _stream())
    return out


def sqdist_eye(pat: Pattern, X, alpha=1.0, prec="f64") -> torch.Tensor:
    _check_vals(pat, X, prec, "sqdist_eye", "X")
    out = _scalar(X.device)
    call("spm_sqdist_eye", pat._h, prec_code(prec), alpha, _ptr(X), _ptr(out), _stream())
    return out


def dot(pat: Pattern, X, Y) -> torch.Tensor:
    _check_vals(pat, X, "f64", "dot", "X")
    _check_vals(pat, Y, "f64", "dot", "Y")
    out = _scalar(X.device)
    call("spm_dot", pat._h, _ptr(X), _ptr(Y), _ptr(out), _stream())
    return out


def quadform(pat: Pattern, X, y) -> torch.Tensor:
    _check_vals(pat, X, "f64", "quadform", "X")
    if not (isinstance(y, torch.Tensor) and y.dtype == torch.float64 and y.numel() == pat.n and y.is_cuda
            and y.is_contiguous()):
        raise ValueError(f"quadform: y must be a contiguous CUDA float64 tensor of {pat.n} values")
    out = _scalar(X.device)
    call("spm_quadform", pat._h, _ptr(X), _ptr(y), _ptr(out), _stream())
    return out


def fill_outer(pat: Pattern, y, alpha=1.0, out=None) -> torch.Tensor:
    if not (isinstance(y, torch.Tensor) and y.dtype == torch.float64 and y.numel() == pat.n and y.is_cuda
            and y.is_contiguous()):
        raise ValueError(f"fill_outer: y must be a contiguous CUDA float64 tensor of {pat.n} values")
    out = pat.empty("f64", device=y.device) if out is None else out
    _check_vals(pat, out, "f64", "fill_outer", "out")
    call("spm_fill_outer", pat._h, alpha, _ptr(y), _ptr(out), _stream())
    return out


def contour_rule(lam_min: float, lam_max: float, nodes: int):
    """Shifts w_k^2 and weights c_k of the contour quadrature for A^{-1/2} (host arrays)."""
    w2 = np.empty(nodes, np.float64)
    c = np.empty(nodes, np.float64)
    call("spm_contour_rule", float(lam_min), float(lam_max), int(nodes), _ptr(w2), _ptr(c))
    return w2, c


def contour_invsqrt(pat: Pattern, A: torch.Tensor, lam_min: float, lam_max: float, nodes: int, ns_iters: int):
    """A^{-1/2} on S by the contour quadrature with masked Newton-Schulz inverses;
    returns (A^{-1/2}, final residual of each shifted inverse)."""
    _check_vals(pat, A, "f64", "contour_invsqrt", "A")
    need = ctypes.c_size_t()
    call("spm_contour_invsqrt_scratch", pat._h, int(ns_iters), ctypes.byref(need))
    scratch = torch.empty((need.value + 7) // 8, dtype=torch.float64, device=A.device)
    out = pat.empty("f64")
    res = torch.zeros(max(nodes, 1), dtype=torch.float64, device=A.device)
    call("spm_contour_invsqrt", pat._h, _ptr(A), float(lam_min), float(lam_max), int(nodes), int(ns_iters),
         _ptr(out), _ptr(res), _ptr(scratch), scratch.numel() * 8, _stream())
    return out, res[:nodes]


def fst(tree: Tree, X: torch.Tensor, inverse: bool = False) -> torch.Tensor:
    """Fast samplet transform of the rows of X (shape (r, n)): T x (original point order ->
    basis order), or T^T x with inverse=True."""
    assert X.dtype == torch.float64 and X.dim() == 2 and X.shape[1] == tree.n
    X = X.contiguous()
    Y = torch.empty_like(X)
    call("spm_fst", tree._h, _ptr(X), int(X.shape[0]), _ptr(Y), int(bool(inverse)), _stream())
    return Y


def spmm(pat: Pattern, A: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    """A X for a block X of shape (r, n) (row j = column j of the n x r block, basis order)."""
    assert X.dtype == torch.float64 and X.dim() == 2 and X.shape[1] == pat.n and X.is_cuda
    _check_vals(pat, A, "f64", "spmm", "A")
    X = X.contiguous()
    Y = torch.empty_like(X)
    call("spm_spmm", pat._h, _ptr(A), _ptr(X), int(X.shape[0]), _ptr(Y), _stream())
    return Y


def ns_sqrt(pat: Pattern, A: torch.Tensor, iters: int):
    """Coupled masked Newton-Schulz iteration; returns (Y ~ A^{1/2}, Z ~ A^{-1/2}, residuals)."""
    _check_vals(pat, A, "f64", "ns_sqrt", "A")
    need = ctypes.c_size_t()
    call("spm_ns_sqrt_scratch", pat._h, ctypes.byref(need))
    scratch = torch.empty((need.value + 7) // 8, dtype=torch.float64, device=A.device)
    Y, Z = pat.empty("f64"), pat.empty("f64")
    res = torch.zeros(max(iters, 1), dtype=torch.float64, device=A.device)
    call("spm_ns_sqrt", pat._h, _ptr(A), _ptr(Y), _ptr(Z), int(iters), _ptr(res), _ptr(scratch),
         scratch.numel() * 8, _stream())
    return Y, Z, res[:iters]


def expm_taylor(pat: Pattern, A: torch.Tensor, terms: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """sum_{j <= terms} A^j / j! on S by Horner's rule with formatted products (FP64)."""
    _check_vals(pat, A, "f64", "expm_taylor", "A")
    if out is not None:
        _check_vals(pat, out, "f64", "expm_taylor", "out")
    need = ctypes.c_size_t()
    call("spm_expm_taylor_scratch", pat._h, ctypes.byref(need))
    scratch = torch.empty((need.value + 7) // 8, dtype=torch.float64, device=A.device)
    E = pat.empty("f64") if out is None else out
    call("spm_expm_taylor", pat._h, _ptr(A), _ptr(E), int(terms), _ptr(scratch), scratch.numel() * 8, _stream())
    return E


def newton_schulz(pat: Pattern, A: torch.Tensor, iters: int, n_final_f64: int = 3, bulk="f64",
                  alpha0: float = 1.0, checkpoints: bool = False):
    """Masked Newton-Schulz; returns (X, residuals[iters+1], list of X_0..X_iters or None)."""
    _check_vals(pat, A, "f64", "newton_schulz", "A")
    b = prec_code(bulk)
    need = ctypes.c_size_t()
    call("spm_newton_schulz_scratch", pat._h, b, ctypes.byref(need))
    scratch = torch.empty((need.value + 7) // 8, dtype=torch.float64, device=A.device)
    X = pat.empty("f64")
    res = torch.empty(iters + 1, dtype=torch.float64, device=A.device)
    ck = None
    ck_arr = None
    if checkpoints:
        ck = [pat.empty("f64") for _ in range(iters + 1)]
        ck_arr = (ctypes.c_void_p * (iters + 1))(*[c.data_ptr() for c in ck])
    call("spm_newton_schulz", pat._h, _ptr(A), _ptr(X), iters, n_final_f64, b, alpha0, _ptr(res),
         ck_arr if ck_arr is not None else None, _ptr(scratch), scratch.numel() * 8, _stream())
    return X, res, ck
