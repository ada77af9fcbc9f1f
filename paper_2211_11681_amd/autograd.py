"""torch.autograd wiring of the S-format operations.

Every forward and backward step calls libspm (the hand-written adjoints of the
masked product, the Newton-Schulz reverse sweep and the compressed kernel
derivative); torch only records the graph and owns the buffers.  Values are
FP64 tensors in the library's tile layout (length ``n_stored``).

Adjoints used (one symmetric pattern S, so every adjoint lives on S):
  C = P_S(U V):            U-bar = P_S(C-bar V^T),  V-bar = P_S(U^T C-bar)
  Newton-Schulz step k:    Y_k = P_S(A X_k),  Z_k = 2I - Y_k,  X_{k+1} = P_S(X_k Z_k)
  f = y^T X y:             X-bar = f-bar P_S(y y^T)
  K^eta(l):                l-bar = <K-bar, dK^eta/dl>_S
The Newton-Schulz forward keeps X_0 .. X_{K-1} (one FP64 checkpoint per
iteration; the sweep never reads X_K) and the reverse sweep recomputes Y_k and
Z_k from them.
"""
from __future__ import annotations

import torch

from . import spm


class MaskedGemm(torch.autograd.Function):
    """C = P_S(A B) (the product of Section 4.1) with its adjoint."""

    @staticmethod
    def forward(ctx, pat, A, B):
        ctx.pat = pat
        ctx.save_for_backward(A, B)
        return spm.masked_gemm(pat, A, B)

    @staticmethod
    def backward(ctx, dC):
        A, B = ctx.saved_tensors
        dA, dB = spm.masked_gemm_backward(ctx.pat, dC.contiguous(), A, B, need_a=ctx.needs_input_grad[1],
                                          need_b=ctx.needs_input_grad[2])
        return None, dA, dB


class AddIdentity(torch.autograd.Function):
    """A = K + mu I on the pattern."""

    @staticmethod
    def forward(ctx, pat, K, mu):
        A = K.clone()
        spm.axpy(pat, float(mu), None, 1.0, A)
        return A

    @staticmethod
    def backward(ctx, gA):
        return None, gA, None


class NewtonSchulz(torch.autograd.Function):
    """X_K of the masked Newton-Schulz iteration for A^{-1} (FP64 throughout).

    Returns (X_K, residuals r_0 .. r_K); the residuals are not differentiable.
    """

    @staticmethod
    def forward(ctx, pat, A, iters, alpha0):
        X, res, ck = spm.newton_schulz(pat, A, iters, n_final_f64=iters, bulk="f64", alpha0=alpha0,
                                       checkpoints=True)
        ctx.pat = pat
        ctx.ck = ck[:iters]          # X_K itself is returned as X; the sweep reads X_0 .. X_{K-1}
        del ck
        ctx.save_for_backward(A)
        ctx.mark_non_differentiable(res)
        return X, res

    @staticmethod
    def backward(ctx, Xbar, _res_bar):
        (A,) = ctx.saved_tensors
        pat, ck = ctx.pat, ctx.ck
        Abar = torch.zeros_like(A)
        xbar = Xbar.contiguous()
        for k in range(len(ck) - 1, -1, -1):
            Xk = ck[k]
            Zk = spm.masked_gemm(pat, A, Xk)                      # Y_k
            spm.axpy(pat, 2.0, None, -1.0, Zk)                    # Z_k = 2I - Y_k
            xb, zbar = spm.masked_gemm_backward(pat, xbar, Xk, Zk)  # P(Xbar Z^T), P(X^T Xbar)
            spm.axpy(pat, 0.0, None, -1.0, zbar)                  # Y-bar = -Z-bar
            ab, xb2 = spm.masked_gemm_backward(pat, zbar, A, Xk)  # P(Ybar X^T), P(A^T Ybar)
            spm.axpy(pat, 1.0, ab, 1.0, Abar)
            spm.axpy(pat, 1.0, xb2, 1.0, xb)
            xbar = xb
        ctx.ck = None
        return None, Abar, None, None


class QuadForm(torch.autograd.Function):
    """f = y^T X y for y in basis order."""

    @staticmethod
    def forward(ctx, pat, X, y):
        ctx.pat = pat
        ctx.save_for_backward(y)
        return spm.quadform(pat, X, y).reshape(())

    @staticmethod
    def backward(ctx, gf):
        (y,) = ctx.saved_tensors
        return None, spm.fill_outer(ctx.pat, y, alpha=float(gf)), None


class CompressedKernel(torch.autograd.Function):
    """K^eta(l) = P_S(T K(l) T^T) of a Matern kernel with half-integer smoothness p + 1/2."""

    @staticmethod
    def forward(ctx, ell, pat, tree, matern_p, scale):
        ctx.pat, ctx.tree, ctx.p, ctx.scale = pat, tree, matern_p, scale
        ctx.ell = float(ell)
        return spm.kernel_compress(pat, tree, matern_p, ctx.ell, scale)

    @staticmethod
    def backward(ctx, gK):
        dK = spm.kernel_compress(ctx.pat, ctx.tree, ctx.p, ctx.ell, ctx.scale, deriv=True)
        g = spm.dot(ctx.pat, gK.contiguous(), dK)
        return g.reshape(()).to(torch.float64).cpu(), None, None, None, None


def gp_quadform_and_grad(pat, tree, matern_p: int, ell: float, mu: float, y: torch.Tensor, iters: int,
                         alpha0: float, scale: float):
    """f(l) = y^T X_K(K^eta(l) + mu I) y and df/dl by reverse mode.

    Returns (f, df/dl, residuals of the forward iteration).
    """
    ell_t = torch.tensor(float(ell), dtype=torch.float64, requires_grad=True)
    # K itself is not kept: A = K + mu I is the only consumer, and the backward of
    # the compression recomputes dK^eta/dl
    A = AddIdentity.apply(pat, CompressedKernel.apply(ell_t, pat, tree, matern_p, scale), mu)
    X, res = NewtonSchulz.apply(pat, A, iters, alpha0)
    f = QuadForm.apply(pat, X, y)
    f.backward()
    return float(f.detach()), float(ell_t.grad), res
