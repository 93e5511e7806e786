"""torch.autograd.Function wrappers of the library's network and training loss.

The forward and backward (adjoint) passes are the library's HIP kernels
(`mdnp_cnn_forward`, `mdnp_cnn_backward`, `mdnp_loss_grad`); autograd only
chains them, so the gradient of the Section 5.1 risk with respect to the
weights comes out of `loss.backward()` while every arithmetic step runs on
the GPU in the library.

    y = unet(w, X, ctx, n, "bf16")          # [B, n^3]
    loss = residual_loss(y, r, inst, S)      # [B] FP64, || r - alpha^-1 C mask(y) ||^2
    loss.sum().backward()                    # w.grad from the library's adjoint kernels
"""
from __future__ import annotations

import torch

from .api import Context, System


class UNetFunction(torch.autograd.Function):
    """y = U(X; w) on a batch: X [B, n^3, 2] FP32 (residual channel, distance
    channel), w the flat FP32 weights; y [B, n^3] FP32.  The activations the
    adjoint needs are stored by the forward kernel in a byte buffer kept for
    backward."""

    @staticmethod
    def forward(fctx, w: torch.Tensor, X: torch.Tensor, ctx: Context, n: int, dtype: str):
        w = w.contiguous()
        X = X.contiguous()
        batch = X.shape[0]
        saved = torch.empty(ctx.saved_bytes(batch, n, dtype), dtype=torch.uint8, device=X.device)
        y = ctx.cnn_forward(w, X, n, dtype, saved=saved)
        fctx.save_for_backward(w, saved)
        fctx.lib, fctx.n, fctx.dtype, fctx.batch = ctx, n, dtype, batch
        return y

    @staticmethod
    def backward(fctx, gy: torch.Tensor):
        w, saved = fctx.saved_tensors
        want_dx = bool(fctx.needs_input_grad[1])
        dw, dx = fctx.lib.cnn_backward(w, saved, gy.contiguous().float(), fctx.batch, fctx.n, fctx.dtype,
                                       want_dx=want_dx)
        return (dw if fctx.needs_input_grad[0] else None), dx, None, None, None


class ResidualLossFunction(torch.autograd.Function):
    """loss[k] = || r_k - alpha_k^-1 C_k mask(u_k) ||^2 (C = A00 of instance
    inst[k]); its gradient with respect to u comes from the same library call
    and is scaled by the incoming per-slot gradient in backward."""

    @staticmethod
    def forward(fctx, u: torch.Tensor, r: torch.Tensor, inst: torch.Tensor, S: System):
        loss, du = S.loss_grad(inst.contiguous(), r.contiguous(), u.contiguous())
        fctx.save_for_backward(du)
        return loss

    @staticmethod
    def backward(fctx, gl: torch.Tensor):
        (du,) = fctx.saved_tensors
        # d(sum_k g_k loss_k)/du_k = g_k du_k: the chain rule's per-slot factor
        # (1 for loss.sum(), so du is handed on unchanged)
        if bool(torch.all(gl == 1)):
            return du, None, None, None
        return du * gl.to(du.dtype)[:, None], None, None, None


def unet(w: torch.Tensor, X: torch.Tensor, ctx: Context, n: int, dtype: str = "bf16") -> torch.Tensor:
    return UNetFunction.apply(w, X, ctx, n, dtype)


def residual_loss(u: torch.Tensor, r: torch.Tensor, inst: torch.Tensor, S: System) -> torch.Tensor:
    return ResidualLossFunction.apply(u, r, inst, S)
