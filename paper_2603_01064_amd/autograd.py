"""``torch.autograd.Function`` wrappers over the library's training losses.

``CycleLoss`` (end of the module) wraps the combined loss of Sec. 3.2
eq. loss_1; ``LevelwiseSpectralLoss`` the level-wise spectral losses.

Forward evaluates the per-level losses of Sec. 3.2 eq. loss_2_modified (2D:
Sec. 3.3 eq. loss_3) for a batch of true solutions with the handle's cycle
(pre-smoothing only, from zero); backward returns the hand-written adjoint
that the library computed in the same call (``nmg_loss_grad``), scaled by the
incoming loss gradients.  When no weight needs a gradient (evaluation, or
inside ``torch.no_grad()``) forward calls ``nmg_loss_forward`` instead and
the adjoint is never computed.  Level ``l``'s loss is differentiated with respect to
its own smoother only (Algorithm 5 updates each level from its own loss; the
corrections of earlier levels enter as constants), so for weights
``theta_l`` the backward result is ``sum_l' g_l' dL_l'/dtheta_l =
g_l dL_l/dtheta_l``.

This module only marshals tensors: every step of the loss and its gradient
runs in the HIP library.  The library keeps FP32 master weights, so weights
passed here are rounded to FP32 before use.
"""
from __future__ import annotations

import torch

from . import nmg


class LevelwiseSpectralLoss(torch.autograd.Function):
    """``losses = LevelwiseSpectralLoss.apply(handle, e, alpha, mask, use_fprime,
    precision, weight_set, *level_weights)``.

    ``level_weights[l]`` is the flat weight vector of level ``l`` (layout of
    :meth:`nmg.Handle.load_smoother_weights`), on any device; ``e`` and
    ``alpha`` are device tensors as for :meth:`nmg.Handle.loss_grad`.  Returns
    a float64 CPU tensor of the ``L - 1`` level losses.
    """

    @staticmethod
    def forward(ctx, handle: nmg.Handle, e, alpha, mask: str, use_fprime: bool, precision: str, weight_set: int,
                *level_weights):
        if len(level_weights) != handle.problem.levels - 1:
            raise ValueError(f"expected {handle.problem.levels - 1} level weight tensors, got {len(level_weights)}")
        for l, w in enumerate(level_weights):
            handle.load_smoother_weights(l, weight_set, [w.detach().to("cpu", torch.float32).numpy()])
        if not any(ctx.needs_input_grad[7:]):
            return torch.from_numpy(handle.loss_forward(e, alpha, weight_set=weight_set, mask=mask,
                                                        use_fprime=use_fprime, precision=precision))
        losses = handle.loss_grad(e, alpha, weight_set=weight_set, mask=mask, use_fprime=use_fprime,
                                  precision=precision)
        grads = [torch.from_numpy(handle.get_gradient(l, weight_set)).to(w.device, w.dtype)
                 for l, w in enumerate(level_weights)]
        ctx.save_for_backward(*grads)
        return torch.from_numpy(losses)

    @staticmethod
    def backward(ctx, grad_losses):
        grads = ctx.saved_tensors
        out = tuple(grad_losses[l].to(g.device, g.dtype) * g for l, g in enumerate(grads))
        return (None, None, None, None, None, None, None) + out


def levelwise_loss(handle: nmg.Handle, level_weights, e, alpha, mask: str = "ramp", use_fprime: bool = False,
                   precision: str = "fp32", weight_set: int = 0):
    """Functional form of :class:`LevelwiseSpectralLoss`."""
    return LevelwiseSpectralLoss.apply(handle, e, alpha, mask, use_fprime, precision, weight_set, *level_weights)


class CycleLoss(torch.autograd.Function):
    """``loss = CycleLoss.apply(handle, e, alpha, use_fprime, precision,
    weight_set, *level_weights)``: the combined loss of Sec. 3.2 eq. loss_1,
    ``(1/B) sum_i ||e_i - NMG(0, A e_i)||^2`` over one whole cycle, as a
    float64 CPU scalar.  Backward returns the library's joint adjoint: every
    level's weights receive ``dL/dtheta_l``, including the effect of their
    correction on the residuals that coarser levels see."""

    @staticmethod
    def forward(ctx, handle: nmg.Handle, e, alpha, use_fprime: bool, precision: str, weight_set: int,
                *level_weights):
        if len(level_weights) != handle.problem.levels - 1:
            raise ValueError(f"expected {handle.problem.levels - 1} level weight tensors, got {len(level_weights)}")
        for l, w in enumerate(level_weights):
            handle.load_smoother_weights(l, weight_set, [w.detach().to("cpu", torch.float32).numpy()])
        if not any(ctx.needs_input_grad[6:]):
            losses = handle.loss_forward(e, alpha, weight_set=weight_set, mask="cycle", use_fprime=use_fprime,
                                         precision=precision)
            return torch.tensor(float(losses[0]), dtype=torch.float64)
        losses = handle.loss_grad(e, alpha, weight_set=weight_set, mask="cycle", use_fprime=use_fprime,
                                  precision=precision)
        grads = [torch.from_numpy(handle.get_gradient(l, weight_set)).to(w.device, w.dtype)
                 for l, w in enumerate(level_weights)]
        ctx.save_for_backward(*grads)
        return torch.tensor(float(losses[0]), dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_loss):
        out = tuple(grad_loss.to(g.device, g.dtype) * g for g in ctx.saved_tensors)
        return (None, None, None, None, None, None) + out


def cycle_loss(handle: nmg.Handle, level_weights, e, alpha, use_fprime: bool = False, precision: str = "fp32",
               weight_set: int = 0):
    """Functional form of :class:`CycleLoss`."""
    return CycleLoss.apply(handle, e, alpha, use_fprime, precision, weight_set, *level_weights)
