"""torch.autograd.Function around the differentiable path of librcscm.

    s_hat = estimate_and_extract(x, rh0, lam0, a, Rp, b, K=10)

runs the per-bin precomputation, K second-stage accelerated iterations
(Algorithm 2) from (r^h_0, r^u_0, lambda_0) and the Wiener-filter extraction
on the GPU, keeping theta_k of every iteration; backward() runs the
hand-written adjoint kernel (rcscm_backward) and returns gradients for x
(complex64, torch's convention dL/dRe + i dL/dIm), r^h_0 and lambda_0.
a, R' and b are fixed model inputs (no gradient).
"""
from __future__ import annotations

import torch

from .rcscm import Context


class _EstimateExtract(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, rh0, lam0, a, Rp, b, shape, K, ru0, params):
        I, Js, Ms = shape
        c = Context(I, Js, Ms, checkpoint=True, **params)
        # setup, precompute, K iterations (keeping theta_k) and extraction: one call
        out = c.run(x.detach().contiguous(), a.contiguous(), Rp.contiguous(), b.contiguous(), K,
                    rh0=rh0.detach().contiguous(), ru0=ru0, lam0=lam0.detach().contiguous())
        ctx.rcscm = c
        ctx.save_for_backward(x)
        ctx.mark_non_differentiable(out["rh"], out["ru"], out["lam"])
        return out["s_hat"], out["rh"], out["ru"], out["lam"]

    @staticmethod
    def backward(ctx, g_s, g_rh, g_ru, g_lam):
        (x,) = ctx.saved_tensors
        c = ctx.rcscm
        if g_s is None:
            g_s = torch.zeros(c.nbins, dtype=torch.complex64, device=x.device)
        gx, grh, glam = c.backward(x.detach().contiguous(), g_s.contiguous(),
                                   want_x=ctx.needs_input_grad[0],
                                   want_rh0=ctx.needs_input_grad[1],
                                   want_lam0=ctx.needs_input_grad[2])
        c.close()
        ctx.rcscm = None
        return gx, grh, glam, None, None, None, None, None, None, None


def estimate_and_extract(x, rh0, lam0, a, Rp, b, K, I=None, Js=None, Ms=None, ru0=None,
                         **params):
    """Differentiable s_hat (complex64, batch layout) plus the final (r^h, r^u, lambda).

    For a single utterance pass x as [I, J, M] (or flat with I, Js=[J], Ms=[M]).
    """
    if I is None:
        I, J, M = x.shape
        Js, Ms = [J], [M]
    shape = (int(I), [int(j) for j in Js], [int(m) for m in Ms])
    xf = x.reshape(-1)
    rh0f = rh0.reshape(-1).to(torch.float32)
    lam0f = lam0.reshape(-1).to(torch.float32)
    ru0f = None if ru0 is None else ru0.reshape(-1).to(torch.float32).contiguous()
    s_hat, rh, ru, lam = _EstimateExtract.apply(xf, rh0f, lam0f, a.reshape(-1), Rp.reshape(-1),
                                                b.reshape(-1), shape, int(K), ru0f, params)
    return s_hat, rh, ru, lam
