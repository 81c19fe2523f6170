"""Reference gradients of the differentiable path, FP64 on the CPU.

Forward (the path whose adjoint the GPU computes):
  precompute sigma/tau from x (eqs. (32), (33), (46)-(48)),
  K second-stage iterations (Algorithm 2, eqs. (49)-(56)) from
  (r^h_0, r^u_0, lambda_0),
  s_hat = r^h a^H Sigma^{-1} x at the final parameters (posterior mean,
  inside eq. (15)),
  loss  = sum_ij |s_hat_ij - s_ij|^2.

Two independent routes:
  * ``torch_grads``: plain torch CPU float64 autograd of that forward.
  * ``fd_directional``: central finite differences of the numpy forward
    (``oracle.accel`` + ``oracle.extract``) along a given direction.

Complex-gradient convention (torch's): for real L and complex x the gradient
is dL/dRe(x) + i dL/dIm(x), so the directional derivative along v is
Re(sum conj(g) v).
"""
import numpy as np
import torch

from . import accel, extract
from .linalg import pinv_rank


def _forward_torch(x, a, Rpp, b, rh0, ru0, lam0, K, alpha, beta, s_true, Rp):
    M = x.shape[-1]
    s_ab = torch.einsum("im,im->i", a.conj(), b)[:, None]
    s_bx = torch.einsum("im,ijm->ij", b.conj(), x)
    t_aa = torch.einsum("im,imn,in->i", a.conj(), Rpp, a).real[:, None]
    t_ax = torch.einsum("im,imn,ijn->ij", a.conj(), Rpp, x)
    t_xx = torch.einsum("ijm,imn,ijn->ij", x.conj(), Rpp, x).real
    rh, ru, lam = rh0, ru0, lam0
    for _ in range(K):
        lt = lam[:, None]
        rho_aa_t = t_aa + s_ab.abs() ** 2 / lt
        rho_ax_t = t_ax + s_ab * s_bx / lt
        g = rh / (ru + rh * rho_aa_t)
        rh_new = (g * (ru + g * rho_ax_t.abs() ** 2) + beta) / (alpha + 2.0)
        lam_new = torch.mean(g * s_ab.abs() ** 2
                             + (s_bx - g * s_ab.conj() * rho_ax_t).abs() ** 2 / ru, dim=1)
        ln = lam_new[:, None]
        rho_aa = t_aa + s_ab.abs() ** 2 / ln
        rho_ax = t_ax + s_ab * s_bx / ln
        rho_xx = t_xx + s_bx.abs() ** 2 / ln
        ru_new = (g * rho_aa * (ru + g * rho_ax_t.abs() ** 2) + rho_xx
                  - 2.0 * g * torch.real(rho_ax_t * rho_ax.conj())) / M
        rh, ru, lam = rh_new, ru_new, lam_new
    # posterior mean by a direct solve with Sigma (not through the rho terms)
    R = Rp + lam[:, None, None] * torch.einsum("im,in->imn", b, b.conj())
    aa = torch.einsum("im,in->imn", a, a.conj())
    S = rh[..., None, None] * aa[:, None] + ru[..., None, None] * R[:, None]
    y = torch.linalg.solve(S, x[..., None])[..., 0]
    s_hat = rh * torch.einsum("im,ijm->ij", a.conj(), y)
    loss = torch.sum((s_hat - s_true).abs() ** 2)
    return loss, s_hat


def torch_grads(x, a, Rp, b, rh0, ru0, lam0, K, alpha, beta, s_true):
    """Returns (loss, s_hat, grad_x [I,J,M] complex, grad_rh0 [I,J], grad_lam0 [I])."""
    M = x.shape[-1]
    Rpp = torch.from_numpy(pinv_rank(Rp, M - 1))
    xt = torch.from_numpy(x.astype(np.complex128)).requires_grad_(True)
    rh0t = torch.from_numpy(np.array(rh0, np.float64)).requires_grad_(True)
    lam0t = torch.from_numpy(np.array(lam0, np.float64)).requires_grad_(True)
    loss, s_hat = _forward_torch(xt, torch.from_numpy(a), Rpp, torch.from_numpy(b), rh0t,
                                 torch.from_numpy(np.array(ru0, np.float64)), lam0t, K,
                                 alpha, beta, torch.from_numpy(s_true.astype(np.complex128)),
                                 torch.from_numpy(Rp))
    loss.backward()
    return (float(loss), s_hat.detach().numpy(), xt.grad.numpy(), rh0t.grad.numpy(),
            lam0t.grad.numpy())


def loss_numpy(x, a, Rp, b, rh0, ru0, lam0, K, alpha, beta, s_true):
    rh, ru, lam = accel.run(x, a, Rp, b, rh0, ru0, lam0, K, alpha, beta)
    sh = extract.s_hat(x, a, Rp, b, rh, ru, lam)
    return float(np.sum(np.abs(sh - s_true) ** 2))


def fd_directional(x, a, Rp, b, rh0, ru0, lam0, K, alpha, beta, s_true,
                   vx=None, vrh=None, vlam=None, h=1e-3):
    """Central difference of the loss along (vx, vrh, vlam) with step h."""
    x = x.astype(np.complex128)
    vx = np.zeros_like(x) if vx is None else vx
    vrh = np.zeros_like(rh0) if vrh is None else vrh
    vlam = np.zeros_like(lam0) if vlam is None else vlam

    def L(e):
        return loss_numpy(x + e * vx, a, Rp, b, rh0 + e * vrh, ru0, lam0 + e * vlam,
                          K, alpha, beta, s_true)
    return (L(h) - L(-h)) / (2.0 * h)
