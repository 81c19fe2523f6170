"""Multichannel Wiener filter output (Sec. II-A; the final extraction step).

The paper names the filter but does not print it.  Under the model of
eqs. (2)-(10) the MMSE estimate of the dry target is the posterior mean

  s_hat_ij = E[s_ij | x_ij] = r^h_ij a_i^H Sigma_ij^{-1} x_ij,

the same quantity that appears inside eq. (15).  Computed here by a direct
linear solve with Sigma_ij (its definition), FP64.
"""
import numpy as np

from .objective import sigma


def s_hat(x, a, Rp, b, rh, ru, lam):
    S = sigma(a, Rp, b, rh, ru, lam)
    x = x.astype(np.complex128)
    y = np.linalg.solve(S, x[..., None])[..., 0]
    return rh * np.einsum("im,ijm->ij", np.conj(a), y)


def spatial_image(x, a, Rp, b, rh, ru, lam):
    """Target image h_hat_ij = a_i s_hat_ij [I, J, M]."""
    return s_hat(x, a, Rp, b, rh, ru, lam)[..., None] * a[:, None, :]
