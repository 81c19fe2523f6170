"""Rank-(M-1) SCM of the diffuse noise from a demixing matrix, and the paper's
initialisation of r^u and lambda (Sec. II-B-1 eq. (11); Sec. II-B-3 eqs. (22), (23)), FP64.

Given W_i = (w_1 ... w_M)^H (so y_ij = W_i x_ij are the separated signals) and
the index n_h of the target:
  R'_i   = (1/J) sum_j W^{-1} diag(|w_1^H x|^2, .., 0 (at n_h), .., |w_M^H x|^2) W^{-H}   eq. (11)
  b_i    = unit eigenvector of R'_i for the zero eigenvalue
  a_i    = the n_h-th steering vector, column n_h of W^{-1}
  y^(u)  = W^{-1} (w_1^H x, .., 0 (at n_h), .., w_M^H x)^T                              eq. (23)
  r^u_0  = (1/M) y^(u)H (R')^+ y^(u)                                                  eq. (22)
  lambda_0 = minimum nonzero eigenvalue of R'_i                      (text after eq. (23))
Each step is written literally (per-bin diagonal matrices, numpy inverse,
eigendecomposition, pseudoinverse of known rank).
"""
import numpy as np

from .linalg import herm, pinv_rank


def rprime(x, W, n_h):
    """R' [I, M, M] by eq. (11)."""
    I, J, M = x.shape
    x = x.astype(np.complex128)
    Winv = np.linalg.inv(W)
    out = np.empty((I, M, M), np.complex128)
    for i in range(I):
        y = np.einsum("mn,jn->jm", W[i], x[i])               # w_m^H x for every frame
        d = np.abs(y) ** 2
        d[:, n_h] = 0.0
        D = np.zeros((J, M, M))
        D[:, np.arange(M), np.arange(M)] = d                 # per-frame diagonal matrices
        S = Winv[i][None] @ D @ herm(Winv[i])[None]
        out[i] = S.mean(axis=0)
    return out


def null_vector(Rp):
    """Unit eigenvector of each R' for its smallest (zero) eigenvalue [I, M]."""
    w, V = np.linalg.eigh(Rp)
    return V[..., :, 0]


def steering(W, n_h):
    """a_i = column n_h of W_i^{-1} [I, M]."""
    return np.linalg.inv(W)[..., :, n_h]


def noise_image(x, W, n_h):
    """y^(u) [I, J, M] by eq. (23)."""
    x = x.astype(np.complex128)
    Winv = np.linalg.inv(W)
    y = np.einsum("imn,ijn->ijm", W, x)
    y[..., n_h] = 0.0
    return np.einsum("imn,ijn->ijm", Winv, y)


def ru_init(x, W, n_h, Rp=None):
    """r^u_0 [I, J] by eq. (22)."""
    M = x.shape[-1]
    if Rp is None:
        Rp = rprime(x, W, n_h)
    yu = noise_image(x, W, n_h)
    P = pinv_rank(Rp, M - 1)
    return np.einsum("ijm,imn,ijn->ij", np.conj(yu), P, yu).real / M


def lam_init(Rp):
    """Minimum nonzero eigenvalue of each R' [I] (R' has rank M-1)."""
    return np.linalg.eigvalsh(Rp)[..., 1]
