"""Naive EM/MAP update of rank-constrained SCM estimation, FP64.

Follows Sec. II-B-2 literally: the E-step builds the per-bin model covariance
R~^(x)_ij and inverts it (eqs. (13)-(16)); the M-step updates r^h, then
lambda (with r~^u), then R^(u) and r^u with the new lambda (eqs. (17)-(20)).
One M x M ``numpy.linalg.inv`` per time-frequency bin.

Array layout: x [I, J, M] complex; a, b [I, M]; Rp [I, M, M];
state rh, ru [I, J], lam [I] (float64).
"""
import numpy as np

from .linalg import herm


def estep(x, a, Rp, b, rh_t, ru_t, lam_t):
    """E-step for one frequency row (vectorised over frames).

    x [J, M], a, b [M], Rp [M, M], rh_t, ru_t [J], lam_t scalar.
    Returns (R~, h_hat [J], U_hat [J, M, M]).
    """
    R_t = Rp + lam_t * np.outer(b, np.conj(b))                           # eq. (13)
    Rx = (rh_t[:, None, None] * np.outer(a, np.conj(a))[None]
          + ru_t[:, None, None] * R_t[None])                            # eq. (14)
    Rx_inv = np.linalg.inv(Rx)
    aH_Rxinv_a = np.einsum("m,jmn,n->j", np.conj(a), Rx_inv, a)
    xH_Rxinv_a = np.einsum("jm,jmn,n->j", np.conj(x), Rx_inv, a)
    h_hat = rh_t - rh_t ** 2 * aH_Rxinv_a.real + np.abs(rh_t * xH_Rxinv_a) ** 2  # eq. (15)
    R_Rxinv = np.einsum("mk,jkn->jmn", R_t, Rx_inv)
    R_Rxinv_R = np.einsum("jmk,kn->jmn", R_Rxinv, R_t)
    v = np.einsum("jmn,jn->jm", R_Rxinv, x)        # R~ (R~^(x))^{-1} x
    U_hat = (ru_t[:, None, None] * R_t[None]
             - ru_t[:, None, None] ** 2 * R_Rxinv_R
             + ru_t[:, None, None] ** 2 * v[:, :, None] * np.conj(v)[:, None, :])  # eq. (16)
    return R_t, h_hat, U_hat


def mstep(Rp, b, ru_t, h_hat, U_hat, alpha, beta):
    """M-step for one frequency row; returns (rh [J], lam scalar, ru [J])."""
    M = Rp.shape[-1]
    rh = (h_hat + beta) / (alpha + 2.0)                                    # eq. (17)
    bUb = np.einsum("m,jmn,n->j", np.conj(b), U_hat, b).real
    lam = np.mean(bUb / ru_t)                                              # eq. (18)
    R = Rp + lam * np.outer(b, np.conj(b))                                 # eq. (19)
    R_inv = np.linalg.inv(R)
    ru = np.einsum("mn,jnm->j", R_inv, U_hat).real / M                     # eq. (20)
    return rh, lam, ru


def step(x, a, Rp, b, rh, ru, lam, alpha, beta):
    """One naive iteration over all frequencies; returns new (rh, ru, lam)."""
    I = x.shape[0]
    rh_n = np.empty_like(rh)
    ru_n = np.empty_like(ru)
    lam_n = np.empty_like(lam)
    for i in range(I):
        _, h_hat, U_hat = estep(x[i].astype(np.complex128), a[i], Rp[i], b[i],
                                rh[i], ru[i], lam[i])
        rh_n[i], lam_n[i], ru_n[i] = mstep(Rp[i], b[i], ru[i], h_hat, U_hat, alpha, beta)
    return rh_n, ru_n, lam_n


def run(x, a, Rp, b, rh0, ru0, lam0, K, alpha, beta, history=False):
    """K naive iterations from (rh0, ru0, lam0).  Returns (rh, ru, lam) or a list of states."""
    rh = np.array(rh0, dtype=np.float64)
    ru = np.array(ru0, dtype=np.float64)
    lam = np.array(lam0, dtype=np.float64)
    hist = [(rh, ru, lam)]
    for _ in range(K):
        rh, ru, lam = step(x, a, Rp, b, rh, ru, lam, alpha, beta)
        hist.append((rh, ru, lam))
    return hist if history else (rh, ru, lam)
