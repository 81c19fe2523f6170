"""First-stage accelerated update (Algorithm 1), FP64.

The per-bin inverse of R~^(x)_ij is expanded by Sherman-Morrison
(eqs. (24)-(25)); what remains per iteration is one M x M inverse of R~_i and
one of R_i per frequency, plus quadratic forms per bin (eqs. (27)-(34)).
Update rules: r^h by eq. (39), lambda by eq. (43), r^u by eq. (45).
"""
import numpy as np


def step(x, a, Rp, b, rh, ru, lam, alpha, beta):
    I, J, M = x.shape
    x = x.astype(np.complex128)
    bb = np.einsum("im,in->imn", b, np.conj(b))
    s_ab = np.einsum("im,im->i", np.conj(a), b)[:, None]                 # eq. (32)
    s_bx = np.einsum("im,ijm->ij", np.conj(b), x)                        # eq. (33)
    R_t_inv = np.linalg.inv(Rp + lam[:, None, None] * bb)
    rho_aa_t = np.einsum("im,imn,in->i", np.conj(a), R_t_inv, a).real[:, None]   # eq. (28)
    rho_ax_t = np.einsum("im,imn,ijn->ij", np.conj(a), R_t_inv, x)                # eq. (30)
    gamma_t = rh / (ru + rh * rho_aa_t)                                            # eq. (34)
    rh_new = (gamma_t * (ru + gamma_t * np.abs(rho_ax_t) ** 2) + beta) / (alpha + 2.0)  # eq. (39)
    lam_new = np.mean(gamma_t * np.abs(s_ab) ** 2
                      + np.abs(s_bx - gamma_t * np.conj(s_ab) * rho_ax_t) ** 2 / ru, axis=1)  # eq. (43)
    R_inv = np.linalg.inv(Rp + lam_new[:, None, None] * bb)
    rho_aa = np.einsum("im,imn,in->i", np.conj(a), R_inv, a).real[:, None]        # eq. (27)
    rho_ax = np.einsum("im,imn,ijn->ij", np.conj(a), R_inv, x)                     # eq. (29)
    rho_xx = np.einsum("ijm,imn,ijn->ij", np.conj(x), R_inv, x).real               # eq. (31)
    ru_new = (gamma_t * rho_aa * (ru + gamma_t * np.abs(rho_ax_t) ** 2)
              + rho_xx - 2.0 * gamma_t * np.real(rho_ax_t * np.conj(rho_ax))) / M  # eq. (45)
    return rh_new, ru_new, lam_new


def run(x, a, Rp, b, rh0, ru0, lam0, K, alpha, beta):
    rh, ru, lam = (np.array(v, dtype=np.float64) for v in (rh0, ru0, lam0))
    for _ in range(K):
        rh, ru, lam = step(x, a, Rp, b, rh, ru, lam, alpha, beta)
    return rh, ru, lam
