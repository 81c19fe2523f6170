"""Objective of the rank-constrained SCM model, FP64, by slogdet + solve.

Marginalising s and u in eqs. (2)-(10) gives x_ij ~ N_c(0, Sigma_ij) with
Sigma_ij = r^h_ij a_i a_i^H + r^u_ij (R'_i + lambda_i b_i b_i^H).  The
estimation is MAP with the inverse-gamma prior of eq. (7) on r^h (Sec. II-B-2),
so the quantity the EM iteration cannot increase is the negative
log-posterior

  NLP = sum_ij [ M log pi + log det Sigma_ij + x^H Sigma_ij^{-1} x ]
        + sum_ij [ (alpha + 1) log r^h_ij + beta / r^h_ij ]   (+ const).

With alpha = -1, beta = 0 the prior term vanishes and NLP = NLL.
"""
import numpy as np


def sigma(a, Rp, b, rh, ru, lam):
    """Model covariance Sigma [I, J, M, M]."""
    R = Rp + lam[:, None, None] * np.einsum("im,in->imn", b, np.conj(b))
    aa = np.einsum("im,in->imn", a, np.conj(a))
    return rh[..., None, None] * aa[:, None] + ru[..., None, None] * R[:, None]


def nll_terms(x, a, Rp, b, rh, ru, lam):
    """Per-bin negative log-likelihood [I, J]."""
    M = x.shape[-1]
    S = sigma(a, Rp, b, rh, ru, lam)
    sign, logdet = np.linalg.slogdet(S)
    x = x.astype(np.complex128)
    q = np.einsum("ijm,ijm->ij", np.conj(x), np.linalg.solve(S, x[..., None])[..., 0]).real
    return M * np.log(np.pi) + logdet + q


def nll(x, a, Rp, b, rh, ru, lam):
    return float(np.sum(nll_terms(x, a, Rp, b, rh, ru, lam)))


def nlp(x, a, Rp, b, rh, ru, lam, alpha, beta):
    prior = (alpha + 1.0) * np.log(rh) + beta / rh
    return nll(x, a, Rp, b, rh, ru, lam) + float(np.sum(prior))
