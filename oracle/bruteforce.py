"""Brute-force E- and M-steps, used only to pin the closed forms on tiny inputs.

E-step: the sufficient statistics h_hat = E[|s|^2 | x] and
U_hat = E[u u^H | x] of eqs. (15)-(16) are recomputed two ways that do not
use those equations:
  * ``estep_joint``: generic conditioning of the stacked Gaussian vector
    [s; u; x] (x = a s + u, Sec. II-B-1), covariance form, one linear solve.
  * ``estep_precision``: u = x - a s is determined by s, so p(s | x) is a
    one-dimensional Gaussian whose precision is 1/r~h + a^H (r~u R~)^{-1} a.
M-step: the Q function of eq. (12) is maximised numerically in one variable
at a time (r^h; then lambda with r^u held at r~u; then r^u with the new
lambda), by bounded Brent search over the log of the variable.
"""
import numpy as np
from scipy.optimize import minimize_scalar


def estep_joint(x, a, R_t, rh_t, ru_t):
    """One bin. Returns (h_hat, U_hat, s_mean) from generic Gaussian conditioning."""
    M = a.shape[0]
    # latent z = [s; u] with block-diagonal prior covariance
    D = np.zeros((1 + M, 1 + M), np.complex128)
    D[0, 0] = rh_t
    D[1:, 1:] = ru_t * R_t
    # full vector [s; u; x] = L z
    L = np.zeros((1 + 2 * M, 1 + M), np.complex128)
    L[0, 0] = 1.0
    L[1:1 + M, 1:] = np.eye(M)
    L[1 + M:, 0] = a
    L[1 + M:, 1:] = np.eye(M)
    C = L @ D @ L.conj().T
    Czx = C[:1 + M, 1 + M:]
    Cxx = C[1 + M:, 1 + M:]
    Czz = C[:1 + M, :1 + M]
    mean = Czx @ np.linalg.solve(Cxx, x)
    cov = Czz - Czx @ np.linalg.solve(Cxx, Czx.conj().T)
    second = cov + np.outer(mean, np.conj(mean))
    return float(second[0, 0].real), second[1:, 1:], complex(mean[0])


def estep_precision(x, a, R_t, rh_t, ru_t):
    """One bin. Posterior of the scalar s given x; returns (h_hat, U_hat, s_mean)."""
    Ru_inv = np.linalg.inv(ru_t * R_t)
    prec = 1.0 / rh_t + np.real(np.conj(a) @ Ru_inv @ a)
    var = 1.0 / prec
    mean = var * (np.conj(a) @ Ru_inv @ x)
    h_hat = var + abs(mean) ** 2
    r = x - a * mean
    U_hat = np.outer(r, np.conj(r)) + var * np.outer(a, np.conj(a))
    return float(h_hat), U_hat, complex(mean)


def _argmax_log(f, lo, hi):
    """Maximise f(v) over v in [lo, hi] (v > 0) by bounded search on log v."""
    res = minimize_scalar(lambda t: -f(np.exp(t)), bounds=(np.log(lo), np.log(hi)),
                          method="bounded", options=dict(xatol=1e-12, maxiter=2000))
    return float(np.exp(res.x))


def mstep_numeric(Rp, b, ru_t, h_hat, U_hat, alpha, beta, lo=1e-12, hi=1e6):
    """One frequency row: maximise Q (eq. (12)) coordinate-wise.

    ru_t, h_hat [J]; U_hat [J, M, M].  Returns (rh [J], lam, ru [J]).
    """
    J, M = U_hat.shape[0], U_hat.shape[1]
    bb = np.outer(b, np.conj(b))

    rh = np.array([_argmax_log(lambda r: -(alpha + 2.0) * np.log(r) - (h + beta) / r, lo, hi)
                   for h in h_hat])

    def q_lam(lam):
        R = Rp + lam * bb
        _, logdet = np.linalg.slogdet(R)
        R_inv = np.linalg.inv(R)
        tr = np.einsum("mn,jnm->j", R_inv, U_hat).real
        return float(np.sum(-logdet - tr / ru_t))

    lam = _argmax_log(q_lam, lo, hi)
    R_inv = np.linalg.inv(Rp + lam * bb)
    tr = np.einsum("mn,jnm->j", R_inv, U_hat).real
    ru = np.array([_argmax_log(lambda r: -M * np.log(r) - t / r, lo, hi) for t in tr])
    return rh, lam, ru
