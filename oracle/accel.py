"""Second-stage accelerated update (Algorithm 2), FP64.

Precomputation, done once before the iterations (Sec. III-C-2):
  sigma^(ab)_i  = a_i^H b_i                         eq. (32)
  sigma^(bx)_ij = b_i^H x_ij                        eq. (33)
  tau^(aa)_i    = a_i^H (R'_i)^+ a_i                eq. (46)
  tau^(ax)_ij   = a_i^H (R'_i)^+ x_ij               eq. (47)
  tau^(xx)_ij   = x_ij^H (R'_i)^+ x_ij              eq. (48)

Each iteration uses only these scalars (eqs. (49)-(56)), in the order of
Algorithm 2: gamma~ from the values at the start of the iteration, then r^h,
then lambda, then r^u with the *new* lambda.

Array layout as in ``oracle.naive``.
"""
import numpy as np

from .linalg import pinv_rank, quad


def precompute(x, a, Rp, b):
    """Returns dict(s_ab [I], s_bx [I,J], t_aa [I], t_ax [I,J], t_xx [I,J])."""
    M = Rp.shape[-1]
    x = x.astype(np.complex128)
    Rpp = pinv_rank(Rp, M - 1)
    s_ab = np.einsum("im,im->i", np.conj(a), b)                          # eq. (32)
    s_bx = np.einsum("im,ijm->ij", np.conj(b), x)                        # eq. (33)
    t_aa = quad(a, Rpp, a).real                                          # eq. (46)
    t_ax = np.einsum("im,imn,ijn->ij", np.conj(a), Rpp, x)               # eq. (47)
    t_xx = np.einsum("ijm,imn,ijn->ij", np.conj(x), Rpp, x).real         # eq. (48)
    return dict(s_ab=s_ab, s_bx=s_bx, t_aa=t_aa, t_ax=t_ax, t_xx=t_xx, M=M)


def step(pre, rh, ru, lam, alpha, beta):
    """One second-stage iteration on all bins; returns new (rh, ru, lam)."""
    M = pre["M"]
    s_ab = pre["s_ab"][:, None]
    s_bx = pre["s_bx"]
    t_aa = pre["t_aa"][:, None]
    t_ax = pre["t_ax"]
    t_xx = pre["t_xx"]
    # values at the start of the iteration (tilde)
    rh_t, ru_t, lam_t = rh, ru, lam[:, None]
    rho_aa_t = t_aa + np.abs(s_ab) ** 2 / lam_t                           # eq. (50)
    rho_ax_t = t_ax + s_ab * s_bx / lam_t                                # eq. (52)
    gamma_t = rh_t / (ru_t + rh_t * rho_aa_t)                            # eq. (34)
    rh_new = (gamma_t * (ru_t + gamma_t * np.abs(rho_ax_t) ** 2) + beta) / (alpha + 2.0)  # eq. (54)
    lam_new = np.mean(gamma_t * np.abs(s_ab) ** 2
                      + np.abs(s_bx - gamma_t * np.conj(s_ab) * rho_ax_t) ** 2 / ru_t,
                      axis=1)                                            # eq. (55)
    lam_n = lam_new[:, None]
    rho_aa = t_aa + np.abs(s_ab) ** 2 / lam_n                             # eq. (49)
    rho_ax = t_ax + s_ab * s_bx / lam_n                                  # eq. (51)
    rho_xx = t_xx + np.abs(s_bx) ** 2 / lam_n                             # eq. (53)
    ru_new = (gamma_t * rho_aa * (ru_t + gamma_t * np.abs(rho_ax_t) ** 2)
              + rho_xx
              - 2.0 * gamma_t * np.real(rho_ax_t * np.conj(rho_ax))) / M  # eq. (56)
    return rh_new, ru_new, lam_new


def run(x, a, Rp, b, rh0, ru0, lam0, K, alpha, beta, history=False, pre=None):
    """K second-stage iterations from (rh0, ru0, lam0)."""
    if pre is None:
        pre = precompute(x, a, Rp, b)
    rh = np.array(rh0, dtype=np.float64)
    ru = np.array(ru0, dtype=np.float64)
    lam = np.array(lam0, dtype=np.float64)
    hist = [(rh, ru, lam)]
    for _ in range(K):
        rh, ru, lam = step(pre, rh, ru, lam, alpha, beta)
        hist.append((rh, ru, lam))
    return hist if history else (rh, ru, lam)


def init_state(I, J, rh0=1.0, ru0=1.0, lam0=1.0):
    """Constant initial state (the workloads start from r^h = r^u = lambda = 1)."""
    return (np.full((I, J), float(rh0)), np.full((I, J), float(ru0)), np.full(I, float(lam0)))
