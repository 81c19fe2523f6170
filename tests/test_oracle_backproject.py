"""Pins of the back-projection oracle (eq. (11)) and the paper's initialisation (eqs. (22),
(23), minimum nonzero eigenvalue), against closed forms of a determined mixture."""
import numpy as np
import pytest

from oracle import backproject as bp
from oracle.linalg import herm
from synth import make_bss_problem


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("M,n_h", [(2, 0), (4, 1), (6, 5)])
def test_perfect_separation_closed_forms(M, n_h):
    """W = A^{-1}: y = W x = s, so R' = sum_{m != n_h} mean_j |s_m|^2 a_m a_m^H and the
    noise image is x - a_{n_h} s_{n_h}."""
    d = make_bss_problem(M, 3, 40, config=610 + M, target=n_h)
    x, W, A = d["x"], d["W"], d["A"]
    s = np.einsum("imn,ijn->ijm", W, x.astype(np.complex128))   # = the sources, up to rounding
    p = np.mean(np.abs(s) ** 2, axis=1)                         # [I, M]
    Rp_ref = np.zeros((3, M, M), np.complex128)
    for m in range(M):
        if m != n_h:
            Rp_ref += p[:, m, None, None] * np.einsum("im,in->imn", A[:, :, m], A[:, :, m].conj())
    Rp = bp.rprime(x, W, n_h)
    assert _rel(Rp, Rp_ref) < 1e-10
    assert _rel(bp.steering(W, n_h), A[:, :, n_h]) < 1e-10
    yu = bp.noise_image(x, W, n_h)
    yu_ref = x.astype(np.complex128) - A[:, None, :, n_h] * s[:, :, n_h, None]
    assert _rel(yu, yu_ref) < 1e-9
    # r^u_0: for y^(u) in range(R') the pseudoinverse form reduces to whitened energies
    ru_ref = np.sum(np.delete(np.abs(s) ** 2 / p[:, None, :], n_h, axis=2), axis=2) / M
    assert _rel(bp.ru_init(x, W, n_h), ru_ref) < 1e-9


@pytest.mark.parametrize("M", [3, 5, 8])
def test_rank_null_vector_and_min_eigenvalue(M):
    d = make_bss_problem(M, 4, 60, config=620 + M, target=1, perturb=0.3)
    x, W = d["x"], d["W"]
    Rp = bp.rprime(x, W, 1)
    assert np.allclose(Rp, herm(Rp))
    ev = np.linalg.eigvalsh(Rp)
    assert np.all(np.abs(ev[:, 0]) < 1e-12 * ev[:, -1]) and np.all(ev[:, 1] > 0)
    b = bp.null_vector(Rp)
    assert np.max(np.abs(np.einsum("imn,in->im", Rp, b))) < 1e-12 * ev[:, -1].max()
    # b spans the same line as w_{n_h} (W A = I kills the other components)
    w = W[:, 1, :].conj()
    w = w / np.linalg.norm(w, axis=1, keepdims=True)
    assert np.allclose(np.abs(np.einsum("im,im->i", b.conj(), w)), 1.0, atol=1e-10)
    # minimum nonzero eigenvalue = smallest eigenvalue of the (M-1)x(M-1) Gram matrix
    y = np.einsum("imn,ijn->ijm", W, x.astype(np.complex128))
    p = np.mean(np.abs(y) ** 2, axis=1)
    B = np.delete(np.linalg.inv(W), 1, axis=2)                  # columns m != n_h
    sq = np.sqrt(np.delete(p, 1, axis=1))
    G = sq[:, :, None] * (herm(B) @ B) * sq[:, None, :]
    assert _rel(bp.lam_init(Rp), np.linalg.eigvalsh(G)[:, 0]) < 1e-10
