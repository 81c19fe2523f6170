"""Small FP64 linear-algebra definitions shared by the oracle modules."""
import numpy as np


def herm(A):
    """Conjugate transpose over the last two axes."""
    return np.conj(np.swapaxes(A, -1, -2))


def pinv_rank(Rp, rank):
    """Moore-Penrose pseudoinverse of Hermitian PSD matrices of known rank.

    (R')^+ is the pseudoinverse of the rank-(M-1) SCM (Sec. III-B-2); for a
    Hermitian PSD matrix it inverts the ``rank`` largest eigenvalues and
    drops the rest.  Rp: [..., M, M].
    """
    w, V = np.linalg.eigh(Rp)
    M = Rp.shape[-1]
    inv = np.zeros_like(w)
    inv[..., M - rank:] = 1.0 / w[..., M - rank:]
    return (V * inv[..., None, :]) @ herm(V)


def quad(u, A, v):
    """u^H A v for batches: u [..., M], A [..., M, M], v [..., M]."""
    return np.einsum("...m,...mn,...n->...", np.conj(u), A, v)
