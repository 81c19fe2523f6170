"""Pin of the FP64 autograd reference: central finite differences of the numpy forward."""
import numpy as np
import pytest

from oracle import adjoint_ref
from synth import ALPHA, BETA, make_problem


@pytest.mark.parametrize("M,K", [(2, 3), (4, 5)])
def test_torch_reference_matches_central_differences(M, K):
    p = make_problem(M, 3, 12, config=301, spatial="sinc", n_fft=8)
    rng = np.random.default_rng(11)
    rh0 = np.ones((p.I, p.J))
    ru0 = np.ones((p.I, p.J))
    lam0 = np.ones(p.I)
    loss, s_hat, gx, grh, glam = adjoint_ref.torch_grads(p.x, p.a, p.Rp, p.b, rh0, ru0, lam0, K,
                                                         ALPHA, BETA, p.s_true)
    assert abs(loss - adjoint_ref.loss_numpy(p.x, p.a, p.Rp, p.b, rh0, ru0, lam0, K, ALPHA, BETA,
                                             p.s_true)) < 1e-10 * abs(loss)
    vx = rng.standard_normal(p.x.shape) + 1j * rng.standard_normal(p.x.shape)
    vrh = rng.standard_normal(rh0.shape)
    vlam = rng.standard_normal(lam0.shape)
    for kw, pred in ((dict(vx=vx), np.sum(np.real(np.conj(gx) * vx))),
                     (dict(vrh=vrh), np.sum(grh * vrh)),
                     (dict(vlam=vlam), np.sum(glam * vlam))):
        fd = adjoint_ref.fd_directional(p.x, p.a, p.Rp, p.b, rh0, ru0, lam0, K, ALPHA, BETA,
                                        p.s_true, h=1e-5, **kw)
        assert abs(fd - pred) <= 1e-5 * max(abs(pred), 1e-8 * abs(loss)), (kw.keys(), fd, pred)
