"""GPU adjoint (rcscm_backward through torch.autograd) against the FP64 torch autograd reference.

The reference (oracle/adjoint_ref.py) is itself pinned to central finite
differences of the numpy oracle in tests/test_oracle_adjoint.py.  Loss:
L = sum |s_hat - s_true|^2 after K accelerated iterations and extraction.
Rows are independent, so gradients of sampled rows are exact references for
a full-size run.
"""
import numpy as np
import pytest

from helpers import nrel
from oracle import adjoint_ref
from synth import ALPHA, BETA, config, make_problem

pytestmark = pytest.mark.gpu

TOL_GRAD = 1e-4  # normwise, FP32 forward + adjoint vs FP64 (measured <= 1.4e-5)


def _gpu_grads(p, K, rh0, lam0, **params):
    import torch

    from paper_1908_01964_amd import to_device
    from paper_1908_01964_amd.autograd import estimate_and_extract
    x, a, Rp, b = to_device(p)
    x = x.clone().requires_grad_(True)
    rh0_t = torch.from_numpy(rh0.astype(np.float32).ravel()).cuda().requires_grad_(True)
    lam0_t = torch.from_numpy(lam0.astype(np.float32)).cuda().requires_grad_(True)
    s_true = torch.from_numpy(p.s_true.ravel()).cuda()
    s_hat, rh, ru, lam = estimate_and_extract(x, rh0_t, lam0_t, a, Rp, b, K, I=p.I, Js=[p.J],
                                              Ms=[p.M], **params)
    loss = torch.sum(torch.abs(s_hat - s_true) ** 2)
    loss.backward()
    torch.cuda.synchronize()
    return (float(loss), x.grad.cpu().numpy().reshape(p.x.shape),
            rh0_t.grad.cpu().numpy().reshape(p.I, p.J), lam0_t.grad.cpu().numpy())


@pytest.mark.parametrize("M,J,K,block", [(2, 100, 3, 0), (4, 150, 5, 0), (4, 300, 10, 64),
                                         (6, 65, 4, 256), (8, 257, 5, 128)])
def test_adjoint_matches_fp64_autograd(M, J, K, block):
    p = make_problem(M, 5, J, config=500 + M, spatial="sinc" if M % 2 == 0 else "random",
                     n_fft=16)
    rng = np.random.default_rng(M)
    rh0 = rng.uniform(0.5, 2.0, (p.I, p.J))
    lam0 = rng.uniform(0.5, 2.0, p.I)
    rh0 = rh0.astype(np.float32).astype(np.float64)
    lam0 = lam0.astype(np.float32).astype(np.float64)
    ru0 = np.ones((p.I, p.J))
    loss_r, _, gx_r, grh_r, glam_r = adjoint_ref.torch_grads(p.x, p.a, p.Rp, p.b, rh0, ru0, lam0,
                                                             K, ALPHA, BETA, p.s_true)
    loss, gx, grh, glam = _gpu_grads(p, K, rh0, lam0, block=block)
    e = dict(loss=abs(loss - loss_r) / loss_r, x=nrel(gx, gx_r), rh0=nrel(grh, grh_r),
             lam0=nrel(glam, glam_r))
    print("adjoint", M, J, K, e)
    assert e["loss"] < 1e-4
    assert e["x"] < TOL_GRAD and e["rh0"] < TOL_GRAD and e["lam0"] < TOL_GRAD, e


def test_adjoint_config3_full_size_sampled_rows():
    """Config 3: M=4, I=513, J=1000, K=10, FP32 forward + adjoint over every row; 12 rows checked."""
    p = config(3)
    K = p.meta["K"]
    rh0 = np.ones((p.I, p.J))
    lam0 = np.ones(p.I)
    loss, gx, grh, glam = _gpu_grads(p, K, rh0, lam0)
    assert np.isfinite(loss)
    sel = np.linspace(0, p.I - 1, 12).round().astype(int)
    sub = config(3, freqs=sel)
    _, _, gx_r, grh_r, glam_r = adjoint_ref.torch_grads(sub.x, sub.a, sub.Rp, sub.b,
                                                        rh0[sel], np.ones((len(sel), p.J)),
                                                        lam0[sel], K, ALPHA, BETA, sub.s_true)
    e = dict(x=nrel(gx[sel], gx_r), rh0=nrel(grh[sel], grh_r), lam0=nrel(glam[sel], glam_r))
    print("adjoint config3 (sampled rows)", e)
    assert all(v < TOL_GRAD for v in e.values()), e


def test_backward_requires_checkpoints():
    import torch

    from paper_1908_01964_amd import Context, RcscmError, to_device
    p = make_problem(2, 2, 10, config=510)
    x, a, Rp, b = to_device(p)
    c = Context.single(p.I, p.J, p.M)
    c.init(x, a, Rp, b).iterate(2)
    with pytest.raises(RcscmError) as ei:
        c.backward(x, torch.zeros(p.I * p.J, dtype=torch.complex64, device="cuda"))
    assert ei.value.status == -8
    c.close()


def test_backward_after_run_equals_after_separate_calls():
    """Checkpoints kept by the fused rcscm_run drive the same adjoint as init + iterate + extract."""
    import torch

    from paper_1908_01964_amd import Context, to_device
    p = make_problem(4, 6, 700, config=511, spatial="sinc", n_fft=16)
    x, a, Rp, b = to_device(p)
    K = 6
    g = torch.randn(p.I * p.J, dtype=torch.complex64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(5))
    grads = []
    for fused in (False, True):
        c = Context.single(p.I, p.J, p.M, checkpoint=True, schedule="resident", block=256)
        if fused:
            c.run(x, a, Rp, b, K)
        else:
            c.init(x, a, Rp, b).iterate(K)
            c.extract()
        grads.append([t.cpu() for t in c.backward(x, g)])
        c.sync()
        c.close()
    for u, v in zip(*grads):
        assert torch.equal(u, v)


def test_checkpoint_storage_grows():
    """A longer second run replaces the checkpoint buffers; the adjoint then equals a fresh one."""
    import torch

    from paper_1908_01964_amd import Context, to_device
    p = make_problem(3, 4, 300, config=512)
    x, a, Rp, b = to_device(p)
    g = torch.randn(p.I * p.J, dtype=torch.complex64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(6))
    c1 = Context.single(p.I, p.J, p.M, checkpoint=True)
    c1.run(x, a, Rp, b, 3)
    c1.run(x, a, Rp, b, 8)
    g1 = [t.cpu() for t in c1.backward(x, g)]
    c1.sync()
    c1.close()
    c2 = Context.single(p.I, p.J, p.M, checkpoint=True)
    c2.run(x, a, Rp, b, 8)
    g2 = [t.cpu() for t in c2.backward(x, g)]
    c2.sync()
    c2.close()
    for u, v in zip(g1, g2):
        assert torch.equal(u, v)
