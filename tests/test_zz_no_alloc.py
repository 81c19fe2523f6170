"""rcscm_run_noalloc (no context, no device allocation; status words in the library's static
scratch) against rcscm_run on a context, through the C ABI: bitwise equal outputs on two calls in
a row, the second with a smaller input, plus the oracle bar and the data-error report."""
import numpy as np
import pytest
import torch

from helpers import assert_close, oracle_accel
from synth import make_problem

pytestmark = pytest.mark.gpu


def _out(I, J, dev):
    return dict(rh=torch.empty(I * J, dtype=torch.float32, device=dev),
                ru=torch.empty(I * J, dtype=torch.float32, device=dev),
                lam=torch.empty(I, dtype=torch.float32, device=dev),
                s_hat=torch.empty(I * J, dtype=torch.complex64, device=dev))


def test_noalloc_equals_run_on_two_calls_second_smaller():
    from paper_1908_01964_amd import Context, to_device
    from paper_1908_01964_amd.rcscm import run_noalloc
    K = 12
    for (M, I, J, cfg) in ((4, 96, 1000, 491), (3, 17, 300, 492)):
        p = make_problem(M, I, J, config=cfg, spatial="sinc" if M % 2 == 0 else "random",
                         n_fft=2 * (I - 1))
        x, a, Rp, b = to_device(p)
        ctx = Context(I, [J], [M])
        ref = ctx.run(x, a, Rp, b, K)
        ctx.sync()
        out = _out(I, J, x.device)
        for v in out.values():
            v.fill_(float("nan"))  # every output element must be written by the call
        run_noalloc(I, J, M, x, a, Rp, b, K, out, check=True)
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(out[k], ref[k]), (M, I, J, k)
        ctx.close()
        o = {k: v.cpu().numpy().reshape((I, J) if k != "lam" else (I,)) for k, v in out.items()}
        assert_close(o, oracle_accel(p, K), what=f"noalloc M={M} I={I} J={J}")


def test_noalloc_unchecked_then_checked_and_data_error():
    from paper_1908_01964_amd import RcscmError, to_device
    from paper_1908_01964_amd.rcscm import run_noalloc
    p = make_problem(4, 6, 200, config=493)
    x, a, Rp, b = to_device(p)
    out = _out(p.I, p.J, x.device)
    run_noalloc(p.I, p.J, p.M, x, a, Rp, b, 5, out, check=False)
    torch.cuda.synchronize()
    first = {k: v.clone() for k, v in out.items()}
    run_noalloc(p.I, p.J, p.M, x, a, Rp, b, 5, out, check=True)
    for k in out:
        assert torch.equal(out[k], first[k]), k
    xb = x.clone()
    xb[3 * p.J * p.M + 7] = float("nan")  # one observation of row 3
    with pytest.raises(RcscmError) as ei:
        run_noalloc(p.I, p.J, p.M, xb, a, Rp, b, 5, out, check=True)
    assert ei.value.status == -5 and "row 3" in str(ei.value)
    # the next clean call on the same scratch reports no error
    run_noalloc(p.I, p.J, p.M, x, a, Rp, b, 5, out, check=True)
    for k in out:
        assert torch.equal(out[k], first[k]), k
    assert np.isfinite(out["rh"].cpu().numpy()).all()
