"""Shared helpers of the GPU parity tests: run the HIP path and the FP64 oracle on the same input."""
import numpy as np

from oracle import accel as o_accel
from oracle import extract as o_extract
from oracle import naive as o_naive
from synth import ALPHA, BETA

TOL = 1e-4  # normwise relative error after K iterations (FP32 kernel vs FP64 oracle)
# Normwise relative error of every single frequency row (r^h, r^u, s_hat over the row's frames;
# lambda per row).  Looser than TOL: one row can be ill-conditioned (the sinc-coherence DC row
# is rank one plus 1e-3 loading), and a row holds as few as one frame.
ROW_TOL = 1e-3


def nrel(est, ref):
    est = np.asarray(est).ravel()
    ref = np.asarray(ref).ravel()
    return float(np.linalg.norm(est - ref) / max(np.linalg.norm(ref), 1e-300))


def gpu_run(problems, K, init_arrays=None, fused=False, **params):
    """Runs init + iterate(K) + extract on the GPU (fused=True: the single call rcscm_run);
    returns per-utterance numpy dicts."""
    import torch

    from paper_1908_01964_amd import Context, to_device
    probs = problems if isinstance(problems, (list, tuple)) else [problems]
    I = probs[0].x.shape[0]
    Js = [p.x.shape[1] for p in probs]
    Ms = [p.x.shape[2] for p in probs]
    x, a, Rp, b = to_device(probs)
    ctx = Context(I, Js, Ms, **params)
    kw = {}
    if init_arrays is not None:
        kw = {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32).ravel()).cuda()
              for k, v in init_arrays.items()}
    if fused:
        out = ctx.run(x, a, Rp, b, K, **kw)
    else:
        ctx.init(x, a, Rp, b, **kw)
        ctx.iterate(K)
        out = ctx.extract()
    ctx.sync()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    ctx.close()
    return split(res, I, Js)


def split(res, I, Js):
    outs = []
    bo, ro = 0, 0
    for J in Js:
        d = {}
        for k in ("rh", "ru", "s_hat"):
            if k in res:
                d[k] = res[k][bo:bo + I * J].reshape(I, J)
        d["lam"] = res["lam"][ro:ro + I]
        outs.append(d)
        bo += I * J
        ro += I
    return outs


def oracle_accel(p, K, rh0=None, ru0=None, lam0=None, alpha=ALPHA, beta=BETA):
    st = o_accel.init_state(p.I, p.J)
    rh0 = st[0] if rh0 is None else rh0
    ru0 = st[1] if ru0 is None else ru0
    lam0 = st[2] if lam0 is None else lam0
    rh, ru, lam = o_accel.run(p.x, p.a, p.Rp, p.b, rh0, ru0, lam0, K, alpha, beta)
    sh = o_extract.s_hat(p.x, p.a, p.Rp, p.b, rh, ru, lam)
    return dict(rh=rh, ru=ru, lam=lam, s_hat=sh)


def oracle_naive(p, K, alpha=ALPHA, beta=BETA):
    st = o_accel.init_state(p.I, p.J)
    rh, ru, lam = o_naive.run(p.x, p.a, p.Rp, p.b, *st, K, alpha, beta)
    sh = o_extract.s_hat(p.x, p.a, p.Rp, p.b, rh, ru, lam)
    return dict(rh=rh, ru=ru, lam=lam, s_hat=sh)


def errors(gpu, ref):
    return {k: nrel(gpu[k], ref[k]) for k in ("rh", "ru", "lam", "s_hat") if k in gpu}


def row_errors(gpu, ref):
    """Per quantity: (largest normwise relative error of one row, that row's index)."""
    out = {}
    for k in ("rh", "ru", "lam", "s_hat"):
        if k not in gpu:
            continue
        r = np.asarray(ref[k])
        g = np.asarray(gpu[k]).reshape(r.shape)
        if r.ndim == 2:
            e = np.linalg.norm(g - r, axis=1) / np.maximum(np.linalg.norm(r, axis=1), 1e-300)
        else:
            e = np.abs(g - r) / np.maximum(np.abs(r), 1e-300)
        out[k] = (float(e.max()), int(e.argmax()))
    return out


def elementwise(gpu, ref):
    """Per quantity: max and 99.9th percentile of |est - ref| / |ref| (reported, not gated:
    r^h near its floor beta / (alpha + 2) makes single elements meaningless)."""
    out = {}
    for k in ("rh", "ru", "lam", "s_hat"):
        if k not in gpu:
            continue
        r = np.asarray(ref[k]).ravel()
        g = np.asarray(gpu[k]).ravel()
        e = np.abs(g - r) / np.maximum(np.abs(r), 1e-300)
        out[k] = (float(e.max()), float(np.percentile(e, 99.9)))
    return out


def assert_close(gpu, ref, tol=TOL, what="", row_tol=ROW_TOL):
    """The parity bar: normwise relative error <= tol per quantity, and <= row_tol for every
    frequency row.  Prints the elementwise max and 99.9th percentile beside them."""
    e = errors(gpu, ref)
    bad = {k: v for k, v in e.items() if not (v <= tol)}
    assert not bad, f"{what} normwise relative errors above {tol}: {e}"
    r = row_errors(gpu, ref)
    bad = {k: v for k, v in r.items() if not (v[0] <= row_tol)}
    assert not bad, f"{what} row errors above {row_tol} (error, row): {r}"
    el = elementwise(gpu, ref)
    print(f"{what} normwise {e} worst row {r} elementwise (max, p99.9) {el}")
    return e
