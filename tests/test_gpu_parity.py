"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle, element by element.

Bar: normwise relative error <= 1e-4 after K iterations for r^h, r^u, lambda
and s_hat (FP32 kernels vs FP64 oracle); bit-exact where the same schedule
runs the same reduction order (resume, batch vs single, graph vs eager).
"""
import numpy as np
import pytest

from helpers import assert_close, gpu_run, oracle_accel, oracle_naive
from synth import ALPHA, BETA, config, make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c0():
    return config(0)


@pytest.mark.parametrize("schedule,lamsum,graph", [("resident", "f64", False),
                                                   ("resident", "kahan32", False),
                                                   ("stream", "f64", False),
                                                   ("stream", "kahan32", True)])
def test_config0_accel_vs_oracle(c0, schedule, lamsum, graph):
    ref = oracle_accel(c0, 20)
    out = gpu_run(c0, 20, schedule=schedule, lamsum=lamsum, graph=graph)[0]
    e = assert_close(out, ref, what=f"config 0 {schedule}/{lamsum}")
    print("config0", schedule, lamsum, e)


@pytest.mark.parametrize("M", [2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("J", [1, 63, 64, 65, 1001])
def test_shapes_and_ragged_tails(M, J):
    p = make_problem(M, 3, J, config=400 + M, spatial="sinc" if M % 2 == 0 else "random",
                     n_fft=8)
    ref = oracle_accel(p, 10)
    for schedule in ("resident", "stream"):
        out = gpu_run(p, 10, schedule=schedule, chunk=256)[0]
        assert_close(out, ref, what=f"M={M} J={J} {schedule}")


@pytest.mark.parametrize("block", [64, 128, 256, 512, 1024])
def test_resident_block_sizes(c0, block):
    sub = config(0, freqs=range(0, 257, 16))
    ref = oracle_accel(sub, 20)
    out = gpu_run(sub, 20, schedule="resident", block=block)[0]
    assert_close(out, ref, what=f"block {block}")


@pytest.mark.parametrize("M", [2, 4, 6, 8])
def test_naive_vs_oracle(M):
    p = make_problem(M, 4, 300, config=420 + M, spatial="random")
    ref = oracle_naive(p, 10)
    out = gpu_run(p, 10, rule="naive")[0]
    assert_close(out, ref, what=f"naive M={M}")


def test_naive_recompute_equals_stored_u():
    """The naive rule with U^ recomputed in the second launch (RCSCM_FLAG_NAIVE_RECOMPUTE)
    gives the stored form's results bit for bit: same E-step, same trace order.  A ragged
    batch of mixed M with an odd number of iterations (the recompute form swaps its lambda
    buffers every iteration)."""
    probs = [make_problem(m, 5, j, config=480 + m, utterance=u, spatial="random")
             for u, (j, m) in enumerate([(300, 2), (777, 4), (129, 8), (513, 5)])]
    a = gpu_run(probs, 7, rule="naive")
    b = gpu_run(probs, 7, rule="naive", naive_recompute=True)
    for u, (ra, rb) in enumerate(zip(a, b)):
        for k in ra:
            assert np.array_equal(ra[k], rb[k]), (u, k)
    ref = oracle_naive(probs[1], 7)
    assert_close(b[1], ref, what="naive recompute M=4")


def test_naive_config0(c0):
    ref = oracle_naive(c0, 20)
    out = gpu_run(c0, 20, rule="naive")[0]
    assert_close(out, ref, what="naive config 0")


def test_resume_is_exact(c0):
    import torch

    from paper_1908_01964_amd import Context, to_device
    x, a, Rp, b = to_device(c0)
    for schedule in ("resident", "stream"):
        c1 = Context.single(c0.I, c0.J, c0.M, schedule=schedule)
        c1.init(x, a, Rp, b).iterate(20)
        o1 = c1.extract()
        c2 = Context.single(c0.I, c0.J, c0.M, schedule=schedule)
        c2.init(x, a, Rp, b).iterate(7).iterate(13)
        o2 = c2.extract()
        c3 = Context.single(c0.I, c0.J, c0.M, schedule=schedule)
        c3.init(x, a, Rp, b).iterate(7)
        mid = c3.extract(s_hat=False)
        c4 = Context.single(c0.I, c0.J, c0.M, schedule=schedule)
        c4.init(x, a, Rp, b).set_state(mid["rh"], mid["ru"], mid["lam"]).iterate(13)
        o4 = c4.extract()
        torch.cuda.synchronize()
        for k in o1:
            assert torch.equal(o1[k], o2[k]), (schedule, k)
            assert torch.equal(o1[k], o4[k]), (schedule, k)
        for c in (c1, c2, c3, c4):
            c.close()


def test_get_state_round_trip_is_exact(c0):
    """rcscm_get_state equals the state extract reports, and set_state(get_state) on a fresh
    context resumes bitwise (both schedules; after the fused run too)."""
    import torch

    from paper_1908_01964_amd import Context, to_device
    x, a, Rp, b = to_device(c0)
    for schedule, fused in (("resident", False), ("stream", False), ("auto", True)):
        c1 = Context.single(c0.I, c0.J, c0.M, schedule=schedule)
        if fused:
            c1.run(x, a, Rp, b, 7)
        else:
            c1.init(x, a, Rp, b).iterate(7)
        st = c1.get_state()
        ex = c1.extract(s_hat=False)
        torch.cuda.synchronize()
        for k in st:
            assert torch.equal(st[k], ex[k]), (schedule, k)
        c2 = Context.single(c0.I, c0.J, c0.M, schedule=schedule)
        c2.init(x, a, Rp, b).set_state(st["rh"], st["ru"], st["lam"]).iterate(5)
        c1.iterate(5)
        o1, o2 = c1.extract(), c2.extract()
        torch.cuda.synchronize()
        for k in o1:
            assert torch.equal(o1[k], o2[k]), (schedule, k)
        c1.close()
        c2.close()


@pytest.mark.parametrize("batch", [False, True])
def test_run_only_equals_run_and_keeps_no_state(batch):
    """RCSCM_FLAG_RUN_ONLY: the fused launch stores only the caller's outputs; they equal the
    default run bitwise, and calls that need the state are refused until the next init."""
    import torch

    from paper_1908_01964_amd import Context, RcscmError, to_device
    if batch:
        probs = [make_problem(m, 12, j, config=482, utterance=u, spatial="random")
                 for u, (j, m) in enumerate([(300, 2), (1500, 4), (3000, 3)])]
    else:
        probs = [make_problem(4, 16, 700, config=483, spatial="sinc", n_fft=30)]
    I, Js, Ms = 12 if batch else 16, [q.J for q in probs], [q.M for q in probs]
    x, a, Rp, b = to_device(probs)
    ref = Context(I, Js, Ms)
    o_ref = ref.run(x, a, Rp, b, 9)
    ref.sync()
    ctx = Context(I, Js, Ms, run_only=True)
    out = ctx.run(x, a, Rp, b, 9)
    ctx.sync()
    for k in o_ref:
        assert torch.equal(out[k], o_ref[k]), k
    for call in (lambda: ctx.iterate(1), lambda: ctx.extract(), lambda: ctx.get_state(),
                 lambda: ctx.objective()):
        with pytest.raises(RcscmError) as ei:
            call()
        assert ei.value.status == -8 and "RUN_ONLY" in str(ei.value)
    # a new init gives the context a state again: the same as the three calls on a context
    # without the flag (the RESIDENT classes sum lambda in their own lane grouping)
    ctx.init(x, a, Rp, b).iterate(9)
    o2 = ctx.extract()
    o3 = ref.init(x, a, Rp, b).iterate(9).extract()
    ctx.sync()
    ref.sync()
    for k in o3:
        assert torch.equal(o2[k], o3[k]), k
    ctx.close()
    ref.close()


def test_graph_equals_eager(c0):
    import torch

    from paper_1908_01964_amd import Context, to_device
    x, a, Rp, b = to_device(c0)
    ce = Context.single(c0.I, c0.J, c0.M, schedule="stream")
    ce.init(x, a, Rp, b)
    cg = Context.single(c0.I, c0.J, c0.M, schedule="stream", graph=True)
    cg.init(x, a, Rp, b)
    for K in (5, 5, 3, 1):  # replays of the same graph and new ones, with eager work between
        ce.iterate(K)
        cg.iterate(K)
        oe, og = ce.extract(), cg.extract()
        torch.cuda.synchronize()
        for k in oe:
            assert torch.equal(oe[k], og[k]), (K, k)
    ce.close()
    cg.close()


@pytest.mark.parametrize("batch", [False, True])
def test_fused_run_captured_in_a_graph(batch):
    """rcscm_run captured into a HIP graph (through torch.cuda.graph) and replayed: every replay,
    with eager work and synchronisation between replays, equals the eager call bitwise.  The
    batch has three workgroup classes, so the capture includes the fork to and join from the
    auxiliary streams (created by the warm-up call)."""
    import torch

    from paper_1908_01964_amd import Context, to_device
    if batch:
        probs = [make_problem(m, 16, j, config=481, utterance=u, spatial="random")
                 for u, (j, m) in enumerate([(300, 2), (1500, 4), (3000, 3)])]
    else:
        probs = [make_problem(4, 16, 600, config=480, spatial="sinc", n_fft=32)]
    I = 16
    Js = [q.J for q in probs]
    Ms = [q.M for q in probs]
    x, a, Rp, b = to_device(probs)
    ref = Context(I, Js, Ms)
    o_ref = ref.run(x, a, Rp, b, 7)
    ref.sync()
    s = torch.cuda.Stream()
    ctx = Context(I, Js, Ms, stream=s)
    out = {k: torch.empty_like(v) for k, v in o_ref.items()}
    with torch.cuda.stream(s):
        ctx.run(x, a, Rp, b, 7, out=out)  # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ctx.run(x, a, Rp, b, 7, out=out)
    for rep in range(3):
        for v in out.values():
            v.fill_(float("nan"))  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in o_ref:
            assert torch.equal(out[k], o_ref[k]), (rep, k)
    ctx.sync()
    ctx.close()
    ref.close()


@pytest.mark.parametrize("fused", [False, True])
def test_explicit_initial_state(fused):
    p = make_problem(4, 5, 200, config=430)
    rng = np.random.default_rng(1)
    rh0 = rng.gamma(1.0, 1.0, (p.I, p.J))
    ru0 = rng.gamma(2.0, 0.5, (p.I, p.J))
    lam0 = rng.uniform(0.2, 2.0, p.I)
    ref = oracle_accel(p, 10, rh0=rh0.astype(np.float32).astype(np.float64),
                       ru0=ru0.astype(np.float32).astype(np.float64),
                       lam0=lam0.astype(np.float32).astype(np.float64))
    out = gpu_run(p, 10, init_arrays=dict(rh0=rh0, ru0=ru0, lam0=lam0), fused=fused)[0]
    assert_close(out, ref, what=f"explicit init fused={fused}")


@pytest.mark.parametrize("fused", [False, True])
def test_zero_iterations_returns_init(c0, fused):
    out = gpu_run(c0, 0, fused=fused)[0]
    assert np.all(out["rh"] == 1.0) and np.all(out["ru"] == 1.0) and np.all(out["lam"] == 1.0)


@pytest.mark.parametrize("fused", [False, True])
def test_degenerate_zero_observations(fused):
    p = make_problem(3, 2, 65, config=431)
    p.x[0, 10:20] = 0  # silent frames are legal: r^u decays but stays positive
    ref = oracle_accel(p, 10)
    out = gpu_run(p, 10, fused=fused)[0]
    assert_close(out, ref, what="zero frames")
    assert np.all(out["ru"] > 0) and np.all(out["rh"] > 0)


@pytest.mark.parametrize("fused", [False, True])
def test_prior_ml_mode(fused):
    p = make_problem(4, 4, 100, config=432)
    ref = oracle_accel(p, 10, alpha=-1.0, beta=0.0)
    out = gpu_run(p, 10, alpha=-1.0, beta=0.0, fused=fused)[0]
    assert_close(out, ref, what="ML mode")


@pytest.mark.parametrize("fused", [False, True])
def test_data_errors_are_reported(fused):
    import torch

    from paper_1908_01964_amd import Context, RcscmError, to_device
    p = make_problem(4, 3, 50, config=433)
    x, a, Rp, b = to_device(p)

    def go(ctx, xx, bb_, K):  # init + iterate, or the single call rcscm_run
        if fused:
            ctx.run(xx, a, Rp, bb_, K)
        else:
            ctx.init(xx, a, Rp, bb_).iterate(K)
    # non-finite observation
    xb = x.clone()
    xb[7] = float("nan")
    ctx = Context.single(p.I, p.J, p.M)
    go(ctx, xb, b, 2)
    with pytest.raises(RcscmError) as ei:
        ctx.sync()
    assert ei.value.status == -5
    ctx.close()
    # b not in the null space of R'
    bb = b.clone().reshape(p.I, p.M)
    bb[1] = torch.tensor([1, 0, 0, 0], dtype=torch.complex128)
    ctx = Context.single(p.I, p.J, p.M)
    go(ctx, x, bb.reshape(-1), 1)
    with pytest.raises(RcscmError) as ei:
        ctx.sync()
    assert ei.value.status == -3 and "frequency 1" in str(ei.value)
    ctx.close()
    # a non-unit b is normalised, not an error
    ctx = Context.single(p.I, p.J, p.M)
    go(ctx, x, b * 3.0, 5)
    o3 = ctx.extract()
    ctx.sync()
    ctx.close()
    ref = oracle_accel(p, 5)
    assert_close({k: v.cpu().numpy().reshape(ref[k].shape) for k, v in o3.items()}, ref)


def test_objective_matches_oracle_and_decreases(c0):
    from oracle import accel as o_accel
    from oracle import objective as o_obj
    from paper_1908_01964_amd import Context, to_device
    sub = config(0, freqs=range(0, 257, 8))
    x, a, Rp, b = to_device(sub)
    ctx = Context.single(sub.I, sub.J, sub.M)
    ctx.init(x, a, Rp, b)
    vals = [ctx.objective()]
    st = o_accel.init_state(sub.I, sub.J)
    hist = o_accel.run(sub.x, sub.a, sub.Rp, sub.b, *st, 10, ALPHA, BETA, history=True)
    for k in range(10):
        ctx.iterate(1)
        vals.append(ctx.objective())
    ref = [o_obj.nlp(sub.x, sub.a, sub.Rp, sub.b, *h, ALPHA, BETA) for h in hist]
    for v, r in zip(vals, ref):
        assert abs(v - r) <= 1e-5 * abs(r) + 1e-3, (v, r)
    assert all(b2 <= a2 + 1e-6 * abs(a2) for a2, b2 in zip(vals, vals[1:]))
    ctx.close()


@pytest.mark.parametrize("fused", [True, False])
def test_config1_full_size_accel(fused):
    """Config 1 at full size (M=4, I=513, J=1000, K=20), every bin: the bench step (one fused
    rcscm_run) and the three-call path with the default schedule."""
    p = config(1)
    ref = oracle_accel(p, 20)
    if fused:  # as the bench times it: run-only context, autotuned class
        from paper_1908_01964_amd.autotune import best_run_classes
        out = gpu_run(p, 20, fused=True, run_only=True,
                      run_classes=best_run_classes(p.I, [p.J], [p.M], 20))[0]
    else:
        out = gpu_run(p, 20)[0]
    e = assert_close(out, ref, what=f"config 1 fused={fused}")
    print("config1 accel", fused, e)


def test_config1_full_size_naive_sampled_rows():
    """Naive rule at full config 1 size; rows are independent, so 24 sampled rows are exact."""
    p = config(1)
    out = gpu_run(p, 20, rule="naive")[0]
    sel = np.linspace(0, p.I - 1, 24).round().astype(int)
    sub = config(1, freqs=sel)
    ref = oracle_naive(sub, 20)
    got = {k: (v[sel] if v.ndim == 2 else v[sel]) for k, v in out.items()}
    assert_close(got, ref, what="config1 naive (sampled rows)")


def _gpu_run_fused(probs, K, **params):
    from helpers import split
    from paper_1908_01964_amd import Context, to_device
    probs = probs if isinstance(probs, list) else [probs]
    x, a, Rp, b = to_device(probs)
    I = probs[0].x.shape[0]
    Js = [p.x.shape[1] for p in probs]
    ctx = Context(I, Js, [p.x.shape[2] for p in probs], **params)
    out = ctx.run(x, a, Rp, b, K)
    ctx.sync()
    res = split({k: v.cpu().numpy() for k, v in out.items()}, I, Js)
    return res, ctx, (x, a, Rp, b)


@pytest.mark.parametrize("M,J", [(2, 1), (3, 250), (4, 1000), (5, 1025), (6, 2047), (8, 3000),
                                 (4, 8000)])
def test_fused_run_vs_oracle(M, J):
    p = make_problem(M, 3, J, config=450 + M, spatial="sinc" if M % 2 == 0 else "random",
                     n_fft=8)
    ref = oracle_accel(p, 12)
    out, ctx, _ = _gpu_run_fused(p, 12)
    ctx.close()
    assert_close(out[0], ref, what=f"fused M={M} J={J}")


@pytest.mark.parametrize("J", [256, 257, 512, 513, 1024, 1025, 2048, 2049, 4096, 4097, 8192])
def test_fused_run_class_boundaries(J):
    """Rows that exactly fill, or overflow by one frame, each workgroup class of the fused launch
    (256 x 1/2/4/8, 512 x 8, 1024 x 8): the last lane's last bin and the first padded one."""
    p = make_problem(2, 2, J, config=455, spatial="random")
    ref = oracle_accel(p, 6)
    out, ctx, _ = _gpu_run_fused(p, 6)
    ctx.close()
    assert_close(out[0], ref, what=f"fused J={J}")


@pytest.mark.parametrize("K", [1, 2, 3, 5, 20])
def test_fused_run_equals_separate_calls(c0, K):
    """Same per-bin code and reduction order as init + iterate + extract with 256-lane rows.  The
    fused launch runs its K iterations in four segments (its rows are all resident at once, so its
    waves step their priority down between segments), the RESIDENT kernel as one loop: K below 4
    and K not divisible by 4 leave segments empty or uneven."""
    out_f, ctx, _ = _gpu_run_fused(c0, K)
    ctx.close()
    out_s = gpu_run(c0, K, schedule="resident", block=256)
    for k in ("rh", "ru", "lam", "s_hat"):
        assert np.array_equal(out_f[0][k], out_s[0][k]), k


def test_fused_run_then_continue_and_objective():
    import torch
    p = make_problem(4, 5, 300, config=460, spatial="sinc", n_fft=16)
    out, ctx, inputs = _gpu_run_fused(p, 7)
    ctx.iterate(5)
    o2 = {k: v.cpu().numpy().reshape(-1) for k, v in ctx.extract().items()}
    nlp = ctx.objective()
    ctx.close()
    ref = oracle_accel(p, 12)
    assert_close({k: v.reshape(ref[k].shape) for k, v in o2.items()}, ref, what="run(7)+iterate(5)")
    from oracle import objective as o_obj
    r_nlp = o_obj.nlp(p.x, p.a, p.Rp, p.b, ref["rh"], ref["ru"], ref["lam"], ALPHA, BETA)
    assert abs(nlp - r_nlp) <= 1e-5 * abs(r_nlp) + 1e-3


def test_fused_run_ragged_batch():
    from synth import batch_utterance
    probs = [batch_utterance(u, I=9) for u in (4, 7, 16, 0)]  # J = 227, 336, 3888, 2199
    out, ctx, _ = _gpu_run_fused(probs, 20)
    ctx.close()
    for p, o in zip(probs, out):
        assert_close(o, oracle_accel(p, 20), what=f"ragged J={p.J} M={p.M}")


def _oracle_first(p, K):
    from oracle import accel as o_accel
    from oracle import extract as o_extract
    from oracle import first_stage
    st = o_accel.init_state(p.I, p.J)
    rh, ru, lam = first_stage.run(p.x, p.a, p.Rp, p.b, *st, K, ALPHA, BETA)
    return dict(rh=rh, ru=ru, lam=lam, s_hat=o_extract.s_hat(p.x, p.a, p.Rp, p.b, rh, ru, lam))


@pytest.mark.parametrize("M,J", [(2, 1), (3, 65), (4, 257), (5, 300), (6, 1001), (8, 129)])
def test_first_stage_rule_vs_oracle(M, J):
    p = make_problem(M, 3, J, config=440 + M, spatial="sinc" if M % 2 == 0 else "random",
                     n_fft=8)
    ref = _oracle_first(p, 10)
    out = gpu_run(p, 10, rule="first")[0]
    assert_close(out, ref, what=f"first-stage M={M} J={J}")


def test_first_stage_config1_sampled_rows():
    """Algorithm 1 at full config 1 size; 16 sampled rows against the FP64 first-stage oracle."""
    p = config(1)
    out = gpu_run(p, 20, rule="first")[0]
    sel = np.linspace(0, p.I - 1, 16).round().astype(int)
    ref = _oracle_first(config(1, freqs=sel), 20)
    got = {k: v[sel] for k, v in out.items()}
    assert_close(got, ref, what="config1 first-stage (sampled rows)")


def test_rows_longer_than_a_workgroup():
    """J = 9000 > 8192: AUTO falls back to STREAM, rcscm_run to the three calls; RESIDENT is refused."""
    from paper_1908_01964_amd import Context, RcscmError
    p = make_problem(2, 2, 9000, config=470, spatial="sinc", n_fft=4)
    ref = oracle_accel(p, 6)
    out = gpu_run(p, 6)[0]
    assert_close(out, ref, what="J=9000 auto")
    out = gpu_run(p, 6, fused=True)[0]
    assert_close(out, ref, what="J=9000 run")
    with pytest.raises(RcscmError):
        Context.single(p.I, p.J, p.M, schedule="resident")
