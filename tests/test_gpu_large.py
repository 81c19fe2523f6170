"""Full-size GPU runs of the ragged batch (64 utterances) and the large instance (M=8, I=1025,
J=8000, K=30), checked on sampled rows against the FP64 oracle (rows are independent, so a
regenerated row is an exact reference), plus properties that hold at any size."""
import numpy as np
import pytest

from helpers import TOL, assert_close, errors, gpu_run, nrel, oracle_accel
from synth import batch_shapes, batch_utterance, config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    Js, Ms = batch_shapes()
    probs = [batch_utterance(u) for u in range(len(Js))]
    return Js, Ms, probs


def _sample_rows(Js, n=16, seed=0):
    rng = np.random.default_rng(seed)
    us = rng.integers(0, len(Js), n)
    iis = rng.integers(0, 513, n)
    return list(zip(us.tolist(), iis.tolist()))


@pytest.mark.parametrize("schedule", ["resident", "stream", "fused"])
def test_config2_full_batch_sampled_rows(batch, schedule):
    Js, Ms, probs = batch
    K = 20
    if schedule == "fused":
        # the bench step: rcscm_run on a run-only context with the autotuned classes, one launch
        # per class, the classes spread over the library's streams
        from paper_1908_01964_amd.autotune import best_run_classes
        outs = gpu_run(probs, K, fused=True, run_only=True,
                       run_classes=best_run_classes(513, Js, Ms, K))
    else:
        outs = gpu_run(probs, K, schedule=schedule)
    got = {k: [] for k in ("rh", "ru", "lam", "s_hat")}
    ref = {k: [] for k in got}
    for u, i in _sample_rows(Js):
        p = batch_utterance(u, freqs=[i])
        r = oracle_accel(p, K)
        for k in got:
            got[k].append(np.atleast_1d(outs[u][k][i]).ravel())
            ref[k].append(np.atleast_1d(r[k][0]).ravel())
    g = {k: np.concatenate(v) for k, v in got.items()}
    rr = {k: np.concatenate(v) for k, v in ref.items()}
    e = assert_close(g, rr, what=f"config 2 {schedule}")
    print("config2", schedule, e)
    for o in outs:
        assert np.all(np.isfinite(o["rh"])) and np.all(o["ru"] > 0) and np.all(o["lam"] > 0)


def test_config2_batch_equals_single_runs(batch):
    Js, Ms, probs = batch
    K = 20
    outs = gpu_run(probs, K, schedule="resident", block=256)
    for u in (0, 17, 63):
        single = gpu_run(probs[u], K, schedule="resident", block=256)[0]
        for k in ("rh", "ru", "lam", "s_hat"):
            assert np.array_equal(single[k], outs[u][k]), (u, k)


def test_config2_fused_batch_equals_single_runs(batch):
    """rcscm_run over the batch (ten classes on several streams: no priority steps) against the
    same utterances run alone (one 256-lane class holding all its rows at once: priority steps
    on; or a 512-lane one: off): the same class kernel, so the results are equal bitwise."""
    Js, Ms, probs = batch
    K = 20
    outs = gpu_run(probs, K, fused=True)
    short = [u for u in range(len(Js)) if Js[u] <= 2048][:3]
    long_ = [u for u in range(len(Js)) if Js[u] > 2048][:1]
    for u in short + long_:
        single = gpu_run(probs[u], K, fused=True)[0]
        for k in ("rh", "ru", "lam", "s_hat"):
            assert np.array_equal(single[k], outs[u][k]), (u, Js[u], k)


def test_config4_full_size_subsample():
    """M=8, I=1025, J=8000, K=30; the FP64 oracle checks 64 frequencies incl. DC and Nyquist."""
    p = config(4)
    K = p.meta["K"]
    sel = np.round(np.linspace(0, p.I - 1, 64)).astype(int)
    sub = config(4, freqs=sel)
    ref = oracle_accel(sub, K)
    for schedule in ("resident", "stream", "fused"):
        if schedule == "fused":  # the bench step: accel_fused_kernel<8, 1024, 8>, run-only
            out = gpu_run(p, K, fused=True, run_only=True)[0]
        else:
            out = gpu_run(p, K, schedule=schedule)[0]
        got = {k: v[sel] for k, v in out.items()}
        e = assert_close(got, ref, what=f"config 4 {schedule}")
        print("config4", schedule, e)
