"""Autotuner of the accelerated rule's launches, on synthetic data of the problem's shape.

Two tunings, both cached in ``tune_cache.json`` next to this file:

* ``tune`` - the K loop of ``iterate(K)``: for every candidate
    RESIDENT: block in {64, 128, 256, 512, 1024} (bins per lane follow from J)
    STREAM:   chunk in {256, 512, 1024, 2048} bins per workgroup (with hipGraph)
  keyed by architecture, the set of microphone counts, a power-of-two bucket of
  the longest row, the number of rows and K.
* ``tune_run`` - the workgroup class of ``run``'s fused launch (one workgroup
  per row: nt threads, bpl frames per lane; see rcscm_set_run_classes).  The
  rows are grouped by (M, power-of-two bucket of J); for each group, largest
  first, every instantiated class that holds the bucket is timed (the whole
  run, the other groups at their current choice) and the fastest kept.  The
  result is a class table (M, j_max, nt, bpl) for ``Context(run_classes=...)``,
  keyed like ``tune`` under "run".

    python -m paper_1908_01964_amd.autotune --I 513 --J 1000 --M 4 --K 20 [--run]
"""
from __future__ import annotations

import argparse
import json
import os
from typing import Sequence

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
ARCH = "gfx950"
RESIDENT_BLOCKS = (64, 128, 256, 512, 1024)
STREAM_CHUNKS = (256, 512, 1024, 2048)


def _bucket(n: int) -> int:
    b = 1
    while b < n:
        b <<= 1
    return b


def cache_key(I: int, Js: Sequence[int], Ms: Sequence[int], K: int) -> str:
    ms = "-".join(str(m) for m in sorted(set(Ms)))
    return f"{ARCH}/accel/M{ms}/Jmax{_bucket(max(Js))}/rows{I * len(Js)}/K{K}"


def load_cache() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def best_params(I: int, Js: Sequence[int], Ms: Sequence[int], K: int, tune_if_missing=False) -> dict:
    """Cached best schedule for this shape ({} if unknown and tune_if_missing is False)."""
    c = load_cache().get(cache_key(I, Js, Ms, K))
    if c is not None:
        return c["best"]
    if not tune_if_missing:
        return {}
    return tune(I, Js, Ms, K)["best"]


def _candidates(maxJ: int):
    if maxJ <= 8192:
        yield dict(schedule="resident", block=0, chunk=0)  # per-row workgroup sizes
    for b in RESIDENT_BLOCKS:
        cap = b * (8 if b == 1024 else 16)
        if maxJ <= cap:
            yield dict(schedule="resident", block=b, chunk=0)
    for c in STREAM_CHUNKS:
        yield dict(schedule="stream", block=0, chunk=c, graph=True)


def tune(I: int, Js: Sequence[int], Ms: Sequence[int], K: int, reps: int = 10,
         save: bool = True, inputs=None) -> dict:
    """Times every candidate on synthetic data of this shape; returns {'best', 'timings_us'}."""
    import torch

    from synth import make_problem

    from .rcscm import Context, to_device
    if inputs is None:
        probs = [make_problem(m, I, j, config=900, utterance=u, spatial="random",
                              with_truth=False) for u, (j, m) in enumerate(zip(Js, Ms))]
        inputs = to_device(probs)
    timings = []
    for cand in _candidates(max(Js)):
        ctx = Context(I, Js, Ms, **cand)
        ctx.init(*inputs)
        ctx.iterate(K)  # warm-up (and graph capture)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record()
        for r in range(reps):
            ctx.iterate(K)
            ev[r + 1].record()
        ctx.sync()
        us = min(ev[r].elapsed_time(ev[r + 1]) for r in range(reps)) * 1e3
        timings.append(dict(cand, us=us))
        ctx.close()
    best = min(timings, key=lambda t: t["us"])
    best_p = {k: v for k, v in best.items() if k != "us"}
    res = dict(best=best_p, timings_us=timings)
    if save:
        cache = load_cache()
        cache[cache_key(I, Js, Ms, K)] = res
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return res


# (threads per workgroup, frames per lane) pairs the fused launch is instantiated for
FUSED_CLASSES = ((256, 1), (256, 2), (256, 4), (256, 8), (512, 2), (512, 4), (512, 8),
                 (1024, 1), (1024, 2), (1024, 4), (1024, 8))
MAX_FUSED_J = 8192


def run_cache_key(I: int, Js: Sequence[int], Ms: Sequence[int], K: int) -> str:
    ms = "-".join(str(m) for m in sorted(set(Ms)))
    return f"{ARCH}/run/M{ms}/Jmax{_bucket(max(Js))}/rows{I * len(Js)}/K{K}"


def run_groups(Js: Sequence[int], Ms: Sequence[int]):
    """(M, j_max) groups of the rows, j_max the power-of-two bucket of J (at most 8192), with
    the frames each group holds per frequency; largest first."""
    g = {}
    for j, m in zip(Js, Ms):
        key = (int(m), min(_bucket(int(j)), MAX_FUSED_J))
        g[key] = g.get(key, 0) + int(j)
    return sorted(g.items(), key=lambda kv: -kv[1])


def run_candidates(j_max: int):
    """Classes that hold rows of j_max frames without more than 4x idle capacity."""
    return [c for c in FUSED_CLASSES if j_max <= c[0] * c[1] <= max(4 * j_max, 256)]


def best_run_classes(I: int, Js: Sequence[int], Ms: Sequence[int], K: int):
    """Cached class table for run() on this shape, or None."""
    c = load_cache().get(run_cache_key(I, Js, Ms, K))
    return None if c is None else [tuple(e) for e in c["best"]]


def _time_run(ctx, inputs, K, out, reps, torch):
    for _ in range(3):
        ctx.run(*inputs, K, out=out)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for r in range(reps):
        ctx.run(*inputs, K, out=out)
        ev[r + 1].record()
    torch.cuda.synchronize()
    t = sorted(ev[r].elapsed_time(ev[r + 1]) * 1e3 for r in range(reps))
    return t[len(t) // 2]


def tune_run(I: int, Js: Sequence[int], Ms: Sequence[int], K: int, reps: int = 30,
             save: bool = True, inputs=None) -> dict:
    """Chooses the fused launch's class per (M, J bucket) group by timing run(); returns
    {'best': table, 'timings_us': [...]}.  Only for shapes whose rows all fit one workgroup."""
    import torch

    from synth import make_problem

    from .rcscm import Context, to_device
    if max(Js) > MAX_FUSED_J:
        raise ValueError("run() makes no fused launch for rows longer than 8192 frames")
    if inputs is None:
        probs = [make_problem(m, I, j, config=900, utterance=u, spatial="random",
                              with_truth=False) for u, (j, m) in enumerate(zip(Js, Ms))]
        inputs = to_device(probs)
    nbins = I * sum(Js)
    dev = inputs[0].device
    out = dict(rh=torch.empty(nbins, dtype=torch.float32, device=dev),
               ru=torch.empty(nbins, dtype=torch.float32, device=dev),
               lam=torch.empty(I * len(Js), dtype=torch.float32, device=dev),
               s_hat=torch.empty(nbins, dtype=torch.complex64, device=dev))
    choice = {}
    timings = []

    def table(ch):
        return [(m, jm, nt, bpl) for (m, jm), (nt, bpl) in sorted(ch.items())]
    # About 0.1 s of back-to-back calls first, so the first candidates are not timed while the
    # GPU is still raising its clock.
    ctx = Context(I, Js, Ms, run_only=True)
    per = _time_run(ctx, inputs, K, out, 3, torch) * 1e-6
    for _ in range(int(min(5000, max(10, 0.1 / max(per, 1e-6))))):
        ctx.run(*inputs, K, out=out)
    torch.cuda.synchronize()
    ctx.sync()
    ctx.close()
    for (m, jm), _ in run_groups(Js, Ms):
        best = None
        for cand in run_candidates(jm):
            trial = dict(choice)
            trial[(m, jm)] = cand
            ctx = Context(I, Js, Ms, run_only=True, run_classes=table(trial))
            us = _time_run(ctx, inputs, K, out, reps, torch)
            ctx.sync()
            ctx.close()
            timings.append(dict(M=m, j_max=jm, nt=cand[0], bpl=cand[1], us=us))
            if best is None or us < best[1]:
                best = (cand, us)
        choice[(m, jm)] = best[0]
    res = dict(best=table(choice), timings_us=timings)
    if save:
        cache = load_cache()
        cache[run_cache_key(I, Js, Ms, K)] = res
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--I", type=int, default=513)
    ap.add_argument("--J", type=int, nargs="+", default=[1000])
    ap.add_argument("--M", type=int, nargs="+", default=[4])
    ap.add_argument("--K", type=int, default=20)
    ap.add_argument("--run", action="store_true", help="tune run()'s fused classes instead")
    ap.add_argument("--workload", type=int, default=0,
                    help="tune on a named workload's own shapes (2 = the ragged batch)")
    ap.add_argument("--out", default=None, help="also write the result (with its key) here")
    a = ap.parse_args()
    if a.workload == 2:
        from synth import batch_shapes
        Js, Ms = batch_shapes()
        I, K = 513, 20
    else:
        Js = a.J
        Ms = a.M if len(a.M) == len(a.J) else a.M * len(a.J)
        I, K = a.I, a.K
    if a.run:
        r = tune_run(I, Js, Ms, K)
        key = run_cache_key(I, Js, Ms, K)
    else:
        r = tune(I, Js, Ms, K)
        key = cache_key(I, Js, Ms, K)
    print(json.dumps(r, indent=1))
    if a.out:
        with open(a.out, "w") as f:
            json.dump({key: r}, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
