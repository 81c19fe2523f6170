"""Autotuner of the accelerated K loop: schedule, workgroup size and chunk size.

For a problem shape it times ``iterate(K)`` for every candidate
  RESIDENT: block in {64, 128, 256, 512, 1024} (bins per lane follow from J)
  STREAM:   chunk in {256, 512, 1024, 2048} bins per workgroup (with hipGraph)
on synthetic data of that shape and keeps the fastest.  Results are cached in
``tune_cache.json`` next to this file, keyed by architecture, rule, the set
of microphone counts, a power-of-two bucket of the longest row, the number of
rows and K.

    python -m paper_1908_01964_amd.autotune --I 513 --J 1000 --M 4 --K 20
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--I", type=int, default=513)
    ap.add_argument("--J", type=int, nargs="+", default=[1000])
    ap.add_argument("--M", type=int, nargs="+", default=[4])
    ap.add_argument("--K", type=int, default=20)
    a = ap.parse_args()
    Ms = a.M if len(a.M) == len(a.J) else a.M * len(a.J)
    r = tune(a.I, a.J, Ms, a.K)
    print(json.dumps(r, indent=1))


if __name__ == "__main__":
    main()
