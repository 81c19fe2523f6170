"""Host logic of the autotuner (no GPU): cache keys, the (M, J-bucket) groups of a batch, the
candidate classes of a group, and that every cached run table holds only classes the fused
launch is instantiated for and covers every row of its shape."""
import json

import pytest

from paper_1908_01964_amd import autotune as T


def test_bucket_and_keys():
    assert [T._bucket(n) for n in (1, 2, 3, 1000, 1024, 1025)] == [1, 2, 4, 1024, 1024, 2048]
    assert T.run_cache_key(513, [1000], [4], 20) == "gfx950/run/M4/Jmax1024/rows513/K20"
    assert T.cache_key(513, [300, 2000], [6, 2], 20) == "gfx950/accel/M2-6/Jmax2048/rows1026/K20"


def test_run_groups_sum_frames_per_bucket_largest_first():
    Js, Ms = [300, 500, 1000, 3000, 9000], [2, 2, 4, 4, 4]
    g = T.run_groups(Js, Ms)
    assert g == [((4, 8192), 9000), ((4, 4096), 3000), ((4, 1024), 1000), ((2, 512), 800)]


@pytest.mark.parametrize("jm", [256, 512, 1024, 2048, 4096, 8192])
def test_run_candidates_hold_the_bucket(jm):
    c = T.run_candidates(jm)
    assert c, jm
    for nt, bpl in c:
        assert (nt, bpl) in T.FUSED_CLASSES
        assert jm <= nt * bpl <= max(4 * jm, 256)


def test_cached_run_tables_are_valid():
    with open(T.CACHE) as f:
        cache = json.load(f)
    runs = {k: v for k, v in cache.items() if "/run/" in k}
    assert runs, "no tuned run tables"
    for key, v in runs.items():
        for m, jm, nt, bpl in v["best"]:
            assert (nt, bpl) in T.FUSED_CLASSES, (key, nt, bpl)
            assert 2 <= m <= 8 and jm <= nt * bpl and jm <= T.MAX_FUSED_J, (key, m, jm)
        for t in v["timings_us"]:
            assert t["us"] > 0


def test_best_run_classes_reads_the_cache():
    t = T.best_run_classes(513, [1000], [4], 20)
    assert t is not None and all(len(e) == 4 for e in t)
    assert T.best_run_classes(7, [13], [3], 5) is None
