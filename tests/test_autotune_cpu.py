"""Host logic of the autotuner: the candidate set obeys the library's tile-shape
rules (the same ones isaac_set_tile_shape enforces), size classes, cache
round trip and the tie rule of the pick."""

import itertools

from paper_1611_09048_amd import autotune


def valid(c):
    w, x, u, g, m, p = c
    return (g in (1, 2, 4, 8, 16, 32, 64) and 1 <= w <= 64 // g and (w & (w - 1)) == 0 and x in (1, 2, 4)
            and u in (1, 2)
            and (g == 1 or u == 1) and m in (0, 4) and not (m and (g == 2 or g >= 32 or u == 2))
            and p in (0, 1) and (p == 0 or (2 <= g <= 16 and u == 1)))


def test_candidates_are_valid_and_unique():
    cands = autotune.candidates()
    assert len(cands) == len(set(cands)) > 20
    assert all(valid(c) for c in cands)
    assert autotune.DEFAULT in cands or valid(autotune.DEFAULT)
    # restricting the axes restricts the set
    sub = autotune.candidates(unrolls=(1,), lanes=(4, 16), pooled=(0,))
    assert set(sub) <= set(cands) and all(c[3] in (4, 16) and c[5] == 0 for c in sub)


def test_every_lane_count_has_a_full_wave_shape():
    cands = autotune.candidates(pooled=(0,))
    for g in autotune.LANES:
        assert any(c[3] == g and c[0] == 64 // g for c in cands), g


def test_size_classes():
    assert autotune.size_class(1, 1) == 0
    assert autotune.size_class(1920, 1080) == 11
    assert autotune.size_class(2048, 16) == 11
    assert autotune.size_class(2049, 16) == 12
    assert autotune.size_class(1 << 20, 8) == 15


def test_cache_round_trip_and_pick(tmp_path):
    path = str(tmp_path / "tuned.json")
    assert autotune.load_cache(path) == {}
    table = {autotune.cache_key("gfx950", 11, "tri:f32x1"): [4, 2, 1, 16, 4, 0]}
    autotune.save_cache(path, table)
    assert autotune.load_cache(path) == table
    times = {(8, 2, 1, 1, 0, 0): 0.5, (4, 1, 1, 16, 4, 0): 0.2, (4, 2, 1, 16, 4, 0): 0.2}
    assert autotune.pick(times) == (4, 1, 1, 16, 4, 0)       # ties go to the smaller shape
    for a, b in itertools.combinations(sorted(times), 2):
        assert a < b


class _FakeCtx:
    def __init__(self):
        self.shapes = {}

    def set_tile_shape(self, cls, *shape):
        self.shapes[cls] = tuple(shape)


def test_per_class_refinement_keeps_the_launch_variant_and_caches():
    """Each class takes the tile shape that times fastest with the others fixed; the
    kernel variant (unroll, lanes, min_waves, schedule) stays the shared one."""
    ctx = _FakeCtx()
    base = (8, 2, 1, 4, 0, 1)
    best = {7: (16, 1), 8: (8, 4), 9: (16, 4), 10: (8, 2)}

    def time_batch():
        return sum(0.0 if ctx.shapes[c][:2] == best[c] else 1.0 + 0.01 * ctx.shapes[c][0] for c in best)

    cache = {}
    got = autotune.refine_per_class(ctx, sorted(best), base, time_batch, cache=cache, sig="b:class")
    for c, (w, x) in best.items():
        assert got[c] == (w, x) + base[2:] and ctx.shapes[c] == got[c]
        assert cache[autotune.cache_key("gfx950", c, "b:class")] == list(got[c])
    # a second run takes the cache and times nothing
    ctx2 = _FakeCtx()
    got2 = autotune.refine_per_class(ctx2, sorted(best), base, lambda: 1 / 0, cache=cache, sig="b:class")
    assert got2 == got and ctx2.shapes == ctx.shapes
    assert all(s in autotune.class_shapes(4) for s in best.values())
