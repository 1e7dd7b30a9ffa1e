"""The stored scan-point counts of the headline workload's 26 views are the
oracle's: rows stored beside the per-view totals are recomputed here with
the oracle and compared exactly."""

import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "pic3_256_1080p_view_samples.json")


def test_stored_view_counts_match_the_oracle():
    import oracle
    from scenes import configs
    ref = json.load(open(GOLDEN))
    views = configs.views26()
    assert [tuple(v) for v in ref["views"]] == [tuple(v) for v in views]
    assert len(ref["samples"]) == 26 and len(ref["row_samples"]) == 26
    sc = configs.pic3(n=256, width=1920, height=1080)
    for k in (0, 12, 25):                              # a diagonal, an axis and the opposite diagonal
        scene = sc.with_(camera=configs.orbit_camera(sc.dims, views[k]))
        for r, want in zip(ref["check_rows"], ref["row_samples"][k]):
            px = np.stack([np.arange(sc.width), np.full(sc.width, r)], axis=-1)
            got = int(oracle.render_pixels(scene, px)["samples"].sum())
            assert got == want, (k, r)
    # totals are consistent with the stored rows and with a frame's pixel count
    for k in range(26):
        assert sum(ref["row_samples"][k]) <= ref["samples"][k]
        assert 0 < ref["hit_pixels"][k] <= 1920 * 1080
