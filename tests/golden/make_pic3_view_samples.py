"""Writes pic3_256_1080p_view_samples.json: the oracle's exact scan-point counts
of the three-source 256^3 workload at 1920x1080 for each of the 26 views.

    python tests/golden/make_pic3_view_samples.py [--threads N]

A scan point counts once where the active sources are composited: after the
clipping planes and up to early termination (the counting convention of the
sample-throughput metric).  The counts come from the FP64 oracle alone (every
pixel of every view), with the per-view sums of the oracle's count slack (scan
points within their margin of a clip plane or the box exit, which an FP32
renderer may keep or drop) and of flagged pixels, so that a GPU count can be
checked against them.  Takes a few minutes on 8 host threads.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "pic3_256_1080p_view_samples.json")
CHECK_ROWS = (270, 540, 810)      # rows whose per-view sums are stored too, so a test can recompute them


def main():
    import numpy as np

    import oracle
    from scenes import configs
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()
    sc = configs.pic3(n=256, width=1920, height=1080)
    views = configs.views26()
    res = dict(workload="pic3: density+E+B 256^3, 1 guard layer, trilinear, step 0.5, 2 clip planes, 1920x1080",
               storage="f32", views=[list(v) for v in views], samples=[], count_slack=[], flagged_pixels=[],
               hit_pixels=[], check_rows=list(CHECK_ROWS), row_samples=[])
    t0 = time.time()
    for k, v in enumerate(views):
        rec = oracle.render(sc.with_(camera=configs.orbit_camera(sc.dims, v)), threads=args.threads)
        res["samples"].append(int(rec["samples"].sum()))
        res["count_slack"].append(int(rec["count_slack"].sum()))
        res["flagged_pixels"].append(int((rec["flags"] > 0).sum()))
        res["hit_pixels"].append(int((rec["samples"] > 0).sum()))
        per_row = rec["samples"].reshape(sc.height, sc.width).sum(axis=1)
        res["row_samples"].append([int(per_row[r]) for r in CHECK_ROWS])
        print(f"view {k} {v}: {res['samples'][-1]} samples, slack {res['count_slack'][-1]}, "
              f"{time.time() - t0:.0f} s", flush=True)
    res["mean_samples"] = float(np.mean(res["samples"]))
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")
    print("wrote", args.out)


if __name__ == "__main__":
    main()
