"""Helpers comparing GPU images with the FP64 oracle.

Tolerance: every channel of every pixel within 2e-3 of the oracle, plus the
oracle's per-pixel allowance for decisions (nearest cell, clip plane, box
exit, termination threshold, iso crossing) taken within the decision margin, where both
outcomes are correct.  Sample counts must match exactly wherever the oracle
flagged no such decision.
"""

from __future__ import annotations

import sys

import numpy as np

from oracle.oracle import FLAG_ERT, FLAG_ISO, FLAG_NEAREST

TOL = 2e-3


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare(gpu_rgba: np.ndarray, gpu_cnt, rec: np.ndarray, tol: float = TOL, label: str = "",
            check_counts: bool = True) -> dict:
    """gpu_rgba: (n,4) float32; gpu_cnt: (n,) int or None; rec: oracle records for the same pixels."""
    g = np.asarray(gpu_rgba, dtype=np.float64).reshape(-1, 4)
    o = rec["rgba"].reshape(-1, 4)
    assert np.all(np.isfinite(g)), f"{label}: non-finite GPU pixels"
    diff = np.abs(g - o)
    bound = tol + rec["allowance"][:, None]
    bad = diff > bound
    flagged = rec["flags"] > 0
    stats = dict(label=label, pixels=int(g.shape[0]), max_diff=float(diff.max()) if diff.size else 0.0,
                 max_diff_unflagged=float(diff[~flagged].max()) if (~flagged).any() else 0.0,
                 flagged_pixels=int(flagged.sum()),
                 unconstrained_pixels=int((rec["allowance"] >= 1.0).sum()),
                 max_allowance_used=float(np.max(np.where(flagged[:, None], diff, 0.0))) if diff.size else 0.0,
                 samples=int(rec["samples"].sum()))
    if bad.any():
        idx = np.argwhere(bad.any(axis=1))[:5, 0]
        details = [(int(i), g[i].tolist(), o[i].tolist(), float(rec["allowance"][i]), int(rec["flags"][i]),
                    int(rec["samples"][i]), (int(gpu_cnt[i]) if gpu_cnt is not None else None)) for i in idx]
        raise AssertionError(f"{label}: {int(bad.any(axis=1).sum())} pixels outside tolerance; first: {details}")
    if check_counts and gpu_cnt is not None:
        # counts move only with clip-plane and box-exit decisions, unless a nearest-cell,
        # termination or iso-crossing decision changed where the ray stops
        c = np.asarray(gpu_cnt).reshape(-1).astype(np.int64)
        free = (rec["kinds"] & (FLAG_NEAREST | FLAG_ERT | FLAG_ISO)) != 0
        mism = (np.abs(c - rec["samples"]) > rec["count_slack"]) & ~free
        assert not mism.any(), (f"{label}: sample counts differ at {int(mism.sum())} pixels, e.g. "
                                f"{[(int(i), int(c[i]), int(rec['samples'][i])) for i in np.argwhere(mism)[:5, 0]]}")
        stats["counts_checked"] = int((~free).sum())
        stats["count_differences"] = int((c != rec["samples"]).sum())
    log("parity", stats)
    return stats


def pixel_list(h: int, w: int, n_random: int, rng, extra_rows=(), extra_cols=(), hit_mask=None, n_hit=0):
    """(col,row) pairs: random pixels, random pixels inside hit_mask, and whole rows/columns."""
    px = set()
    for _ in range(n_random):
        px.add((int(rng.integers(0, w)), int(rng.integers(0, h))))
    if hit_mask is not None and n_hit:
        rows, cols = np.nonzero(hit_mask)
        if rows.size:
            sel = rng.choice(rows.size, size=min(n_hit, rows.size), replace=False)
            for k in sel:
                px.add((int(cols[k]), int(rows[k])))
    for r in extra_rows:
        for i in range(w):
            px.add((i, int(r)))
    for c in extra_cols:
        for j in range(h):
            px.add((int(c), j))
    return np.array(sorted(px, key=lambda t: (t[1], t[0])), dtype=np.int32)
