"""Autotuner for the plain entry points.

Results never depend on the tuning: the cell occupancy, the smallest cell
edge and the choice between one target per wavefront and 64 targets per
wavefront change only speed (the GPU tests run every mode against the
oracle).  The tuner times a small grid of settings on the caller's own cloud
and queries with the library's stage events and keeps the fastest.  It runs
the library; it computes nothing itself.
"""
from __future__ import annotations

import itertools
import time

from . import Cloud, Workspace, count_targets, get_tuning, knn_rdf, set_tuning, trace_enable, trace_read

STAGES = ("binning", "pair", "tile", "nbr")

DEFAULT_GRID = {
    "tile_policy": (1, 2, 3, 4),
    "cell_occ": (2.0, 4.0, 8.0),
    "h_min_frac": (0.35, 0.5, 0.7),
    "tile_occ": (0.5, 1.0, 2.0),
    "rdf_kernel": (0,),
}


def autotune(cloud: Cloud, queries, d_srf: float = 0.0, k: int = 10, r_max: float = 2.0, n_bins: int = 200,
             grid: dict | None = None, reps: int = 3, ws: Workspace | None = None, apply: bool = True) -> dict:
    """Time knn_rdf over `queries` [(A, B), ...] for every combination of
    `grid` (keys: tile_policy, cell_occ, h_min_frac, tile_occ, rdf_kernel; a missing key keeps the
    current value) and keep the fastest, timed as the GPU time of the
    binning, pair and tile stages averaged over `reps` passes.

    Returns {"best": {...}, "ms": {setting: ms per pass}}; with apply=True the
    best setting becomes the process-wide tuning (set_tuning)."""
    import torch

    grid = dict(DEFAULT_GRID if grid is None else grid)
    ws = ws if ws is not None else Workspace()
    caps = [int(count_targets(cloud, A, d_srf, ws=ws).item()) for A, _ in queries]
    before = get_tuning()
    keys = ("tile_policy", "cell_occ", "h_min_frac", "tile_occ", "rdf_kernel")
    settings = []
    for st in itertools.product(*(grid.get(kk, (before[kk],)) for kk in keys)):
        # the cell occupancy of the mode not chosen does not matter
        if st[0] == 1:
            st = (st[0], st[1], st[2], before["tile_occ"], before["rdf_kernel"])
        elif st[0] in (2, 3):
            st = (st[0], before["cell_occ"], st[2], st[3], before["rdf_kernel"])
        if st not in settings:
            settings.append(st)
    times = {}

    def one_pass():
        for (A, B), cap in zip(queries, caps):
            knn_rdf(cloud, A, B, d_srf, k, r_max=r_max, n_bins=n_bins, capacity=cap, ws=ws)

    for stage in STAGES:
        trace_read(stage)
    try:
        for st in settings:
            set_tuning(*st)
            one_pass()                      # warm-up: workspace growth, first launches
            torch.cuda.synchronize()
            trace_enable(True)
            t0 = time.perf_counter()
            for _ in range(reps):
                one_pass()
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) * 1e3 / reps
            trace_enable(False)
            gpu = sum(trace_read(stage)[0] for stage in STAGES) / reps
            times[st] = gpu if gpu > 0 else wall
    finally:
        trace_enable(False)
    best = min(times, key=times.get)
    if apply:
        set_tuning(*best)
    else:
        set_tuning(*(before[kk] for kk in keys))
    return {"best": dict(zip(keys, best)), "ms": {str(dict(zip(keys, s))): v for s, v in times.items()}}
