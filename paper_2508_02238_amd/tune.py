"""Tile-size autotuner for batched calls.

The integration tile size (256 to 2048 pixels) changes the results only to
rounding (N, P, T not at all), and the time: event-dense calls want many
small tiles (more workgroups), calls with few events per tile want large
ones (fewer chains of dependent memory accesses per call).  ``tune_tiles`` times batched calls on
throwaway states of the same sizes and parameters, over sample windows, and
picks a size per sensor size, one size class at a time (coordinate descent:
the other classes keep their current choice).  Results are cached per
workload key (the sensor-size mix and an event-rate bucket).
"""
from __future__ import annotations

import math

import torch

from . import Batch, State

CANDIDATES = (256, 512, 1024, 2048)
_cache: dict = {}


def workload_key(sizes, events_per_window) -> tuple:
    """Sensor-size mix and the rate bucket (powers of two of the mean events
    per stream and window)."""
    mix = tuple(sorted(set(sizes)))
    mean = max(1.0, sum(events_per_window) / max(1, len(events_per_window)))
    return mix, int(math.log2(mean))


def tune_tiles(sizes, params, windows, reps: int = 3, candidates=CANDIDATES) -> dict:
    """sizes: (W, H) per stream; params: esi params dict per stream (or one
    dict for all); windows: list of (events, t_frames) per sample window, with
    events a list of (x, y, t, p) device tensors per stream and t_frames a
    list of int64 device tensors (or None) per stream.  Returns
    {(W, H): tile_pixels}."""
    n = len(sizes)
    prms = params if isinstance(params, list) else [params] * n
    key = workload_key(sizes, [sum(int(e[2].numel()) for e in w[0]) / n for w in windows[:1]])
    if key in _cache:
        return dict(_cache[key])
    states = [State(w, h, **prms[i]) for i, (w, h) in enumerate(sizes)]
    batch = Batch(n)
    choice = {s: 0 for s in set(sizes)}

    def timed() -> float:
        for st, s in zip(states, sizes):
            st.set_tile_pixels(choice[s])
        best = float("inf")
        for _ in range(reps):
            for st in states:
                st.reset()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for evs, tfs in windows:
                batch.integrate(states, evs, tfs)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    base = timed()
    for s in sorted(choice, key=lambda s: -s[0] * s[1]):
        for c in candidates:
            if c == choice[s]:
                continue
            old = choice[s]
            choice[s] = c
            t = timed()
            if t < base:
                base = t
            else:
                choice[s] = old
    batch.close()
    for st in states:
        st.close()
    _cache[key] = dict(choice)
    return choice
