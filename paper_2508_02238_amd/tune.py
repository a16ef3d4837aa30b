"""Autotuner for batched calls: integration tile size, scan threshold and
chunk size.

Three schedule choices change the results only to rounding (N, P, T not at
all) and change the time:
  - the integration tile size (256 to 2048 pixels), per sensor size:
    event-dense calls want many small tiles (more workgroups), calls with few
    events per tile large ones (fewer chains of dependent memory accesses);
  - the scan threshold (esi_set_scan_run), per call: the run length above
    which a pixel's events go through its wave's scan of the per-event maps
    instead of one lane's loop (long runs: hot pixels, same-time bursts);
  - the chunk size of 512-pixel tiles (esi_set_chunk), per call: 1536
    records at four workgroups per CU or 2048 at three (tried only when some
    sensor size took 512-pixel tiles).
``tune`` times batched calls on throwaway states of the same sizes and
parameters over sample windows and picks them by coordinate descent (one
choice at a time; the others keep their current value).  Results are cached
per workload key: the sensor-size mix, the method parameters, and an
event-rate bucket.  The waves per workgroup of the kernels are compile-time
constants (they size LDS arrays and register budgets), and so are the other
tile sizes' chunks.
"""
from __future__ import annotations

import math

import torch

from . import Batch, State

TILE_CANDIDATES = (256, 512, 1024, 2048)
SCAN_CANDIDATES = (16, 32, 64, 128, 2**31 - 1)   # the last: serial loop only
CHUNK_CANDIDATES = (2048,)                        # besides the default
_cache: dict = {}


def _default_tile(w: int, h: int) -> int:
    """The library's default tile: the smallest that keeps a call within
    2000 tiles."""
    for tp in TILE_CANDIDATES:
        if -(-w * h // tp) <= 2000:
            return tp
    return TILE_CANDIDATES[-1]


def workload_key(sizes, events_per_window, params=None) -> tuple:
    """Sensor-size mix, method parameters (each distinct parameter set) and
    the rate bucket (powers of two of the mean events per stream and
    window)."""
    mix = tuple(sorted(set(sizes)))
    mean = max(1.0, sum(events_per_window) / max(1, len(events_per_window)))
    if params is None:
        return mix, int(math.log2(mean))
    plist = params if isinstance(params, list) else [params]
    methods = tuple(sorted({tuple(sorted(p.items())) for p in plist}))
    return mix, methods, int(math.log2(mean))


def tune(sizes, params, windows, reps: int = 3, tile_candidates=TILE_CANDIDATES,
         scan_candidates=SCAN_CANDIDATES, chunk_candidates=CHUNK_CANDIDATES) -> dict:
    """sizes: (W, H) per stream; params: esi params dict per stream (or one
    dict for all); windows: list of (events, t_frames) per sample window, with
    events a list of (x, y, t, p) device tensors per stream and t_frames a
    list of int64 device tensors (or None) per stream.  Returns
    {"tile_pixels": {(W, H): tile_pixels}, "scan_run": run, "chunk": records}
    (chunk 0: the library's default)."""
    n = len(sizes)
    prms = params if isinstance(params, list) else [params] * n
    key = (workload_key(sizes, [sum(int(e[2].numel()) for e in w[0]) / n for w in windows[:1]],
                        prms), tuple(tile_candidates), tuple(scan_candidates),
           tuple(chunk_candidates))
    if key in _cache:
        c = _cache[key]
        return {"tile_pixels": dict(c["tile_pixels"]), "scan_run": c["scan_run"],
                "chunk": c["chunk"]}
    states = [State(w, h, **prms[i]) for i, (w, h) in enumerate(sizes)]
    batch = Batch(n)
    tiles = {s: 0 for s in set(sizes)}
    scan = [0]   # 0: the library's default
    chunk = [0]  # likewise

    def timed() -> float:
        for st, s in zip(states, sizes):
            st.set_tile_pixels(tiles[s])
            st.set_scan_run(scan[0])
            st.set_chunk(chunk[0])
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
    for s in sorted(tiles, key=lambda s: -s[0] * s[1]):
        for c in tile_candidates:
            if c == tiles[s]:
                continue
            old = tiles[s]
            tiles[s] = c
            t = timed()
            if t < base:
                base = t
            else:
                tiles[s] = old
    for r in scan_candidates:
        old = scan[0]
        scan[0] = r
        t = timed()
        if t < base:
            base = t
        else:
            scan[0] = old
    if any((tp or _default_tile(w, h)) == 512 for (w, h), tp in tiles.items()):
        for c in chunk_candidates:
            old = chunk[0]
            chunk[0] = c
            t = timed()
            if t < base:
                base = t
            else:
                chunk[0] = old
    batch.close()
    for st in states:
        st.close()
    _cache[key] = {"tile_pixels": dict(tiles), "scan_run": scan[0], "chunk": chunk[0]}
    return {"tile_pixels": dict(tiles), "scan_run": scan[0], "chunk": chunk[0]}


def tune_tiles(sizes, params, windows, reps: int = 3, candidates=TILE_CANDIDATES) -> dict:
    """The tile sizes alone (scan threshold at the library's default)."""
    return tune(sizes, params, windows, reps, candidates, scan_candidates=(),
                chunk_candidates=())["tile_pixels"]
