"""Phase A's wave scan of the per-event clamp-affine maps against the FP64
oracle, through the C ABI.

The scan takes the runs of a chunk longer than the state's scan_run
(esi_set_scan_run): forcing scan_run down to 1 sends nearly every run through
it, so these cases run the scan over every decay kind, both orders of add
and decay, active clamps (the composed bounds), same-time bursts with mixed
polarity, runs that cross chunk and frame-segment bounds, all tile sizes,
split calls and the batched call.  N, P, T bit-exact; S and frames within
the tolerance of the serial loop.
"""
from __future__ import annotations

import numpy as np
import pytest

import evgen
from esi_parity import assert_frames, assert_state, assert_u8, gpu_run, oracle_run

pytestmark = pytest.mark.gpu

DEFAULT = dict(C=0.2, k_per_us=2e-6, b=2.0, s_min=-1.0, s_max=1.0)
SCAN_OFF = 2**31 - 1


@pytest.fixture(scope="module")
def esi():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2508_02238_amd as m
    return m


def _check(esi, s, prm, tf, scan_run, calls=None, u8=False, where="", tile=None, chunk=0):
    if tile is None:
        fg, ug, stg, diag = gpu_run(esi, s, prm, t_frames=tf, calls=calls, want_u8=u8,
                                    scan_run=scan_run)
    else:
        fg, ug, stg, diag = _run_tile(esi, s, prm, tf, scan_run, tile, chunk)
    fo, o = oracle_run(s, prm, t_frames=tf)
    where = f"{where} scan_run={scan_run}"
    assert_state(stg, o, prm["C"], where)
    assert diag["dropped"] == o.dropped
    assert diag["flags"] & 8 == 0, where  # no internal flag
    assert_frames(fg, fo, prm, where)
    if u8:
        assert_u8(ug, fo, prm, where)


def _run_tile(esi, s, prm, tf, scan_run, tile, chunk=0):
    import torch
    st = esi.State(s.width, s.height, **prm)
    st.set_tile_pixels(tile)
    st.set_scan_run(scan_run)
    if chunk:
        st.set_chunk(chunk)
    fr, _ = st.integrate(s.x, s.y, s.t, s.p, t_frames=tf)
    torch.cuda.synchronize()
    S, T, N, P = (a.cpu().numpy() for a in st.read_state())
    out = (fr.cpu().numpy(), None, (S, T, N.view(np.uint32), P), st.diagnostics())
    st.close()
    return out


PARAMS = [
    ("pow b=2", DEFAULT),
    ("b=1", dict(C=0.2, k_per_us=1e-4, b=1.0, s_min=-1.0, s_max=1.0)),
    ("b=0.5 clamps", dict(C=0.25, k_per_us=2e-5, b=0.5, s_min=-0.3, s_max=0.7)),
    ("b=4.7", dict(C=0.2, k_per_us=1e-5, b=4.7, s_min=-1e30, s_max=1e30)),
    ("decay then add", dict(C=0.2, k_per_us=2e-5, b=2.0, s_min=-0.5, s_max=0.9, flags=1)),
    ("exp", dict(C=0.2, k_per_us=3e-5, b=2.0, s_min=-1.0, s_max=1.0, flags=4)),
    ("exp decay then add", dict(C=0.15, k_per_us=3e-5, b=2.0, s_min=-0.4, s_max=0.6, flags=5)),
    ("k=0", dict(C=0.25, k_per_us=0.0, b=2.0, s_min=-1e30, s_max=1e30)),
    ("lazy", dict(C=0.2, k_per_us=2e-5, b=2.0, s_min=-1.0, s_max=1.0, flags=2)),
]


@pytest.mark.parametrize("scan_run", [1, 5])
@pytest.mark.parametrize("name,prm", PARAMS, ids=[p[0] for p in PARAMS])
def test_scan_dense_runs(esi, name, prm, scan_run):
    """A small sensor with many events per pixel and same-time bursts: runs
    of tens to hundreds of events per chunk, frames inside the runs."""
    s = evgen.random_stream(seed=101, width=40, height=9, n=120_000, t_max=300_000,
                            burst_frac=0.3, oob_frac=0.01)
    tf = np.sort(np.random.default_rng(5).integers(0, 300_000, 37)).astype(np.int64)
    _check(esi, s, prm, tf, scan_run, u8=True, where=name)


@pytest.mark.parametrize("scan_run", [1, 64, SCAN_OFF])
def test_scan_hot_pixels(esi, scan_run):
    """Hot pixels (runs of thousands of events per chunk, over many chunks)
    with the scan at every run, at the default threshold, and off."""
    s = evgen.hot_pixel_stream(seed=6, width=64, height=48, n_bg=50_000, t_max=1_000_000,
                               hot=[(3, 4), (40, 47), (63, 0)], hot_period_us=20)
    tf = np.array([1, 250_000, 500_000, 500_010, 999_999, 1_000_000], np.int64)
    for prm in (DEFAULT, dict(C=0.2, k_per_us=2e-6, b=2.0, s_min=-1e30, s_max=1e30),
                dict(C=0.2, k_per_us=0.0, b=2.0, s_min=-3.0, s_max=1e30)):
        _check(esi, s, prm, tf, scan_run, where="hot")


@pytest.mark.parametrize("scan_run", [1, 3])
def test_scan_bursts_clamped(esi, scan_run):
    """Thousands of events of one pixel at one time with mixed polarity:
    the per-event clamp makes their order matter, so the composed bounds
    decide the result."""
    rng = np.random.default_rng(9)
    n = 30_000
    x = rng.integers(0, 3, n).astype(np.uint16)
    y = np.zeros(n, np.uint16)
    t = np.sort(rng.integers(0, 40, n)).astype(np.int64) * 1000
    p = rng.choice(np.array([-1, 1], np.int8), n)
    s = evgen.Stream(x, y, t, p, 3, 1, 40_000)
    for prm in (dict(C=0.25, k_per_us=0.0, b=1.0, s_min=-0.5, s_max=0.75),
                dict(C=0.25, k_per_us=3e-5, b=2.0, s_min=-0.5, s_max=0.75),
                dict(C=0.25, k_per_us=3e-5, b=2.0, s_min=-0.5, s_max=0.75, flags=1)):
        _check(esi, s, prm, np.arange(0, 41, dtype=np.int64) * 1000, scan_run, where="bursts")


@pytest.mark.parametrize("tile", [256, 512, 1024, 2048])
def test_scan_tile_sizes(esi, tile):
    """Every tile size (1, 2, 4 and 8 pixels per thread) with the scan forced."""
    s = evgen.random_stream(seed=17, width=333, height=29, n=400_000, t_max=200_000,
                            burst_frac=0.25)
    tf = np.linspace(1_000, 200_000, 23).astype(np.int64)
    _check(esi, s, DEFAULT, tf, 2, where=f"tile {tile}", tile=tile)


@pytest.mark.parametrize("scan_run", [1, 64, SCAN_OFF])
@pytest.mark.parametrize("name,prm", [PARAMS[0], PARAMS[2], PARAMS[5]],
                         ids=[PARAMS[0][0], PARAMS[2][0], PARAMS[5][0]])
def test_big_chunks(esi, name, prm, scan_run):
    """2048-record chunks at three workgroups per CU (esi_set_chunk) on
    512-pixel tiles: uniform events, same-time bursts and hot pixels whose
    runs cross chunk and frame-segment bounds, with the scan forced, at its
    default threshold and off."""
    s = evgen.random_stream(seed=31, width=333, height=29, n=400_000, t_max=300_000,
                            burst_frac=0.25)
    rng = np.random.default_rng(5)
    hot = rng.random(s.n) < 0.2
    s.x[hot] = rng.choice(np.array([3, 200, 331], np.uint16), int(hot.sum()))
    s.y[hot] = 7
    tf = np.concatenate([np.linspace(1_000, 300_000, 40), [299_999, 5_000_000]]).astype(np.int64)
    tf.sort()
    _check(esi, s, prm, tf, scan_run, where=f"chunk 2048 {name}", tile=512, chunk=2048)


def test_chunk_argument(esi):
    st = esi.State(8, 8, **DEFAULT)
    for bad in (-1, 1, 1024, 4096):
        assert esi.esi_set_chunk(st.handle, bad) == esi.ESI_ERR_INVALID_ARG
    for good in (0, 1536, 2048):
        assert esi.esi_set_chunk(st.handle, good) == esi.ESI_OK
    st.close()


def test_scan_split_calls_and_long_gaps(esi):
    """Runs across calls, and frames far apart (one-frame segments)."""
    s = evgen.random_stream(seed=23, width=50, height=20, n=150_000, t_max=400_000,
                            burst_frac=0.2)
    tf = np.array([10_000, 200_000, 200_001, 399_999, 400_000_000_000], np.int64)
    cuts = [0, 40_000, 40_001, 120_000, s.n]
    calls = list(zip(cuts[:-1], cuts[1:]))
    _check(esi, s, DEFAULT, tf, 1, calls=calls, where="split")
    prm = dict(C=0.2, k_per_us=1e-3, b=2.0, s_min=-1.0, s_max=1.0, flags=4)
    _check(esi, s, prm, tf, 2, where="exp long gaps")


def test_scan_batched(esi):
    """The batched call takes each state's scan_run: streams with the scan
    forced and off in one call, each against the oracle."""
    import torch
    streams = [evgen.random_stream(seed=200 + i, width=w, height=h, n=n, t_max=50_000,
                                   burst_frac=0.2)
               for i, (w, h, n) in enumerate([(30, 10, 60_000), (90, 40, 100_000),
                                               (17, 3, 20_000), (300, 100, 200_000)])]
    runs = [1, SCAN_OFF, 2, 64]
    states = [esi.State(s.width, s.height, **DEFAULT) for s in streams]
    for st, r in zip(states, runs):
        st.set_scan_run(r)
    batch = esi.Batch(len(streams))
    tf = np.array([25_000, 50_000], np.int64)
    outs = batch.integrate(states, [(s.x, s.y, s.t, s.p) for s in streams],
                           [tf] * len(streams))
    torch.cuda.synchronize()
    for i, s in enumerate(streams):
        fo, o = oracle_run(s, DEFAULT, t_frames=tf)
        S, T, N, P = (a.cpu().numpy() for a in states[i].read_state())
        assert_state((S, T, N.view(np.uint32), P), o, DEFAULT["C"], f"batch {i}")
        assert_frames(outs[i][0].cpu().numpy(), fo, DEFAULT, f"batch {i}")
    batch.close()
    for st in states:
        st.close()


def test_scan_run_argument(esi):
    st = esi.State(8, 8, **DEFAULT)
    assert esi.esi_set_scan_run(st.handle, -1) == esi.ESI_ERR_INVALID_ARG
    assert esi.esi_set_scan_run(None, 4) == esi.ESI_ERR_INVALID_ARG
    assert esi.esi_set_scan_run(st.handle, 0) == esi.ESI_OK
    st.close()
