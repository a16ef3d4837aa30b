"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Sizes run from tiny sensors (brute force) to the full workloads (sampled
frames), including ragged tiles, chunk boundaries inside one pixel's run,
same-time bursts, hot pixels, empty and degenerate calls.
"""
from __future__ import annotations

import numpy as np
import pytest

import evgen
import oracle
from esi_parity import (assert_frames, assert_state, assert_u8, gpu_run, oracle_run)

pytestmark = pytest.mark.gpu

DEFAULT = dict(C=0.2, k_per_us=2e-6, b=2.0, s_min=-1.0, s_max=1.0)


@pytest.fixture(scope="module")
def esi():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2508_02238_amd as m
    return m


def _check(esi, s, prm, tf=None, calls=None, u8=False, where=""):
    fg, ug, stg, diag = gpu_run(esi, s, prm, t_frames=tf, calls=calls, want_u8=u8)
    fo, o = oracle_run(s, prm, t_frames=tf)
    assert_state(stg, o, prm["C"], where)
    assert diag["dropped"] == o.dropped, (diag, o.dropped)
    assert bool(diag["flags"] & 1) == o.unsorted
    if tf is not None and len(tf):
        assert_frames(fg, fo, prm, where)
        if u8:
            assert_u8(ug, fo, prm, where)
    return fg, stg, diag, o


PARAM_SWEEP = [
    dict(C=0.2, k_per_us=0.0, b=2.0, s_min=-1e30, s_max=1e30),
    dict(C=0.25, k_per_us=1e-7, b=0.5, s_min=-1.0, s_max=1.0),
    dict(C=0.2, k_per_us=2e-6, b=2.0, s_min=-1.0, s_max=1.0),
    dict(C=0.15, k_per_us=1e-4, b=4.7, s_min=-0.3, s_max=0.7),
    dict(C=0.2, k_per_us=2e-6, b=1.0, s_min=-1e30, s_max=1e30, flags=1),
    dict(C=0.2, k_per_us=5e-6, b=3.0, s_min=-0.5, s_max=0.5, flags=2),
    dict(C=0.3, k_per_us=3e-6, b=2.0, s_min=-0.3, s_max=0.7, flags=3),
    # exponential decay (flag 4): alone, with decay-then-add, lazy, and with
    # clamp bounds that exclude 0
    dict(C=0.2, k_per_us=2e-6, b=2.0, s_min=-1.0, s_max=1.0, flags=4),
    dict(C=0.25, k_per_us=1e-4, b=0.7, s_min=-0.4, s_max=0.6, flags=5),
    dict(C=0.2, k_per_us=5e-6, b=3.0, s_min=-0.5, s_max=0.5, flags=6),
    dict(C=0.2, k_per_us=3e-6, b=1.0, s_min=0.1, s_max=0.9, flags=4),
]


@pytest.mark.parametrize("W,H", [(1, 1), (2, 2), (4, 3), (17, 19)])
@pytest.mark.parametrize("pi", range(len(PARAM_SWEEP)))
def test_tiny_sensors(esi, W, H, pi):
    prm = PARAM_SWEEP[pi]
    s = evgen.random_stream(seed=100 + pi * 7 + W, width=W, height=H, n=3000,
                            t_max=600_000, burst_frac=0.3)
    tf = np.linspace(0, 650_000, 23).astype(np.int64)
    _check(esi, s, prm, tf, u8=True, where=f"{W}x{H} p{pi}")


def test_brute_force_runs(esi):
    """Every polarity sequence of length 1..5 with every gap from
    {0, 1/(4k), 1/(2k), 1/k, 2/k}, one run per pixel of one sensor."""
    import itertools
    k = 4e-6
    gaps = [0, 62_500, 125_000, 250_000, 500_000]
    xs, ys, ts, ps = [], [], [], []
    r = 0
    W = 400
    for L in range(1, 6):
        for pols in itertools.product([1, -1], repeat=L):
            for gs in itertools.product(gaps, repeat=L):
                tt = np.cumsum(gs) + 1000
                xs += [r % W] * L
                ys += [r // W] * L
                ts += list(tt)
                ps += list(pols)
                r += 1
    H = (r + W - 1) // W
    o = np.argsort(np.array(ts), kind="stable")
    s = evgen.Stream(np.array(xs, np.uint16)[o], np.array(ys, np.uint16)[o],
                     np.array(ts, np.int64)[o], np.array(ps, np.int8)[o], W, H, 3_000_000)
    for prm in (dict(C=0.25, k_per_us=k, b=2.0, s_min=-1e30, s_max=1e30),
                dict(C=0.25, k_per_us=k, b=2.0, s_min=-0.4, s_max=0.6, flags=1)):
        _check(esi, s, prm, np.array([600_000, 1_300_000, 2_600_000]), where="brute")


def test_ragged_tiles_and_chunks(esi):
    """A sensor that is not a multiple of the tile, and more events per tile
    than one LDS chunk (several chunks, frames inside chunks)."""
    s = evgen.random_stream(seed=5, width=333, height=7, n=400_000, t_max=2_000_000,
                            burst_frac=0.1)
    tf = np.arange(1, 201, dtype=np.int64) * 10_000
    _check(esi, s, DEFAULT, tf, u8=True, where="ragged")


def test_hot_pixels_long_runs(esi):
    """Runs of >= 10^4 events at one pixel inside one window (longer than an
    LDS chunk), as a hot pixel gives."""
    s = evgen.hot_pixel_stream(seed=6, width=64, height=48, n_bg=50_000, t_max=1_000_000,
                               hot=[(3, 4), (40, 47), (63, 0)], hot_period_us=20)
    for prm in (DEFAULT, dict(C=0.2, k_per_us=2e-6, b=2.0, s_min=-1e30, s_max=1e30),
                dict(C=0.2, k_per_us=0.0, b=2.0, s_min=-1e30, s_max=1e30)):
        _check(esi, s, prm, np.array([500_000, 1_000_000]), where="hot")


def test_same_time_bursts_clamped(esi):
    """Many events of one pixel at one time with mixed polarity: the clamp
    makes their array order matter."""
    rng = np.random.default_rng(9)
    n = 30_000
    x = rng.integers(0, 3, n).astype(np.uint16)
    y = np.zeros(n, np.uint16)
    t = np.sort(rng.integers(0, 40, n)).astype(np.int64) * 1000
    p = rng.choice(np.array([-1, 1], np.int8), n)
    s = evgen.Stream(x, y, t, p, 3, 1, 40_000)
    _check(esi, s, dict(C=0.25, k_per_us=0.0, b=1.0, s_min=-0.5, s_max=0.75),
           np.arange(0, 41, dtype=np.int64) * 1000, where="bursts")


def test_edge_cases(esi):
    prm = DEFAULT
    # no events, frames only (pure decay of the initial state = 0)
    s0 = evgen.Stream(np.zeros(0, np.uint16), np.zeros(0, np.uint16), np.zeros(0, np.int64),
                      np.zeros(0, np.int8), 5, 4, 1000)
    _check(esi, s0, prm, np.array([0, 10, 1000]), u8=True, where="empty")
    # a single event; frames before, at and after it
    s1 = evgen.Stream(np.array([2], np.uint16), np.array([1], np.uint16),
                      np.array([5000], np.int64), np.array([1], np.int8), 5, 4, 10_000)
    _check(esi, s1, prm, np.array([0, 4999, 5000, 5001, 400_000, 600_000]), u8=True,
           where="single")
    # every event out of range
    s2 = evgen.random_stream(seed=11, width=5, height=4, n=1000, t_max=10_000, oob_frac=1.0)
    _check(esi, s2, prm, np.array([10_000]), where="all-dropped")
    # some out of range, {0,1} polarity
    s3 = evgen.random_stream(seed=12, width=50, height=40, n=20_000, t_max=100_000,
                             oob_frac=0.1, pol01=True)
    _check(esi, s3, prm, np.arange(1, 11, dtype=np.int64) * 10_000, where="oob")
    # no frames at all
    _check(esi, s3, prm, None, where="no-frames")


def test_unsorted_input_state(esi):
    """Unsorted times: the state is that of array order (frames unspecified)."""
    s = evgen.random_stream(seed=13, width=30, height=20, n=50_000, t_max=500_000,
                            sorted_=False)
    fg, stg, diag, o = _check(esi, s, DEFAULT, None, where="unsorted")
    assert diag["flags"] & 1 and o.unsorted


@pytest.mark.parametrize("W,H,n", [(346, 260, 400_000), (1280, 720, 2_000_000)])
def test_unsorted_input_with_frames(esi, W, H, n):
    """Unsorted times with frames requested (one and two pixels per thread,
    many chunks and frame segments): the state is still that of array order,
    and the frames, whose values are unspecified, stay finite in [0, 1]."""
    s = evgen.random_stream(seed=31, width=W, height=H, n=n, t_max=2_000_000, sorted_=False)
    tf = np.arange(1, 41, dtype=np.int64) * 50_000
    fg, _, stg, diag = gpu_run(esi, s, DEFAULT, t_frames=tf)
    _, o = oracle_run(s, DEFAULT, t_frames=None)
    assert_state(stg, o, DEFAULT["C"], f"unsorted {W}x{H}")
    assert diag["flags"] & 1 and o.unsorted
    assert np.isfinite(fg).all() and fg.min() >= 0.0 and fg.max() <= 1.0


def test_window_split_and_fps(esi):
    """One call vs many calls: exact N, P, T and S within tolerance; 100 and
    1000 FPS frames agree at the shared times."""
    s = evgen.random_stream(seed=14, width=120, height=90, n=300_000, t_max=1_000_000,
                            burst_frac=0.1)
    tf100 = np.arange(1, 101, dtype=np.int64) * 10_000
    tf1000 = np.arange(1, 1001, dtype=np.int64) * 1_000
    f1, _, st1, _ = gpu_run(esi, s, DEFAULT, t_frames=tf100)
    f2, _, st2, _ = gpu_run(esi, s, DEFAULT, t_frames=tf1000)
    np.testing.assert_array_equal(f1, f2[9::10])
    cuts = np.searchsorted(s.t, tf100[:-1], side="right")
    calls = list(zip(np.r_[0, cuts], np.r_[cuts, s.n]))
    f3, _, st3, _ = gpu_run(esi, s, DEFAULT, t_frames=tf100, calls=calls)
    fo, o = oracle_run(s, DEFAULT, t_frames=tf100)
    assert_state(st3, o, DEFAULT["C"], "split")
    assert_frames(f3, fo, DEFAULT, "split")
    for a, b in zip(st1[1:], st3[1:]):
        np.testing.assert_array_equal(a, b)


def test_determinism(esi):
    s = evgen.random_stream(seed=15, width=200, height=100, n=500_000, t_max=1_000_000,
                            burst_frac=0.2)
    tf = np.arange(1, 101, dtype=np.int64) * 10_000
    fa, _, sa, _ = gpu_run(esi, s, DEFAULT, t_frames=tf)
    fb, _, sb, _ = gpu_run(esi, s, DEFAULT, t_frames=tf)
    np.testing.assert_array_equal(fa, fb)
    for a, b in zip(sa, sb):
        np.testing.assert_array_equal(a, b)


def test_snapshot_export_import(esi):
    import torch
    s = evgen.random_stream(seed=16, width=64, height=32, n=40_000, t_max=300_000)
    st = esi.State(s.width, s.height, **DEFAULT)
    st.integrate(s.x[:20_000], s.y[:20_000], s.t[:20_000], s.p[:20_000])
    blob = st.export_state()
    st.integrate(s.x[20_000:], s.y[20_000:], s.t[20_000:], s.p[20_000:])
    snap, code = st.snapshot(350_000, want_u8=True)
    snap = snap.cpu().numpy()
    o = oracle.State(s.width, s.height, oracle.Params(**DEFAULT))
    o.integrate(s.x, s.y, s.t, s.p, want_frames=False)
    ref = o.snapshot(350_000)
    assert_frames(snap[None], ref[None], DEFAULT, "snapshot")
    assert_u8(code.cpu().numpy()[None], ref[None], DEFAULT, "snapshot-u8")
    # restore the midpoint and replay: identical final state
    st2 = esi.State(s.width, s.height, **DEFAULT)
    st2.import_state(blob)
    st2.integrate(s.x[20_000:], s.y[20_000:], s.t[20_000:], s.p[20_000:])
    torch.cuda.synchronize()
    for a, b in zip(st.read_state(), st2.read_state()):
        assert torch.equal(a, b)
    st.close()
    st2.close()


def test_invalid_arguments(esi):
    import torch
    prm = esi.make_params()
    for (w, h) in [(0, 4), (4, 0), (70000, 1)]:
        rc, _ = esi.esi_create_state(w, h, prm, 0)
        assert rc == esi.ESI_ERR_INVALID_ARG
    for bad in [dict(C=0.0), dict(b=0.0), dict(k_per_us=-1.0), dict(s_min=1.0, s_max=1.0)]:
        rc, _ = esi.esi_create_state(4, 4, esi.make_params(**bad), 0)
        assert rc == esi.ESI_ERR_INVALID_ARG
    st = esi.State(4, 4)
    # frames requested without a buffer / times
    x = torch.zeros(1, dtype=torch.uint16, device="cuda")
    rc = esi.esi_integrate_window(st.handle, x.data_ptr(), x.data_ptr(), None, None, 1,
                                  None, 0, None, None, 0)
    assert rc == esi.ESI_ERR_INVALID_ARG
    tf = torch.zeros(1, dtype=torch.int64, device="cuda")
    rc = esi.esi_integrate_window(st.handle, None, None, None, None, 0, tf.data_ptr(), 1,
                                  None, None, 0)
    assert rc == esi.ESI_ERR_INVALID_ARG
    st.close()


def test_frames_unsorted_flag(esi):
    s = evgen.random_stream(seed=17, width=16, height=16, n=1000, t_max=100_000)
    _, _, _, diag = gpu_run(esi, s, DEFAULT, t_frames=np.array([50_000, 20_000, 90_000]))
    assert diag["flags"] & esi.ESI_DIAG_FRAMES_UNSORTED


@pytest.mark.parametrize("name", ["c1"])
def test_workload_full(esi, name):
    s = evgen.preset(name)
    tf = s.frame_times(100)
    _check(esi, s, DEFAULT, tf, u8=True, where=name)


@pytest.mark.parametrize("name,fps,sel", [("c2", 100, [0, 1, 99, 500, 998, 999]),
                                          ("c3", 100, [0, 250, 499]),
                                          ("c3", 1000, [0, 1, 2500, 4999])])
def test_workload_sampled(esi, name, fps, sel):
    """Full-size workloads in the launch configuration the benchmark times;
    the oracle computes the final state and the sampled frames."""
    s = evgen.preset(name)
    tf = s.frame_times(fps)
    fg, _, stg, diag = gpu_run(esi, s, DEFAULT, t_frames=tf, frame_sel=sel)
    fo, o = oracle_run(s, DEFAULT, t_frames=tf, frame_sel=sel)
    assert_state(stg, o, DEFAULT["C"], name)
    assert_frames(fg, fo, DEFAULT, name)
    assert diag["accepted"] == s.n - o.dropped


@pytest.mark.parametrize("W,H,prm", [
    (1280, 720, DEFAULT),                   # 2 pixels per thread (1800 tiles)
    (1600, 1000, PARAM_SWEEP[6]),           # 4 pixels per thread (1563 tiles)
    (2000, 2000, PARAM_SWEEP[3]),           # 8 pixels per thread (1954 tiles)
])
def test_large_sensors(esi, W, H, prm):
    """Sensors large enough for several pixels per thread (the ballot-ranked
    tile sizes included): random events with same-time bursts and a few hot
    pixels whose runs span many chunks; full state and sampled frames."""
    s = evgen.hot_pixel_stream(seed=W + H, width=W, height=H, n_bg=1_500_000,
                               t_max=1_000_000, hot=[(0, 0), (W - 1, H - 1), (W // 2, H // 3)],
                               hot_period_us=97)
    tf = np.arange(1, 21, dtype=np.int64) * 50_000
    sel = [0, 7, 19]
    fg, _, stg, diag = gpu_run(esi, s, prm, t_frames=tf, frame_sel=sel)
    fo, o = oracle_run(s, prm, t_frames=tf, frame_sel=sel)
    assert_state(stg, o, prm["C"], f"{W}x{H}")
    assert_frames(fg, fo, prm, f"{W}x{H}")
    assert diag["accepted"] == s.n - o.dropped


@pytest.mark.parametrize("flags", [4, 5])
def test_exp_decay_workload(esi, flags):
    """The exponential decay variant on the 640x480 workload in the
    benchmark's launch configuration: state and sampled frames."""
    s = evgen.preset("c2")
    tf = s.frame_times(100)
    prm = dict(DEFAULT, flags=flags)
    sel = [0, 1, 500, 999]
    fg, _, stg, diag = gpu_run(esi, s, prm, t_frames=tf, frame_sel=sel)
    fo, o = oracle_run(s, prm, t_frames=tf, frame_sel=sel)
    assert_state(stg, o, prm["C"], f"exp {flags}")
    assert_frames(fg, fo, prm, f"exp {flags}")


def test_clamp_range_without_zero(esi):
    """Clamp bounds that exclude 0: a decayed state leaves [s_min, s_max]
    (and the initial S = 0 is outside), so frames clamp the decayed value."""
    s = evgen.random_stream(seed=18, width=300, height=5, n=60_000, t_max=1_000_000,
                            burst_frac=0.2)
    tf = np.arange(1, 101, dtype=np.int64) * 10_000
    for prm in (dict(C=0.2, k_per_us=2e-6, b=2.0, s_min=0.05, s_max=0.9),
                dict(C=0.2, k_per_us=2e-6, b=1.0, s_min=-0.9, s_max=-0.1, flags=1)):
        _check(esi, s, prm, tf, u8=True, where=f"clamp {prm['s_min']}..{prm['s_max']}")


def _blob_state(blob, npix):
    """S (= hi + lo), T, N, P from an exported state (40-byte header)."""
    off = 40
    hi = np.frombuffer(blob, np.float32, npix, off)
    lo = np.frombuffer(blob, np.float32, npix, off + 4 * npix)
    T = np.frombuffer(blob, np.int64, npix, off + 8 * npix)
    N = np.frombuffer(blob, np.uint32, npix, off + 16 * npix)
    P = np.frombuffer(blob, np.int32, npix, off + 20 * npix)
    return hi.astype(np.float64) + lo.astype(np.float64), T, N, P


def test_imported_state_outside_clamp(esi):
    """A state imported from a call with wider clamps holds S outside
    [s_min, s_max]: frames of pixels no later event touches must still clamp."""
    W, H = 70, 40
    s = evgen.random_stream(seed=19, width=W, height=H, n=80_000, t_max=400_000,
                            burst_frac=0.5)
    s.p[:] = 1  # every event +1: S grows well past 1 without a clamp
    wide = dict(C=0.5, k_per_us=1e-6, b=2.0, s_min=-1e30, s_max=1e30)
    narrow = dict(C=0.5, k_per_us=1e-6, b=2.0, s_min=-1.0, s_max=1.0)
    a = esi.State(W, H, **wide)
    a.integrate(s.x, s.y, s.t, s.p)
    blob = a.export_state()
    a.close()
    S0, T0, N0, P0 = _blob_state(blob, W * H)
    assert S0.max() > 1.5  # the case under test
    b = esi.State(W, H, **narrow)
    b.import_state(blob)
    later = evgen.random_stream(seed=20, width=W, height=H, n=2_000, t_max=900_000,
                                t_min=400_000)
    tf = np.array([450_000, 700_000, 1_000_000, 2_000_000], np.int64)
    fg, _ = b.integrate(later.x, later.y, later.t, later.p, t_frames=tf)
    fg = fg.cpu().numpy()
    o = oracle.State(W, H, oracle.Params(**narrow))
    o.S[:], o.T[:], o.N[:], o.P[:] = S0, T0, N0, P0
    fo = o.integrate(later.x, later.y, later.t, later.p, t_frames=tf)
    assert_frames(fg, fo, narrow, "imported")
    b.close()


def test_u8_only_frames(esi):
    """8-bit codes without FP32 frames equal the codes written next to them."""
    s = evgen.random_stream(seed=21, width=257, height=9, n=100_000, t_max=1_000_000)
    tf = np.arange(1, 51, dtype=np.int64) * 20_000
    for prm in (DEFAULT, dict(DEFAULT, flags=2)):
        a = esi.State(s.width, s.height, **prm)
        f, u_both = a.integrate(s.x, s.y, s.t, s.p, t_frames=tf, want_u8=True)
        b = esi.State(s.width, s.height, **prm)
        none, u_only = b.integrate(s.x, s.y, s.t, s.p, t_frames=tf, want_frames=False,
                                   want_u8=True)
        assert none is None
        np.testing.assert_array_equal(u_both.cpu().numpy(), u_only.cpu().numpy())
        fo, _ = oracle_run(s, prm, t_frames=tf)
        assert_u8(u_only.cpu().numpy(), fo, prm, "u8-only")
        a.close()
        b.close()


@pytest.mark.parametrize("scene,k", [("fig2", 0.0), ("fig2", 1.0 / 120_000),
                                     ("fig4", 0.0), ("fig4", 1e-5)])
def test_paper_scenes(esi, scene, k):
    """The paper's illustrative scenes (the moving disc of Fig. 2, the
    noise-only accumulation of Fig. 4; their qualitative claims are checked
    on the oracle in test_scenes.py) on the GPU path, state and frames."""
    if scene == "fig2":
        s = evgen.moving_circle()
        prm = dict(C=0.2, k_per_us=k, b=2.0, s_min=-10.0, s_max=10.0)
        tf = np.array([50_000, 200_000, 320_001, 350_000], np.int64)
    else:
        s = evgen.noise_only()
        prm = dict(C=0.2, k_per_us=k, b=2.0, s_min=-1e6, s_max=1e6)
        tf = np.array([1_000_000, 1_999_999], np.int64)
    _check(esi, s, prm, tf, where=f"{scene} k={k}")


@pytest.mark.parametrize("flags,k,tf_us", [
    # exponential decay: frames 0.1, 0.5, 2 and 10 s apart span more than 600
    # decay lengths at k = 1e-3 /us, so every frame is a segment of its own
    (4, 1e-3, [100_000, 500_000, 2_000_000, 10_000_000]),
    (5, 1e-3, [100_000, 100_400, 500_000, 2_000_000, 2_000_700, 10_000_000]),
    # Eq. (4): frames more than 2^30 / k apart (inside the 2^47 us a call's
    # events may span), near frames between them
    (0, 1e-3, [300_000, 300_500, 600_000, 2_000_000_000_000, 2_000_000_000_600,
               100_000_000_000_000]),
    (1, 2e-6, [400_000, 900_000, 700_000_000_000_000, 700_000_000_400_000]),
])
def test_long_gap_segments(esi, flags, k, tf_us):
    """Frames far apart in decay lengths take the kernel's one-frame
    segments: state and every frame against the oracle, in one call and in
    calls whose events follow the far frames."""
    prm = dict(C=0.2, k_per_us=k, b=2.0, s_min=-1.0, s_max=1.0, flags=flags)
    tf = np.array(tf_us, np.int64)
    # events up to just past the first frames, with same-time bursts
    s = evgen.random_stream(seed=31 + flags, width=70, height=30, n=60_000,
                            t_max=int(tf[1]) + 1, burst_frac=0.2)
    _check(esi, s, prm, tf, u8=True, where=f"long gaps flags {flags}")
    # a second call whose events come after the far frames: T jumps by more
    # than 2^30 decay lengths, frames of both calls
    late = evgen.random_stream(seed=41 + flags, width=70, height=30, n=20_000,
                               t_min=int(tf[-1]) - 2_000, t_max=int(tf[-1]) + 3_000)
    both = evgen.Stream(np.concatenate([s.x, late.x]), np.concatenate([s.y, late.y]),
                        np.concatenate([s.t, late.t]), np.concatenate([s.p, late.p]),
                        70, 30, int(tf[-1]) + 3_000)
    tf2 = np.concatenate([tf[:-1], [int(tf[-1]) + 1_000, int(tf[-1]) + 3_000]]).astype(np.int64)
    _check(esi, both, prm, tf2, calls=[(0, s.n), (s.n, both.n)], where=f"late flags {flags}")


def test_host_frame_times(esi):
    """Frame times in host memory (numpy, pageable; and pinned) give the
    frames of the same times in device memory."""
    import torch
    s = evgen.random_stream(seed=51, width=90, height=40, n=80_000, t_max=500_000,
                            burst_frac=0.1)
    tf = np.arange(1, 51, dtype=np.int64) * 10_000
    fo, o = oracle_run(s, DEFAULT, t_frames=tf)
    dev = torch.device("cuda", 0)
    args = [torch.from_numpy(a).to(dev) for a in (s.x.view(np.int16), s.y.view(np.int16), s.t,
                                                    s.p)]
    stream = torch.cuda.current_stream(dev).cuda_stream
    pinned = torch.from_numpy(tf).pin_memory()
    for where, tf_ptr in (("pageable", tf.ctypes.data), ("pinned", pinned.data_ptr())):
        st = esi.State(s.width, s.height, **DEFAULT)
        fr = torch.empty((tf.size, s.height, s.width), dtype=torch.float32, device=dev)
        rc = esi.esi_integrate_window(st.handle, *(a.data_ptr() for a in args), s.n, tf_ptr,
                                      tf.size, fr.data_ptr(), None, stream)
        assert rc == esi.ESI_OK, esi.esi_status_string(rc)
        torch.cuda.synchronize()
        assert_frames(fr.cpu().numpy(), fo, DEFAULT, where)
        S, T, N, P = (a.cpu().numpy() for a in st.read_state())
        assert_state((S, T, N.view(np.uint32), P), o, DEFAULT["C"], where)
        st.close()


@pytest.mark.parametrize("W,H", [(4000, 1100), (65536, 70)])
def test_banded_sensor(esi, W, H):
    """A sensor of more than 4096000 pixels is integrated in bands of rows
    (one pass over the events each): state, dropped count and frames against
    the oracle, with events on every band, off the sensor and in bursts."""
    s = evgen.random_stream(seed=W + H, width=W, height=H, n=400_000, t_max=400_000,
                            burst_frac=0.2, oob_frac=0.02 if W < 65536 else 0.0)
    tf = np.array([100_000, 250_000, 400_000], np.int64)
    fg, _, stg, diag = gpu_run(esi, s, DEFAULT, t_frames=tf)
    fo, o = oracle_run(s, DEFAULT, t_frames=tf)
    assert_state(stg, o, DEFAULT["C"], f"{W}x{H}")
    assert_frames(fg, fo, DEFAULT, f"{W}x{H}")
    assert diag["dropped"] == o.dropped
    assert diag["accepted"] == s.n - o.dropped


def test_hot_pixel_stress_workload(esi):
    """The 1280x720 spoke workload plus hot pixels (0.01% of the sensor at
    10-100 kHz: runs of 10^4 and more events per pixel) in the benchmark's
    launch configuration: state and sampled frames."""
    s = evgen.preset("c3hot")
    tf = s.frame_times(100)
    sel = [0, 250, 499]
    fg, _, stg, diag = gpu_run(esi, s, DEFAULT, t_frames=tf, frame_sel=sel)
    fo, o = oracle_run(s, DEFAULT, t_frames=tf, frame_sel=sel)
    assert_state(stg, o, DEFAULT["C"], "c3hot")
    assert_frames(fg, fo, DEFAULT, "c3hot")
    assert diag["accepted"] == s.n - o.dropped
