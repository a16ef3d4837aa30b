"""Batched calls (many states per launch) through the C ABI: every item's
state, diagnostics and frames equal those of one esi_integrate_window call
per item, bit for bit, over several consecutive windows; and match the
oracle."""
from __future__ import annotations

import numpy as np
import pytest

import evgen
from esi_parity import assert_frames, assert_state, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def esi():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2508_02238_amd as m
    return m


# (W, H, events per window, params): tile sizes 256 to 1024 pixels, every
# decay kind, both orders, lazy frames, a clamp range without 0, and items
# with no events
ITEMS = [
    (17, 19, 3_000, dict(C=0.2, k_per_us=2e-6, b=2.0, s_min=-1.0, s_max=1.0)),
    (346, 260, 40_000, dict(C=0.2, k_per_us=1e-5, b=1.0, s_min=-1.0, s_max=1.0, flags=1)),
    (640, 480, 120_000, dict(C=0.15, k_per_us=1e-4, b=4.7, s_min=-0.3, s_max=0.7)),
    (640, 480, 0, dict(C=0.2, k_per_us=2e-6, b=2.0, s_min=-1.0, s_max=1.0)),
    (1280, 720, 200_000, dict(C=0.2, k_per_us=3e-6, b=2.0, s_min=-1.0, s_max=1.0, flags=4)),
    (1600, 1000, 150_000, dict(C=0.25, k_per_us=5e-6, b=3.0, s_min=-0.5, s_max=0.5, flags=2)),
    (300, 5, 20_000, dict(C=0.2, k_per_us=3e-6, b=1.0, s_min=0.1, s_max=0.9, flags=5)),
    (64, 48, 50_000, dict(C=0.2, k_per_us=2e-6, b=2.0, s_min=-1.0, s_max=1.0)),
]
WINDOW = 10_000  # us


def _streams():
    out = []
    for i, (W, H, n, prm) in enumerate(ITEMS):
        s = evgen.random_stream(seed=500 + i, width=W, height=H, n=3 * n, t_max=3 * WINDOW,
                                burst_frac=0.1, oob_frac=0.01 if i % 3 == 0 else 0.0)
        out.append(s)
    return out


def _window(s, w):
    lo = np.searchsorted(s.t, w * WINDOW, side="left")
    hi = np.searchsorted(s.t, (w + 1) * WINDOW, side="left")
    return s.slice(int(lo), int(hi))


@pytest.mark.parametrize("chunk", [0, 2048])
def test_batch_equals_single_calls(esi, chunk):
    """chunk 2048: every state takes 2048-record chunks for 512-pixel tiles
    (the 1280x720 item by default, the 64x48 one by its tile setting), so the
    launch mixes that class with the others."""
    import torch
    streams = _streams()
    single = [esi.State(W, H, **prm) for (W, H, _, prm) in ITEMS]
    batched = [esi.State(W, H, **prm) for (W, H, _, prm) in ITEMS]
    if chunk:
        for st in single + batched:
            st.set_chunk(chunk)
        single[-1].set_tile_pixels(512)
        batched[-1].set_tile_pixels(512)
    batch = esi.Batch(len(ITEMS))
    for w in range(3):
        evs, tfs = [], []
        for i, s in enumerate(streams):
            ws = _window(s, w)
            evs.append((ws.x, ws.y, ws.t, ws.p))
            # frames in the window for most items, none for item 2
            tfs.append(None if i == 2 else
                       np.array([w * WINDOW + 2_500, (w + 1) * WINDOW - 1], np.int64))
        outs_b = batch.integrate(batched, evs, tfs, want_frames=True, want_u8=True)
        outs_s = [single[i].integrate(*evs[i], t_frames=tfs[i], want_u8=True)
                  for i in range(len(ITEMS))]
        torch.cuda.synchronize()
        for i in range(len(ITEMS)):
            for a, b in zip(outs_b[i], outs_s[i]):
                assert (a is None) == (b is None), (w, i)
                if a is not None:
                    assert torch.equal(a, b), (w, i)
            for a, b in zip(batched[i].read_state(), single[i].read_state()):
                assert torch.equal(a, b), (w, i)
            assert batched[i].diagnostics() == single[i].diagnostics(), (w, i)
    batch.close()
    for s in single + batched:
        s.close()


def test_batch_matches_oracle(esi):
    """One batched call per window on fresh states, checked against the
    oracle after three windows (frames of the last window)."""
    streams = _streams()
    states = [esi.State(W, H, **prm) for (W, H, _, prm) in ITEMS]
    batch = esi.Batch(len(ITEMS))
    last = None
    for w in range(3):
        evs, tfs = [], []
        for s in streams:
            ws = _window(s, w)
            evs.append((ws.x, ws.y, ws.t, ws.p))
            tfs.append(np.array([(w + 1) * WINDOW - 1], np.int64))
        last = batch.integrate(states, evs, tfs)
    for i, (W, H, _, prm) in enumerate(ITEMS):
        s = streams[i]
        full = s.slice(0, int(np.searchsorted(s.t, 3 * WINDOW, side="left")))
        fo, o = oracle_run(full, prm, t_frames=np.array([3 * WINDOW - 1], np.int64))
        S, T, N, P = (a.cpu().numpy() for a in states[i].read_state())
        assert_state((S, T, N.view(np.uint32), P), o, prm["C"], f"item {i}")
        assert_frames(last[i][0].cpu().numpy(), fo, prm, f"item {i}")
    batch.close()
    for s in states:
        s.close()


def test_batch_rejects_duplicates_and_overflow(esi):
    a = esi.State(8, 8)
    batch = esi.Batch(2)
    ev = (None, None, None, None, 0)
    assert esi.esi_integrate_batch(batch.handle, [a.handle, a.handle], [ev, ev]) == \
        esi.ESI_ERR_INVALID_ARG
    b, c = esi.State(8, 8), esi.State(8, 8)
    assert esi.esi_integrate_batch(batch.handle, [a.handle, b.handle, c.handle],
                                   [ev, ev, ev]) == esi.ESI_ERR_INVALID_ARG
    # frames asked for without an output
    assert esi.esi_integrate_batch(batch.handle, [a.handle], [ev], [12345], [1], None,
                                   None) == esi.ESI_ERR_INVALID_ARG
    batch.close()
    for s in (a, b, c):
        s.close()


@pytest.mark.parametrize("W,H", [(640, 480), (333, 7)])
def test_tile_size_keeps_results(esi, W, H):
    """Every integration tile size (esi_set_tile_pixels) gives the same N, P,
    T exactly and S and frames within the parity tolerance of the oracle (the
    decay bases are taken relative to each chunk's first event, so the
    rounding depends on the chunking)."""
    import torch
    prm = dict(C=0.2, k_per_us=3e-6, b=2.0, s_min=-1.0, s_max=1.0)
    s = evgen.random_stream(seed=77, width=W, height=H, n=200_000, t_max=300_000,
                            burst_frac=0.1)
    tf = np.arange(1, 31, dtype=np.int64) * 10_000
    fo, o = oracle_run(s, prm, t_frames=tf)
    for tile in (0, 256, 512, 1024, 2048):
        st = esi.State(W, H, **prm)
        st.set_tile_pixels(tile)
        fr, _ = st.integrate(s.x, s.y, s.t, s.p, t_frames=tf)
        S, T, N, P = (a.cpu().numpy() for a in st.read_state())
        assert_state((S, T, N.view(np.uint32), P), o, prm["C"], f"tile {tile}")
        assert_frames(fr.cpu().numpy(), fo, prm, f"tile {tile}")
        st.close()
    assert esi.esi_set_tile_pixels(None, 256) == esi.ESI_ERR_INVALID_ARG
    assert esi.esi_set_tile_pixels(None, 300) == esi.ESI_ERR_INVALID_ARG


def test_c4_preset_matches_oracle(esi):
    """The batched workload (64 streams of mixed size and rate, one batched
    call per 10 ms window with one frame per stream) over four windows:
    every stream's frames and final state against the oracle."""
    import torch
    win, nwin = 10_000, 4
    streams = evgen.preset_batch("c4", duration_us=nwin * win)
    prm = dict(C=0.2, k_per_us=2e-6, b=2.0, s_min=-1.0, s_max=1.0)
    states = [esi.State(s.width, s.height, **prm) for s in streams]
    batch = esi.Batch(len(streams))
    frames = [[] for _ in streams]
    for w in range(nwin):
        evs, tfs = [], []
        for s in streams:
            ws = _window_of(s, w, win)
            evs.append((ws.x, ws.y, ws.t, ws.p))
            tfs.append(np.array([(w + 1) * win - 1], np.int64))
        outs = batch.integrate(states, evs, tfs)
        for i, (fr, _) in enumerate(outs):
            frames[i].append(fr)
    torch.cuda.synchronize()
    tf = np.arange(1, nwin + 1, dtype=np.int64) * win - 1
    for i, s in enumerate(streams):
        full = s.slice(0, int(np.searchsorted(s.t, nwin * win, side="left")))
        fo, o = oracle_run(full, prm, t_frames=tf)
        S, T, N, P = (a.cpu().numpy() for a in states[i].read_state())
        assert_state((S, T, N.view(np.uint32), P), o, prm["C"], f"stream {i}")
        fg = torch.cat(frames[i]).cpu().numpy()
        assert_frames(fg, fo, prm, f"stream {i}")
    batch.close()
    for st in states:
        st.close()


def _window_of(s, w, win):
    lo = np.searchsorted(s.t, w * win, side="left")
    hi = np.searchsorted(s.t, (w + 1) * win, side="left")
    return s.slice(int(lo), int(hi))


def test_tuner_chunk_dimension(esi):
    """The autotuner's chunk choice for 512-pixel tiles: one of the
    candidates, and the states it sets up integrate as the oracle does."""
    import torch
    from paper_2508_02238_amd.tune import tune
    prm = dict(C=0.2, k_per_us=2e-6, b=2.0, s_min=-1.0, s_max=1.0)
    sizes = [(200, 60), (200, 60)]
    dev = torch.device("cuda", 0)
    streams = [evgen.random_stream(seed=900 + i, width=200, height=60, n=200_000,
                                   t_max=WINDOW, burst_frac=0.2) for i in range(2)]
    evs = [tuple(torch.from_numpy(a).to(dev) for a in (s.x.view(np.int16), s.y.view(np.int16),
                                                       s.t, s.p)) for s in streams]
    tfs = [torch.tensor([WINDOW - 1], dtype=torch.int64, device=dev)] * 2
    tuned = tune(sizes, prm, [(evs, tfs)], reps=1, tile_candidates=(512,),
                 scan_candidates=())
    assert tuned["tile_pixels"][(200, 60)] in (0, 512)
    assert tuned["chunk"] in (0, 2048)
    st = esi.State(200, 60, **prm)
    st.set_tile_pixels(512)
    st.set_chunk(2048)
    s = streams[0]
    fr, _ = st.integrate(s.x, s.y, s.t, s.p, t_frames=np.array([WINDOW - 1], np.int64))
    S, T, N, P = (a.cpu().numpy() for a in st.read_state())
    fo, o = oracle_run(s, prm, t_frames=np.array([WINDOW - 1], np.int64))
    assert_state((S, T, N.view(np.uint32), P), o, prm["C"], "tuned chunk")
    assert_frames(fr.cpu().numpy(), fo, prm, "tuned chunk")
    st.close()
