"""Served integration on the GPU: sessions fed packet by packet through the
server (one batched call per tick, round-robin picks, sessions admitted
against a memory budget, two ticks in flight) end with the same state, and
give the same frame for every packet, as each session integrated alone, one
call per packet, bit for bit; and both match the FP64 oracle (state and the
frame at every packet's frame time)."""
from __future__ import annotations

import numpy as np
import pytest

import evgen
from esi_parity import assert_frames, assert_state, oracle_run

pytestmark = pytest.mark.gpu

SIZES = [(40, 30), (64, 48), (200, 100), (17, 19), (346, 260), (120, 90), (33, 7), (96, 64),
         (150, 150), (8, 8)]
PACKET_US = 10_000
PACKETS = 4


@pytest.fixture(scope="module")
def esi():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2508_02238_amd as m
    return m


def _stream(i, w, h):
    return evgen.random_stream(seed=900 + i, width=w, height=h, n=2_000 + 300 * i,
                               t_max=PACKETS * PACKET_US, burst_frac=0.1)


def _packet(s, k):
    lo = int(np.searchsorted(s.t, k * PACKET_US, side="left"))
    hi = int(np.searchsorted(s.t, (k + 1) * PACKET_US, side="left"))
    return s.slice(lo, hi), (k + 1) * PACKET_US - 1


def _serve(srv, streams, packets_of, n_packets):
    """Feed every admitted session its packets as fast as the server takes
    them (at most two queued per session), copying each packet's frame when
    its completion is polled.  Returns {sid: [frame per packet]} and the
    final states."""
    import torch
    frames = {sid: {} for sid in streams}
    states = {}
    sent = {sid: 0 for sid in streams}
    while len(states) < len(streams):
        for sid in streams:
            if sid in states or not srv.admitted(sid):
                continue
            s = srv.sessions[sid]
            while sent[sid] < n_packets and len(s.pending) < 2:
                ws, tf = packets_of(sid, sent[sid])
                srv.submit(sid, ws.x, ws.y, ws.t, ws.p, tf, pid=sent[sid])
                sent[sid] += 1
        srv.tick()
        for c in srv.poll():
            assert c.ok
            frames[c.sid][c.pid] = srv.frame(c.sid, c.slot).clone()
        for sid in streams:
            if sid in states or not srv.admitted(sid) or len(frames[sid]) < n_packets:
                continue
            states[sid] = [a.clone() for a in srv.sessions[sid].state.read_state()]
            torch.cuda.synchronize()
            srv.close(sid)
    torch.cuda.synchronize()
    return {sid: [frames[sid][k] for k in range(n_packets)] for sid in streams}, states


def _alone(esi, w, h, prm, packets, tile_pixels=0, scan_run=0):
    import torch
    st = esi.State(w, h, **prm)
    if tile_pixels:
        st.set_tile_pixels(tile_pixels)
    if scan_run:
        st.set_scan_run(scan_run)
    frs = []
    for ws, tf in packets:
        fr, _ = st.integrate(ws.x, ws.y, ws.t, ws.p, t_frames=np.array([tf], np.int64))
        frs.append(fr[0])
    ref = st.read_state()
    torch.cuda.synchronize()
    st.close()
    return frs, ref


def test_served_equals_alone_and_oracle(esi):
    import torch
    from paper_2508_02238_amd.serve import Server
    prm = dict(C=0.2, k_per_us=2e-5, b=2.0, s_min=-1.0, s_max=1.0)
    streams = {i: _stream(i, w, h) for i, (w, h) in enumerate(SIZES)}
    probe = Server(budget_bytes=1 << 40, max_batch=4, max_packet_events=1 << 14)
    costs = [probe._cost(w, h) for (w, h) in SIZES]
    probe.close_all()
    # a budget for about half of the sessions at once; ticks of at most 3
    srv = Server(budget_bytes=sum(sorted(costs)[:5]) + costs[4], max_batch=3,
                 max_packet_events=1 << 14)
    status = [srv.open(i, w, h, **prm) for i, (w, h) in enumerate(SIZES)]
    assert "admitted" in status and "waiting" in status   # the budget is exercised
    got_frames, got_states = _serve(srv, streams, lambda sid, k: _packet(streams[sid], k),
                                    PACKETS)
    lat = [c for c in srv.done if c.ok]
    assert len(lat) == PACKETS * len(SIZES) and all(c.latency_s >= 0 for c in lat)
    srv.close_all()
    tf_all = np.array([(k + 1) * PACKET_US - 1 for k in range(PACKETS)], np.int64)
    for i, (w, h) in enumerate(SIZES):
        pk = [_packet(streams[i], k) for k in range(PACKETS)]
        frs, ref = _alone(esi, w, h, prm, pk)
        for a, b in zip(got_states[i], ref):
            assert torch.equal(a, b), i
        for k in range(PACKETS):
            assert torch.equal(got_frames[i][k], frs[k]), (i, k)
        # the served session against the FP64 oracle: state and every frame
        fo, o = oracle_run(streams[i], prm, t_frames=tf_all)
        S, T, N, P = (a.cpu().numpy() for a in got_states[i])
        assert_state((S, T, N.view(np.uint32), P), o, prm["C"], f"served {i}")
        assert_frames(torch.stack(got_frames[i]).cpu().numpy(), fo, prm, f"served {i}")


def test_served_reuses_pooled_states(esi):
    """Sessions of one size and parameters under a budget for two: later
    sessions run on the reset states of closed ones and still end as if
    integrated alone."""
    import torch
    from paper_2508_02238_amd.serve import Server
    prm = dict(C=0.25, k_per_us=1e-5, b=1.0, s_min=-1.0, s_max=1.0, flags=1)
    W, H = 64, 48
    streams = {i: _stream(20 + i, W, H) for i in range(6)}
    probe = Server(budget_bytes=1 << 40, max_batch=2, max_packet_events=1 << 14)
    cost = probe._cost(W, H)
    probe.close_all()
    srv = Server(budget_bytes=2 * cost, max_batch=8, max_packet_events=1 << 14)
    for i in range(6):
        srv.open(i, W, H, **prm)
    got_frames, got_states = _serve(srv, streams, lambda sid, k: _packet(streams[sid], k),
                                    PACKETS)
    assert sum(len(v) for v in srv.pool.values()) >= 1
    srv.close_all()
    for i in range(6):
        frs, ref = _alone(esi, W, H, prm, [_packet(streams[i], k) for k in range(PACKETS)])
        for a, b in zip(got_states[i], ref):
            assert torch.equal(a, b), i
        for k in range(PACKETS):
            assert torch.equal(got_frames[i][k], frs[k]), (i, k)


def test_served_growing_packets(esi):
    """Packets that grow from tick to tick, so the server's staging buffers
    are replaced while earlier ticks may still run: every session still gives
    the frames and state of its packets integrated alone."""
    import torch
    from paper_2508_02238_amd.serve import Server
    prm = dict(C=0.2, k_per_us=2e-5, b=2.0, s_min=-1.0, s_max=1.0)
    W, H = 346, 260
    sizes = [1_000, 8_000, 30_000, 60_000, 2_000, 45_000]
    n_sess = 3
    packets = [[evgen.random_stream(seed=700 + 10 * i + k, width=W, height=H, n=n,
                                    t_min=k * PACKET_US, t_max=(k + 1) * PACKET_US,
                                    burst_frac=0.05)
                for k, n in enumerate(sizes)] for i in range(n_sess)]
    srv = Server(budget_bytes=1 << 34, max_batch=8, max_packet_events=1 << 17, ring=3,
                 max_inflight=2)
    for i in range(n_sess):
        assert srv.open(i, W, H, **prm) == "admitted"
    frames = {i: {} for i in range(n_sess)}
    for k in range(len(sizes)):
        for i in range(n_sess):
            s = packets[i][k]
            srv.submit(i, s.x, s.y, s.t, s.p, (k + 1) * PACKET_US - 1, pid=k)
        while srv.tick() == 0:          # two ticks in flight: wait for one
            for c in srv.poll(wait=True):
                frames[c.sid][c.pid] = srv.frame(c.sid, c.slot).clone()
        for c in srv.poll():            # no wait: ticks stay in flight
            frames[c.sid][c.pid] = srv.frame(c.sid, c.slot).clone()
    for c in srv.poll(wait=True):
        frames[c.sid][c.pid] = srv.frame(c.sid, c.slot).clone()
    got = [[a.clone() for a in srv.sessions[i].state.read_state()] for i in range(n_sess)]
    torch.cuda.synchronize()
    assert len(srv.done) == n_sess * len(sizes)
    srv.close_all()
    for i in range(n_sess):
        pk = [(packets[i][k], (k + 1) * PACKET_US - 1) for k in range(len(sizes))]
        frs, ref = _alone(esi, W, H, prm, pk)
        for a, b in zip(got[i], ref):
            assert torch.equal(a, b), i
        for k in range(len(sizes)):
            assert torch.equal(frames[i][k], frs[k]), (i, k)


def test_served_with_tuned_tiles(esi):
    """States created with the autotuner's kind of choice (1024-pixel tiles,
    scan above 16 events) serve every session as it integrates alone with
    the same settings, bit for bit, and match the FP64 oracle."""
    import torch
    from paper_2508_02238_amd.serve import HipDevice, Server
    prm = dict(C=0.2, k_per_us=2e-5, b=2.0, s_min=-1.0, s_max=1.0)
    sizes = SIZES[:6]
    streams = {i: _stream(40 + i, w, h) for i, (w, h) in enumerate(sizes)}
    device = HipDevice(4, 1 << 14, tile_pixels={sz: 1024 for sz in sizes}, scan_run=16)
    srv = Server(budget_bytes=1 << 40, max_batch=4, max_packet_events=1 << 14, device=device)
    for i, (w, h) in enumerate(sizes):
        assert srv.open(i, w, h, **prm) == "admitted"
    got_frames, got_states = _serve(srv, streams, lambda sid, k: _packet(streams[sid], k),
                                    PACKETS)
    srv.close_all()
    tf_all = np.array([(k + 1) * PACKET_US - 1 for k in range(PACKETS)], np.int64)
    for i, (w, h) in enumerate(sizes):
        pk = [_packet(streams[i], k) for k in range(PACKETS)]
        frs, ref = _alone(esi, w, h, prm, pk, tile_pixels=1024, scan_run=16)
        for a, b in zip(got_states[i], ref):
            assert torch.equal(a, b), i
        for k in range(PACKETS):
            assert torch.equal(got_frames[i][k], frs[k]), (i, k)
        fo, o = oracle_run(streams[i], prm, t_frames=tf_all)
        S, T, N, P = (a.cpu().numpy() for a in got_states[i])
        assert_state((S, T, N.view(np.uint32), P), o, prm["C"], f"tuned {i}")
        assert_frames(torch.stack(got_frames[i]).cpu().numpy(), fo, prm, f"tuned {i}")
