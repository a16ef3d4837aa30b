"""Served integration: sessions fed packet by packet through the server
(one batched call per tick, sessions admitted against a memory budget) end
with the same state and frames as each session integrated alone, one call
per packet, bit for bit; and latencies are reported for every packet."""
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


def test_served_equals_alone(esi):
    import torch
    from paper_2508_02238_amd.serve import Server
    prm = dict(C=0.2, k_per_us=2e-5, b=2.0, s_min=-1.0, s_max=1.0)
    streams = [_stream(i, w, h) for i, (w, h) in enumerate(SIZES)]
    # a budget for about half of the sessions' states at once
    probe = Server(budget_bytes=1 << 40, max_batch=4, max_packet_events=1 << 14)
    costs = [probe._cost(w, h) for (w, h) in SIZES]
    probe.close_all()
    srv = Server(budget_bytes=sum(sorted(costs)[:5]) + costs[4], max_batch=16,
                 max_packet_events=1 << 14)
    admitted = [srv.open(i, w, h, **prm) for i, (w, h) in enumerate(SIZES)]
    assert any(admitted) and not all(admitted)   # the budget is exercised
    finished = {}
    sent = [0] * len(SIZES)
    while len(finished) < len(SIZES):
        for i in range(len(SIZES)):
            if i in finished or not srv.admitted(i):
                continue
            if sent[i] < PACKETS and not srv.sessions[i].pending:
                ws, tf = _packet(streams[i], sent[i])
                srv.submit(i, ws.x, ws.y, ws.t, ws.p, tf, pid=sent[i])
                sent[i] += 1
        srv.tick()
        srv.poll()
        for i in range(len(SIZES)):
            if i in finished or not srv.admitted(i) or sent[i] < PACKETS:
                continue
            if srv.sessions[i].pending:
                continue
            srv.poll(wait=True)
            st = srv.sessions[i].state
            finished[i] = ([a.clone() for a in st.read_state()],
                           srv.sessions[i].frame.clone())
            torch.cuda.synchronize()
            srv.close(i)
    lat = srv.done
    assert len(lat) == PACKETS * len(SIZES) and all(l >= 0 for _, _, l in lat)
    srv.close_all()
    for i, (w, h) in enumerate(SIZES):
        alone = esi.State(w, h, **prm)
        fr = None
        for k in range(PACKETS):
            ws, tf = _packet(streams[i], k)
            fr, _ = alone.integrate(ws.x, ws.y, ws.t, ws.p, t_frames=np.array([tf], np.int64))
        ref = alone.read_state()
        torch.cuda.synchronize()
        got_state, got_frame = finished[i]
        for a, b in zip(got_state, ref):
            assert torch.equal(a, b), i
        assert torch.equal(got_frame, fr), i
        alone.close()
        # and the served session against the FP64 oracle over its packets
        fo, o = oracle_run(streams[i], prm, t_frames=np.array([PACKETS * PACKET_US - 1], np.int64))
        S, T, N, P = (a.cpu().numpy() for a in got_state)
        assert_state((S, T, N.view(np.uint32), P), o, prm["C"], f"served {i}")
        assert_frames(got_frame.cpu().numpy(), fo, prm, f"served {i}")


def test_served_reuses_pooled_states(esi):
    """Sessions of one size and parameters under a budget for two: later
    sessions run on the reset states of closed ones and still end as if
    integrated alone."""
    import torch
    from paper_2508_02238_amd.serve import Server
    prm = dict(C=0.25, k_per_us=1e-5, b=1.0, s_min=-1.0, s_max=1.0, flags=1)
    W, H = 64, 48
    streams = [_stream(20 + i, W, H) for i in range(6)]
    probe = Server(budget_bytes=1 << 40, max_batch=2, max_packet_events=1 << 14)
    cost = probe._cost(W, H)
    probe.close_all()
    srv = Server(budget_bytes=2 * cost, max_batch=8, max_packet_events=1 << 14)
    got = {}
    for i in range(6):
        srv.open(i, W, H, **prm)
    done_sessions = 0
    sent = [0] * 6
    while done_sessions < 6:
        for i in range(6):
            if i in got or not srv.admitted(i):
                continue
            if sent[i] < PACKETS and not srv.sessions[i].pending:
                ws, tf = _packet(streams[i], sent[i])
                srv.submit(i, ws.x, ws.y, ws.t, ws.p, tf, pid=sent[i])
                sent[i] += 1
        srv.tick()
        srv.poll()
        for i in range(6):
            if i in got or not srv.admitted(i) or sent[i] < PACKETS or srv.sessions[i].pending:
                continue
            srv.poll(wait=True)
            got[i] = ([a.clone() for a in srv.sessions[i].state.read_state()],
                      srv.sessions[i].frame.clone())
            torch.cuda.synchronize()
            srv.close(i)
            done_sessions += 1
    assert sum(len(v) for v in srv.pool.values()) >= 1
    srv.close_all()
    for i in range(6):
        alone = esi.State(W, H, **prm)
        for k in range(PACKETS):
            ws, tf = _packet(streams[i], k)
            fr, _ = alone.integrate(ws.x, ws.y, ws.t, ws.p, t_frames=np.array([tf], np.int64))
        ref = alone.read_state()
        torch.cuda.synchronize()
        for a, b in zip(got[i][0], ref):
            assert torch.equal(a, b), i
        assert torch.equal(got[i][1], fr), i
        alone.close()


def test_served_growing_packets(esi):
    """Packets that grow from tick to tick, so the server's staging buffers
    are replaced while earlier ticks may still run: every session still ends
    as if integrated alone."""
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
    srv = Server(budget_bytes=1 << 34, max_batch=8, max_packet_events=1 << 17)
    for i in range(n_sess):
        assert srv.open(i, W, H, **prm)
    for k in range(len(sizes)):
        for i in range(n_sess):
            s = packets[i][k]
            srv.submit(i, s.x, s.y, s.t, s.p, (k + 1) * PACKET_US - 1, pid=k)
        assert srv.tick() == n_sess
        srv.poll()                      # no wait: ticks stay in flight
    srv.poll(wait=True)
    got = [([a.clone() for a in srv.sessions[i].state.read_state()],
            srv.sessions[i].frame.clone()) for i in range(n_sess)]
    torch.cuda.synchronize()
    assert len(srv.done) == n_sess * len(sizes)
    srv.close_all()
    for i in range(n_sess):
        alone = esi.State(W, H, **prm)
        fr = None
        for k in range(len(sizes)):
            s = packets[i][k]
            fr, _ = alone.integrate(s.x, s.y, s.t, s.p,
                                    t_frames=np.array([(k + 1) * PACKET_US - 1], np.int64))
        ref = alone.read_state()
        torch.cuda.synchronize()
        for a, b in zip(got[i][0], ref):
            assert torch.equal(a, b), i
        assert torch.equal(got[i][1], fr), i
        alone.close()
