"""The served loop's scheduling on the CPU, with a test double for the
device: admission against the budget (waiting in arrival order, rejection),
round-robin fairness, frame ring slots, an injected device-call failure and a
session closed while its packets are queued and in flight.  In every case the
sessions not involved go on unaffected: their packets complete, in order,
once each."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2508_02238_amd.serve import Server


class Token:
    def __init__(self):
        self.done = False


class FakeState:
    def __init__(self, w, h):
        self.w, self.h = w, h
        self.packets = []      # (pid tag, t_frame) integrated, in order
        self.resets = 0
        self.destroyed = False


class FakeDevice:
    """Launches record what each state integrated; tokens complete when the
    test calls run() (the device finishing everything queued so far)."""

    def __init__(self, scratch=1000):
        self.scratch = scratch
        self.tokens = []
        self.launches = []
        self.fail_next = 0
        self.created = 0

    def cost(self, w, h, ring):
        return (24 + 4 * ring) * w * h + self.scratch

    def create(self, w, h, params, ring):
        self.created += 1
        return FakeState(w, h), [None] * ring

    def reset(self, st):
        st.packets.clear()
        st.resets += 1

    def destroy(self, st):
        st.destroyed = True

    def frame(self, frames, slot):
        return frames[slot]

    def launch(self, items):
        if self.fail_next:
            self.fail_next -= 1
            raise RuntimeError("injected device failure")
        states = [id(it[0]) for it in items]
        assert len(set(states)) == len(states), "a state twice in one call"
        for st, frames, slot, host, dev, n, tf in items:
            assert not st.destroyed
            t = host[2]
            tag = int(t[0]) if len(t) else None
            st.packets.append((tag, tf))
            frames[slot] = (tag, tf)
        self.launches.append(len(items))
        tok = Token()
        self.tokens.append(tok)
        return tok

    def ready(self, tok):
        return tok.done

    def wait(self, tok):
        self.run()

    def fence(self):
        tok = Token()
        self.tokens.append(tok)
        return tok

    def run(self):
        for t in self.tokens:
            t.done = True
        self.tokens.clear()

    def close(self):
        pass


def _packet(sid, k):
    # the packet's first event time tags (session, packet)
    t = np.array([sid * 1000 + k, sid * 1000 + k], np.int64)
    z = np.zeros(2, np.uint16)
    return z, z, t, np.ones(2, np.int8), (k + 1) * 10_000 - 1


def _drain(srv, dev):
    while srv.busy() or any(s.pending for s in srv.sessions.values() if s.status == "admitted"):
        srv.tick()
        dev.run()
        srv.poll()


def test_round_robin_fairness():
    dev = FakeDevice()
    srv = Server(budget_bytes=1 << 40, max_batch=3, ring=3, max_inflight=2, device=dev)
    for sid in range(10):
        assert srv.open(sid, 8, 8) == "admitted"
        for k in range(5):
            srv.submit(sid, *_packet(sid, k), pid=k)
    served_at = {sid: [] for sid in range(10)}
    tick = 0
    while any(s.pending for s in srv.sessions.values()):
        n = srv.tick()
        assert n <= 3
        for c in srv.poll():
            pass
        dev.run()
        for c in srv.poll():
            served_at[c.sid].append(tick)
        tick += 1
    # every session is served once per ceil(10 / 3) = 4 ticks: no starvation
    for sid, ticks in served_at.items():
        assert len(ticks) == 5
        assert max(np.diff(ticks)) <= 4, (sid, ticks)
    # packets of each session integrated in order, once each
    for sid in range(10):
        st = srv.sessions[sid].state
        assert [p[0] for p in st.packets] == [sid * 1000 + k for k in range(5)]
    srv.close_all()


def test_budget_admission_waiting_and_rejection():
    dev = FakeDevice()
    srv = Server(budget_bytes=1, max_batch=8, ring=3, device=dev)
    one = srv._cost(16, 16)
    srv = Server(budget_bytes=2 * one + 10, max_batch=8, ring=3, device=dev)
    assert srv.open("a", 16, 16) == "admitted"
    assert srv.open("b", 16, 16) == "admitted"
    assert srv.open("c", 16, 16) == "waiting"
    assert srv.open("d", 16, 16) == "waiting"
    assert srv.open("huge", 4000, 4000) == "rejected"
    with pytest.raises(RuntimeError):
        srv.submit("huge", *_packet(9, 0))
    assert srv.used <= srv.budget
    # packets of a waiting session queue until it is admitted
    srv.submit("c", *_packet(3, 0), pid=0)
    srv.submit("a", *_packet(1, 0), pid=0)
    srv.tick()
    dev.run()
    srv.poll()
    assert [c.sid for c in srv.done] == ["a"]
    # closing a frees its budget once its queued work has finished; the
    # first waiting session (c, not d) takes it, with its queued packet
    srv.close("a")
    assert srv.status("c") == "waiting"
    dev.run()
    srv.poll()
    assert srv.status("c") == "admitted" and srv.status("d") == "waiting"
    assert srv.used <= srv.budget
    _drain(srv, dev)
    assert sorted((c.sid, c.pid) for c in srv.done) == [("a", 0), ("c", 0)]
    # c reused a's pooled state (reset), not a new one
    assert dev.created == 2 and srv.sessions["c"].state.resets == 1
    srv.close_all()


def test_frame_ring_slots():
    dev = FakeDevice()
    srv = Server(budget_bytes=1 << 40, max_batch=4, ring=3, max_inflight=2, device=dev)
    srv.open(0, 8, 8)
    for k in range(7):
        srv.submit(0, *_packet(0, k), pid=k)
    got = []
    while srv.sessions[0].pending or srv.busy():
        srv.tick()
        # two ticks in flight at most
        assert srv.busy() <= 2
        dev.run()
        for c in srv.poll():
            # the frame of packet k is in slot k % ring when it completes
            assert c.slot == c.pid % 3
            assert srv.frame(0, c.slot) == (k_tag := c.pid, (c.pid + 1) * 10_000 - 1)
            got.append(k_tag)
    assert got == list(range(7))
    with pytest.raises(ValueError):
        Server(budget_bytes=1 << 40, ring=2, max_inflight=2, device=dev)
    srv.close_all()


def test_injected_device_failure_leaves_other_sessions():
    dev = FakeDevice()
    srv = Server(budget_bytes=1 << 40, max_batch=2, ring=3, device=dev)
    for sid in range(4):
        srv.open(sid, 8, 8)
        for k in range(3):
            srv.submit(sid, *_packet(sid, k), pid=k)
    srv.tick()               # sessions 0, 1
    dev.run()
    srv.poll()
    dev.fail_next = 1
    assert srv.tick() == 0   # sessions 2, 3: the call fails
    assert srv.status(2) == "failed" and srv.status(3) == "failed"
    bad = [c for c in srv.done if not c.ok]
    assert sorted((c.sid, c.pid) for c in bad) == [(2, 0), (2, 1), (2, 2), (3, 0), (3, 1), (3, 2)]
    with pytest.raises(RuntimeError):
        srv.submit(2, *_packet(2, 3))
    _drain(srv, dev)
    ok = sorted((c.sid, c.pid) for c in srv.done if c.ok)
    assert ok == [(0, 0), (0, 1), (0, 2), (1, 0), (1, 1), (1, 2)]
    for sid in (0, 1):
        assert [p[0] for p in srv.sessions[sid].state.packets] == [sid * 1000 + k for k in range(3)]
    # a failed session's state is destroyed, not pooled, and its budget freed
    used = srv.used
    st2 = srv.sessions[2].state
    srv.close(2)
    dev.run()
    srv.poll()
    assert st2.destroyed and srv.used < used
    assert all(st2 is not s for v in srv.pool.values() for s, _ in v)
    srv.close_all()


def test_killed_session_mid_stream():
    dev = FakeDevice()
    srv = Server(budget_bytes=1, max_batch=8, ring=3, device=dev)
    one = srv._cost(8, 8)
    srv = Server(budget_bytes=3 * one, max_batch=8, ring=3, max_inflight=2, device=dev)
    for sid in range(4):
        srv.open(sid, 8, 8)
    assert srv.status(3) == "waiting"
    for sid in range(4):
        for k in range(4):
            srv.submit(sid, *_packet(sid, k), pid=k)
    srv.tick()                # packet 0 of sessions 0-2 in flight
    srv.tick()                # packet 1 in flight
    srv.close(1)              # killed: packets 2 and 3 dropped, 0 and 1 in flight
    dropped = sorted((c.sid, c.pid) for c in srv.done if not c.ok)
    assert dropped == [(1, 2), (1, 3)]
    assert srv.status(3) == "waiting"   # its state is released only after the ticks
    dev.run()
    srv.poll()
    assert srv.status(3) == "admitted"
    _drain(srv, dev)
    ok = sorted((c.sid, c.pid) for c in srv.done if c.ok)
    assert ok == sorted([(s, k) for s in (0, 2, 3) for k in range(4)] + [(1, 0), (1, 1)])
    for sid in (0, 2, 3):
        assert [p[0] for p in srv.sessions[sid].state.packets] == [sid * 1000 + k for k in range(4)]
    srv.close_all()


def test_admission_prefers_pooled_kind_with_bounded_skips():
    """When the first waiting session would need pooled states of another
    kind destroyed (a device-wide synchronisation on a GPU), a later waiting
    session whose kind has a pooled state is admitted first, at most
    max_skip times before the first one's turn is forced."""
    dev = FakeDevice()
    probe = Server(budget_bytes=1, device=dev)
    ca, cb = probe._cost(16, 16), probe._cost(8, 8)
    srv = Server(budget_bytes=2 * ca + cb // 2, max_batch=8, ring=3, device=dev, max_skip=2)
    assert srv.open("a1", 16, 16) == "admitted" and srv.open("a2", 16, 16) == "admitted"
    assert srv.open("b1", 8, 8) == "waiting"          # needs budget: behind nobody
    for k in range(3, 7):
        assert srv.open(f"a{k}", 16, 16) == "waiting"
    created = srv.created
    # a1 closes: its pooled state goes to a3, ahead of b1 (one skip)
    srv.close("a1"); dev.run(); srv.poll()
    assert srv.status("a3") == "admitted" and srv.status("b1") == "waiting"
    assert srv.created == created and srv.destroyed == 0
    # a2 closes: a4 takes its state (second skip of b1)
    srv.close("a2"); dev.run(); srv.poll()
    assert srv.status("a4") == "admitted" and srv.status("b1") == "waiting"
    # a3 closes: b1 has been passed over twice, so its turn is forced: the
    # pooled 16x16 state is destroyed to make room, and a5 keeps waiting
    srv.close("a3"); dev.run(); srv.poll()
    assert srv.status("b1") == "admitted" and srv.status("a5") == "waiting"
    assert srv.destroyed == 1 and srv.created == created + 1
    assert srv.used <= srv.budget
    srv.close_all()
