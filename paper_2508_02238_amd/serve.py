"""Served integration: many sessions, packets admitted as they arrive.

Each session is an ESI state resident in HBM (S, T, N, P per pixel) fed by
packets of events (e.g. 10 ms each) that end with one frame.  The server
keeps at most one packet per session in a tick: a tick stages the events of
every session that has a packet waiting into one device buffer (a copy
stream, overlapping the previous tick's kernels) and integrates all of them
with one batched call (``esi_integrate_batch``) on the compute stream.  A
packet's frame is ready when its tick's completion event has fired; the
packet-to-frame latency is the host time from its arrival to the first poll
that sees that event.

Sessions are admitted against an HBM budget: a session costs its state
(24 bytes per pixel) plus a scratch reserve; sessions that do not fit wait
until others close.  Within a session packets are integrated in arrival
order, so every session's states and frames are those of integrating its
packets alone, one call per packet.
"""
from __future__ import annotations

import collections
import time

import numpy as np
import torch

from . import Batch, State

STATE_BYTES_PER_PIXEL = 24


class Session:
    def __init__(self, sid, width, height, params, cost):
        self.sid = sid
        self.width, self.height = width, height
        self.params = params
        self.cost = cost
        self.state = None
        self.frame = None          # device f32 [1][H][W], the latest packet's frame
        self.pending = collections.deque()


class Server:
    """budget_bytes: HBM for admitted sessions; max_batch: sessions per tick;
    scratch_per_event: reserve per event of a session's largest packet."""

    def __init__(self, budget_bytes: int, max_batch: int = 256, max_packet_events: int = 1 << 20,
                 scratch_per_event: int = 16):
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.max_packet_events = int(max_packet_events)
        self.scratch_per_event = int(scratch_per_event)
        self.used = 0
        self.sessions = {}
        self.waiting = collections.deque()   # sessions not admitted yet
        self.batch = Batch(self.max_batch)
        self.compute = torch.cuda.current_stream(self.dev)
        self.copy = torch.cuda.Stream(self.dev)   # default priority
        self.inflight = collections.deque()  # (event, [(sid, packet id, arrival)])
        self.retiring = collections.deque()  # (event, session) closed, not freed yet
        # states of closed sessions kept for reuse (same size and parameters):
        # creating and destroying states synchronises the device
        self.pool = collections.defaultdict(list)
        self.done = []                       # (sid, packet id, latency s)
        self._bufs = [None, None]
        self._flip = 0

    # ---- sessions ------------------------------------------------------
    def _cost(self, w, h):
        return STATE_BYTES_PER_PIXEL * w * h + self.scratch_per_event * self.max_packet_events

    def open(self, sid, width: int, height: int, **params) -> bool:
        """Register a session; True if admitted now, False if it waits."""
        s = Session(sid, int(width), int(height), params, self._cost(width, height))
        self.sessions[sid] = s
        if not self.waiting and self._fits(s):
            self._admit(s)
            return True
        self.waiting.append(s)
        return False

    @staticmethod
    def _key(s):
        return (s.width, s.height, tuple(sorted(s.params.items())))

    def _admit(self, s):
        # state set-up runs on the compute stream, in order with the ticks
        with torch.cuda.stream(self.compute):
            pooled = self.pool.get(self._key(s))
            if pooled:
                # a pooled state already counts in `used`; reset it in stream order
                s.state, s.frame = pooled.pop()
                s.state.reset()
                return
            s.state = State(s.width, s.height, **s.params)
            s.frame = torch.empty((1, s.height, s.width), dtype=torch.float32, device=self.dev)
        self.used += s.cost

    def _fits(self, s) -> bool:
        """Room for s: a pooled state of its kind, free budget, or budget
        freed by destroying pooled states of other kinds."""
        if self.pool.get(self._key(s)):
            return True
        while self.used + s.cost > self.budget:
            victim = next((k for k, v in self.pool.items() if v), None)
            if victim is None:
                return False
            st, _ = self.pool[victim].pop()
            st.close()
            self.used -= self._cost(victim[0], victim[1])
        return True

    def close(self, sid):
        """Retire a session.  Its memory is freed, and its budget handed to
        waiting sessions, once the work queued so far has finished (no wait
        here)."""
        s = self.sessions.pop(sid)
        if s.state is None:
            self.waiting.remove(s)
            return
        ev = torch.cuda.Event()
        ev.record(self.compute)
        self.retiring.append((ev, s))
        self._reap()

    def _reap(self):
        while self.retiring and self.retiring[0][0].query():
            _, s = self.retiring.popleft()
            self.pool[self._key(s)].append((s.state, s.frame))
            s.state = None
            s.frame = None
        while self.waiting and self._fits(self.waiting[0]):
            self._admit(self.waiting.popleft())

    def admitted(self, sid) -> bool:
        return self.sessions[sid].state is not None

    # ---- packets -------------------------------------------------------
    def submit(self, sid, x, y, t, p, t_frame: int, pid=None, arrival: float | None = None):
        """A packet of host events (uint16 x, y; int64 t; int8 p) ending with
        a frame at t_frame; arrival: host time (time.perf_counter())."""
        n = len(t)
        if n > self.max_packet_events:
            raise ValueError("packet larger than max_packet_events")
        self.sessions[sid].pending.append(
            (pid, time.perf_counter() if arrival is None else arrival,
             np.asarray(x, np.uint16), np.asarray(y, np.uint16), np.asarray(t, np.int64),
             np.asarray(p, np.int8), int(t_frame)))

    def _buffers(self, n):
        """Double-buffered pinned host and device staging for n events."""
        k = self._flip
        self._flip ^= 1
        b = self._bufs[k]
        if b is not None and b["ready"] is not None:
            # its last tick has consumed it; wait before reuse, and before a
            # larger buffer replaces it (its freed device memory may go to
            # the new buffer, which the copy stream writes)
            b["ready"].synchronize()
            b["ready"] = None
        if b is None or b["cap"] < n:
            cap = max(n, 1 << 16) * 5 // 4
            b = {"cap": cap,
                 "h": [torch.empty(cap, dtype=d, pin_memory=True)
                       for d in (torch.int16, torch.int16, torch.int64, torch.int8)],
                 "d": [torch.empty(cap, dtype=d, device=self.dev)
                       for d in (torch.int16, torch.int16, torch.int64, torch.int8)],
                 "tf": torch.empty(self.max_batch, dtype=torch.int64, pin_memory=True),
                 "tfd": torch.empty(self.max_batch, dtype=torch.int64, device=self.dev),
                 "ready": None}
            self._bufs[k] = b
            # the new device memory comes from the compute stream's pool: the
            # copy stream writes it only after the compute stream's earlier work
            self.copy.wait_stream(self.compute)
        return b

    def tick(self) -> int:
        """Integrate one waiting packet of every admitted session that has one
        (at most max_batch sessions); returns the number of packets."""
        pick = [s for s in self.sessions.values() if s.state is not None and s.pending]
        pick = pick[:self.max_batch]
        if not pick:
            return 0
        packets = [s.pending.popleft() for s in pick]
        n_all = sum(len(pk[4]) for pk in packets)
        b = self._buffers(n_all)
        hx, hy, ht, hp = (a.numpy() for a in b["h"])
        htf = b["tf"].numpy()
        off = 0
        offs = []
        for i, pk in enumerate(packets):
            n = len(pk[4])
            hx[off:off + n] = pk[2].view(np.int16)
            hy[off:off + n] = pk[3].view(np.int16)
            ht[off:off + n] = pk[4]
            hp[off:off + n] = pk[5]
            htf[i] = pk[6]
            offs.append(off)
            off += n
        with torch.cuda.stream(self.copy):
            for hd, dd in zip(b["h"], b["d"]):
                dd[:max(off, 1)].copy_(hd[:max(off, 1)], non_blocking=True)
            b["tfd"][:len(packets)].copy_(b["tf"][:len(packets)], non_blocking=True)
        self.compute.wait_stream(self.copy)
        dx, dy, dt, dp = b["d"]
        evs, tfs, frs = [], [], []
        for i, pk in enumerate(packets):
            n = len(pk[4])
            o = offs[i]
            evs.append((dx.data_ptr() + 2 * o, dy.data_ptr() + 2 * o, dt.data_ptr() + 8 * o,
                        dp.data_ptr() + o, n) if n else (None, None, None, None, 0))
            tfs.append(b["tfd"].data_ptr() + 8 * i)
            frs.append(pick[i].frame.data_ptr())
        from . import ESI_OK, esi_integrate_batch, esi_status_string
        rc = esi_integrate_batch(self.batch.handle, [s.state.handle for s in pick], evs, tfs,
                                 [1] * len(pick), frs, None, self.compute.cuda_stream)
        if rc != ESI_OK:
            raise RuntimeError(f"esi_integrate_batch: {esi_status_string(rc)}")
        ev = torch.cuda.Event()
        ev.record(self.compute)
        b["ready"] = ev
        self.inflight.append((ev, [(s.sid, pk[0], pk[1]) for s, pk in zip(pick, packets)]))
        return len(packets)

    def poll(self, wait: bool = False):
        """Move finished ticks to `done`; returns the packets finished now."""
        out = []
        while self.inflight:
            ev, pk = self.inflight[0]
            if wait:
                ev.synchronize()
            elif not ev.query():
                break
            now = time.perf_counter()
            self.inflight.popleft()
            out += [(sid, pid, now - arr) for sid, pid, arr in pk]
        self.done += out
        self._reap()
        return out

    def busy(self) -> int:
        return len(self.inflight)

    def close_all(self):
        self.poll(wait=True)
        for sid in list(self.sessions):
            self.close(sid)
        self.compute.synchronize()
        self._reap()
        for v in self.pool.values():
            for st, _ in v:
                st.close()
        self.pool.clear()
        self.used = 0
        self.batch.close()
