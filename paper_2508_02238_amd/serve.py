"""Served integration: many sessions, packets admitted as they arrive.

Each session is an ESI state resident in HBM (S, T, N, P per pixel) fed by
packets of events (e.g. 10 ms each), each ending with one frame.  Packets of
one session are integrated in arrival order, so every session's states and
frames are those of integrating its packets alone, one call per packet
(Alg. 2 per pixel; the frame of Eq. (14) at the packet's frame time).

The server is continuous batching: a tick takes at most one waiting packet of
each of up to ``max_batch`` admitted sessions (round robin from where the
last tick stopped, so no session starves) and integrates them all with one
batched call; up to ``max_inflight`` ticks run on the device while the host
stages the next, and sessions are admitted, closed and replaced between
ticks.  A packet's frame goes to the session's next slot of a ring of
``ring`` frames: the frame of packet j stays valid until packet j + ring of
the same session is launched (ring > max_inflight, so no tick in flight
writes a slot whose packet has not completed).

Admission is against an HBM budget: a session costs its state (24 bytes per
pixel), its frame ring (4 bytes per pixel per slot) and the most scratch the
library allocates for its packets (esi_scratch_bound); a session that does
not fit waits, in arrival order, until others close; one that could never fit
is rejected.  Closed sessions' states are pooled and reused by sessions of
the same size and parameters: creating and destroying a state synchronises
the device, which drains the ticks in flight.  So when the first waiting
session would need pooled states of other kinds destroyed, a later waiting
session whose kind has a pooled state is admitted first, at most
``max_skip`` times in a row before the first one's turn is forced.

The device side is an object with a small interface (``HipDevice`` on a GPU;
the scheduling tests substitute a CPU double), so admission, fairness,
failure handling and closing are exercised without a GPU: a device call that
fails completes that tick's packets with an error and fails those sessions
only; the other sessions go on.
"""
from __future__ import annotations

import collections
import itertools
import time
from dataclasses import dataclass

import numpy as np

STATE_BYTES_PER_PIXEL = 24
FRAME_BYTES_PER_PIXEL = 4


@dataclass
class Completion:
    sid: object
    pid: object
    slot: int           # frame ring slot of the packet's frame (-1: none)
    latency_s: float    # arrival to the poll that saw the packet's tick finish
    ok: bool            # False: the tick's device call failed, or the session was closed


class Session:
    def __init__(self, sid, width, height, params, cost):
        self.sid = sid
        self.width, self.height = width, height
        self.params = params
        self.cost = cost
        self.state = None      # device state handle (device-specific object)
        self.frames = None     # device frame ring (device-specific object)
        # (pid, arrival, host (x, y, t, p) or None, device (x, y, t, p) pointers
        # or None, n, t_frame)
        self.pending = collections.deque()
        self.launched = 0      # packets launched so far (ring slot = launched % ring)
        self.inflight = 0      # packets in ticks not completed yet
        self.status = "new"    # waiting, admitted, failed, closing, closed, rejected
        self.skipped = 0       # admissions of later sessions ahead of this one
        self.seq = 0           # arrival number
        self._key = (width, height, tuple(sorted(params.items())))

    def key(self):
        """The kind of state the session needs: size and method parameters."""
        return self._key


class HipDevice:
    """States, frame rings, staging and the batched call on one GPU (the
    current torch device); every step of the method runs in libesi's
    kernels through esi_integrate_batch."""

    def __init__(self, max_batch: int, max_packet_events: int, tile_pixels=None,
                 scan_run: int = 0, chunk: int = 0):
        """tile_pixels: {(W, H): integration tile size} for the states it
        creates (the autotuner's choice; sizes not listed keep the library's
        default); scan_run: their serial-versus-scan run length, chunk: their
        records per chunk for 512-pixel tiles (0: the library's defaults)."""
        import torch

        from . import Batch, esi_events
        self.torch = torch
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.compute = torch.cuda.current_stream(self.dev)
        self.copy = torch.cuda.Stream(self.dev)   # default priority
        self.max_batch = int(max_batch)
        self.max_packet_events = int(max_packet_events)
        self.tile_pixels = dict(tile_pixels or {})
        self.scan_run = int(scan_run)
        self.chunk = int(chunk)
        self.batch = Batch(self.max_batch)
        self._bufs = [None, None]
        self._flip = 0
        self._scratch = {}
        m = self.max_batch
        self._st = np.zeros(m, np.uint64)
        self._tf = np.zeros(m, np.uint64)
        self._fr = np.zeros(m, np.uint64)
        self._nf = np.ones(m, np.int32)
        self._ev = np.zeros(m, dtype=np.dtype([("x", np.uint64), ("y", np.uint64),
                                                ("t", np.uint64), ("p", np.uint64),
                                                ("n", np.uint64)]))
        assert self._ev.dtype.itemsize == __import__("ctypes").sizeof(esi_events)

    def cost(self, w, h, ring):
        from . import ESI_OK, esi_scratch_bound
        key = (w, h)
        if key not in self._scratch:
            rc, b = esi_scratch_bound(w, h, self.max_packet_events)
            assert rc == ESI_OK, rc
            self._scratch[key] = b
        return (STATE_BYTES_PER_PIXEL + FRAME_BYTES_PER_PIXEL * ring) * w * h + self._scratch[key]

    def create(self, w, h, params, ring):
        from . import State
        torch = self.torch
        with torch.cuda.stream(self.compute):
            st = State(w, h, **params)
            frames = torch.empty((ring, h, w), dtype=torch.float32, device=self.dev)
        if (w, h) in self.tile_pixels:
            st.set_tile_pixels(self.tile_pixels[(w, h)])
        if self.scan_run:
            st.set_scan_run(self.scan_run)
        if self.chunk:
            st.set_chunk(self.chunk)
        return st, frames

    def reset(self, st):
        with self.torch.cuda.stream(self.compute):
            st.reset()

    def destroy(self, st):
        st.close()

    def frame(self, frames, slot):
        return frames[slot]

    def _buffers(self, n):
        """Double-buffered pinned host and device staging for n events."""
        torch = self.torch
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
            b["hn"] = [a.numpy() for a in b["h"]]
            self._bufs[k] = b
            # the new device memory comes from the compute stream's pool: the
            # copy stream writes it only after the compute stream's earlier work
            self.copy.wait_stream(self.compute)
        return b

    def launch(self, items):
        """items: (state, frames, slot, host, dev, n, t_frame) per session, at
        most one per state; host: (x, y, t, p) numpy arrays to stage, or dev:
        (x, y, t, p) device pointers.  Stages the host packets (one pinned
        buffer per field, one copy each on the copy stream) and enqueues one
        batched call on the compute stream.  Returns the tick's completion
        event."""
        from . import ESI_OK, EsiError, esi_integrate_batch_arrays
        torch = self.torch
        m = len(items)
        ns = np.fromiter((it[5] for it in items), np.int64, m)
        hosted = [i for i, it in enumerate(items) if it[3] is not None]
        nh = ns[hosted] if hosted else np.zeros(0, np.int64)
        offs = np.zeros(len(hosted) + 1, np.int64)
        np.cumsum(nh, out=offs[1:])
        n_host = int(offs[-1])
        b = self._buffers(n_host)
        if hosted:
            hx, hy, ht, hp = b["hn"]
            if n_host:
                np.concatenate([items[i][3][0] for i in hosted], out=hx[:n_host].view(np.uint16))
                np.concatenate([items[i][3][1] for i in hosted], out=hy[:n_host].view(np.uint16))
                np.concatenate([items[i][3][2] for i in hosted], out=ht[:n_host])
                np.concatenate([items[i][3][3] for i in hosted], out=hp[:n_host])
                with torch.cuda.stream(self.copy):
                    for hd, dd in zip(b["h"], b["d"]):
                        dd[:n_host].copy_(hd[:n_host], non_blocking=True)
        htf = b["tf"].numpy()
        htf[:m] = [it[6] for it in items]
        with torch.cuda.stream(self.copy):
            b["tfd"][:m].copy_(b["tf"][:m], non_blocking=True)
        self.compute.wait_stream(self.copy)
        ev = self._ev[:m]
        devi = [i for i, it in enumerate(items) if it[4] is not None]
        if devi:
            dp = np.array([items[i][4] for i in devi], dtype=np.uint64).reshape(-1, 4)
            nd = ns[devi].astype(np.uint64)
            has = nd > 0
            for j, f in enumerate(("x", "y", "t", "p")):
                ev[f][devi] = np.where(has, dp[:, j], np.uint64(0))
            ev["n"][devi] = nd
        if hosted:
            dx, dy, dt, dp = (d.data_ptr() for d in b["d"])
            o = offs[:-1].astype(np.uint64)
            has = nh > 0
            evh = np.zeros(len(hosted), dtype=ev.dtype)
            evh["x"] = np.where(has, dx + 2 * o, 0)
            evh["y"] = np.where(has, dy + 2 * o, 0)
            evh["t"] = np.where(has, dt + 8 * o, 0)
            evh["p"] = np.where(has, dp + o, 0)
            evh["n"] = nh.astype(np.uint64)
            ev[hosted] = evh
        self._st[:m] = [it[0].handle for it in items]
        self._tf[:m] = b["tfd"].data_ptr() + 8 * np.arange(m, dtype=np.uint64)
        self._fr[:m] = [it[1].data_ptr() + 4 * it[2] * it[1].shape[1] * it[1].shape[2]
                        for it in items]
        rc = esi_integrate_batch_arrays(self.batch.handle, m, self._st, ev, self._tf,
                                        self._nf, self._fr, self.compute.cuda_stream)
        if rc != ESI_OK:
            raise EsiError(rc, "esi_integrate_batch")
        done = torch.cuda.Event()
        done.record(self.compute)
        b["ready"] = done
        return done

    def ready(self, token) -> bool:
        return token.query()

    def wait(self, token):
        token.synchronize()

    def fence(self):
        """A token that completes when the work enqueued so far has."""
        ev = self.torch.cuda.Event()
        ev.record(self.compute)
        return ev

    def close(self):
        self.compute.synchronize()
        self.batch.close()


class Server:
    """budget_bytes: HBM for admitted sessions; max_batch: sessions per tick;
    ring: frame slots per session (> max_inflight); device: the device side
    (default: HipDevice on the current GPU)."""

    def __init__(self, budget_bytes: int, max_batch: int = 256, max_packet_events: int = 1 << 20,
                 ring: int = 3, max_inflight: int = 2, device=None, max_skip: int = 8):
        if ring <= max_inflight:
            raise ValueError("ring must exceed max_inflight")
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.max_packet_events = int(max_packet_events)
        self.ring = int(ring)
        self.max_inflight = int(max_inflight)
        self.device = device if device is not None else HipDevice(max_batch, max_packet_events)
        self.used = 0
        self.sessions = {}
        # sessions not admitted yet, in arrival order, all and per kind (entries
        # whose status is no longer "waiting" are dropped when they reach the
        # front)
        self.waiting = collections.deque()
        self.waiting_kind = {}
        self.n_waiting = 0
        self._arrivals = itertools.count()
        self.order = []                      # admitted sessions, round-robin order
        self.cursor = 0
        self.inflight = collections.deque()  # (token, [(session, pid, arrival, slot)])
        self.retiring = collections.deque()  # (token, session) closed, not released yet
        self.pool = collections.defaultdict(list)  # key -> [(state, frames)]
        self.done = []                       # every Completion so far
        self.max_skip = int(max_skip)
        self.created = self.destroyed = 0    # device states, for the record

    # ---- sessions ------------------------------------------------------
    def _cost(self, w, h):
        return self.device.cost(w, h, self.ring)

    def open(self, sid, width: int, height: int, **params) -> str:
        """Register a session: 'admitted' now, 'waiting' for budget, or
        'rejected' (it could never fit the budget)."""
        if sid in self.sessions:
            raise KeyError(f"session {sid!r} exists")
        s = Session(sid, int(width), int(height), params, self._cost(width, height))
        s.seq = next(self._arrivals)
        self.sessions[sid] = s
        if s.cost > self.budget:
            s.status = "rejected"
            return s.status
        if not self.n_waiting and self._fits(s):
            self._admit(s)
        else:
            s.status = "waiting"
            self.waiting.append(s)
            self.waiting_kind.setdefault(s.key(), collections.deque()).append(s)
            self.n_waiting += 1
        return s.status

    @staticmethod
    def _first_waiting(q):
        while q and q[0].status != "waiting":
            q.popleft()
        return q[0] if q else None

    def _admit_waiting(self, s):
        self.n_waiting -= 1
        self._admit(s)

    def _admit(self, s):
        pooled = self.pool.get(s.key())
        if pooled:
            # a pooled state already counts in `used`; reset it in stream order
            s.state, s.frames = pooled.pop()
            self.device.reset(s.state)
        else:
            s.state, s.frames = self.device.create(s.width, s.height, s.params, self.ring)
            self.used += s.cost
            self.created += 1
        s.status = "admitted"
        self.order.append(s)

    def _fits_as_is(self, s) -> bool:
        """Room for s without destroying pooled states."""
        return bool(self.pool.get(s.key())) or self.used + s.cost <= self.budget

    def _fits(self, s) -> bool:
        """Room for s: a pooled state of its kind, free budget, or budget
        freed by destroying pooled states of other kinds."""
        if self.pool.get(s.key()):
            return True
        while self.used + s.cost > self.budget:
            victim = next((k for k, v in self.pool.items() if v), None)
            if victim is None:
                return False
            st, _ = self.pool[victim].pop()
            self.device.destroy(st)
            self.destroyed += 1
            self.used -= self._cost(victim[0], victim[1])
        return True

    def close(self, sid):
        """Retire a session: its packets not launched yet complete as not ok;
        its state goes back to the pool once the work queued so far has
        finished (no wait here), and its budget to waiting sessions."""
        s = self.sessions.pop(sid)
        now = time.perf_counter()
        for pk in s.pending:
            self.done.append(Completion(sid, pk[0], -1, now - pk[1], False))
        s.pending.clear()
        if s.status in ("waiting", "rejected", "new"):
            if s.status == "waiting":
                self.n_waiting -= 1   # its queue entries are dropped lazily
            s.status = "closed"
            return
        if s.status == "failed":
            # a failed device call may have poisoned the state: it is
            # destroyed, not pooled, once the queued work is done
            s.status = "failed_closing"
        else:
            self._drop_from_order(s)
            s.status = "closing"
        self.retiring.append((self.device.fence(), s))
        self._reap()

    def _drop_from_order(self, s):
        i = self.order.index(s)
        del self.order[i]
        if i < self.cursor:
            self.cursor -= 1
        if self.order:
            self.cursor %= len(self.order)
        else:
            self.cursor = 0

    def _reap(self):
        while self.retiring and self.device.ready(self.retiring[0][0]):
            _, s = self.retiring.popleft()
            if s.status == "failed_closing":
                # a failed device call may have left the state poisoned:
                # destroy it rather than pool it
                self.device.destroy(s.state)
                self.destroyed += 1
                self.used -= s.cost
            else:
                self.pool[s.key()].append((s.state, s.frames))
            s.state = s.frames = None
            s.status = "closed"
        while self.n_waiting:
            head = self._first_waiting(self.waiting)
            if self._fits_as_is(head):
                self._admit_waiting(head)
                continue
            if head.skipped < self.max_skip:
                # the head needs pooled states of other kinds destroyed:
                # admit first the earliest waiting session of a kind that
                # has a pooled state
                later = None
                for key, states in self.pool.items():
                    q = self.waiting_kind.get(key)
                    c = self._first_waiting(q) if (states and q) else None
                    if c is not None and (later is None or c.seq < later.seq):
                        later = c
                if later is not None:
                    head.skipped += 1
                    self._admit_waiting(later)
                    continue
            if not self._fits(head):
                break
            self._admit_waiting(head)

    def admitted(self, sid) -> bool:
        return self.sessions[sid].status == "admitted"

    def status(self, sid) -> str:
        return self.sessions[sid].status

    # ---- packets -------------------------------------------------------
    def _session_for_packet(self, sid, n):
        s = self.sessions[sid]
        if s.status in ("rejected", "failed", "closed", "closing"):
            raise RuntimeError(f"session {sid!r} is {s.status}")
        if n > self.max_packet_events:
            raise ValueError("packet larger than max_packet_events")
        return s

    def submit(self, sid, x, y, t, p, t_frame: int, pid=None, arrival: float | None = None):
        """A packet of host events (uint16 x, y; int64 t; int8 p) ending with
        a frame at t_frame; arrival: host time (time.perf_counter()).  The
        events are staged through pinned memory when their tick launches."""
        n = len(t)
        s = self._session_for_packet(sid, n)
        host = (np.asarray(x, np.uint16), np.asarray(y, np.uint16), np.asarray(t, np.int64),
                np.asarray(p, np.int8))
        s.pending.append((pid, time.perf_counter() if arrival is None else arrival, host, None,
                          n, int(t_frame)))

    def submit_device(self, sid, x_ptr, y_ptr, t_ptr, p_ptr, n: int, t_frame: int, pid=None,
                      arrival: float | None = None):
        """A packet already in device memory (pointers to n uint16 x, y,
        int64 t, int8 p, e.g. delivered by a camera's DMA or an upstream
        stage); the caller keeps it unchanged until the packet completes."""
        s = self._session_for_packet(sid, int(n))
        s.pending.append((pid, time.perf_counter() if arrival is None else arrival, None,
                          (int(x_ptr), int(y_ptr), int(t_ptr), int(p_ptr)), int(n),
                          int(t_frame)))

    def _pick(self):
        """Up to max_batch admitted sessions with a waiting packet, round
        robin from the cursor; the cursor moves past the last one taken."""
        m = len(self.order)
        pick = []
        last = -1
        for j in range(m):
            i = (self.cursor + j) % m
            s = self.order[i]
            if s.pending:
                pick.append(s)
                last = i
                if len(pick) == self.max_batch:
                    break
        if last >= 0:
            self.cursor = (last + 1) % m
        return pick

    def tick(self) -> int:
        """Launch one tick (if fewer than max_inflight are running): one
        waiting packet of each of up to max_batch sessions.  Returns the
        number of packets launched."""
        self._reap()
        if len(self.inflight) >= self.max_inflight:
            return 0
        pick = self._pick()
        if not pick:
            return 0
        packets = [s.pending.popleft() for s in pick]
        slots = [s.launched % self.ring for s in pick]
        items = [(s.state, s.frames, slot, pk[2], pk[3], pk[4], pk[5])
                 for s, slot, pk in zip(pick, slots, packets)]
        try:
            token = self.device.launch(items)
        except Exception:
            # the call failed: its packets complete as not ok and its
            # sessions fail; every other session goes on
            now = time.perf_counter()
            for s, pk in zip(pick, packets):
                self.done.append(Completion(s.sid, pk[0], -1, now - pk[1], False))
                self._fail(s)
            return 0
        recs = []
        for s, slot, pk in zip(pick, slots, packets):
            s.launched += 1
            s.inflight += 1
            recs.append((s, pk[0], pk[1], slot))
        self.inflight.append((token, recs))
        return len(recs)

    def _fail(self, s):
        now = time.perf_counter()
        for pk in s.pending:
            self.done.append(Completion(s.sid, pk[0], -1, now - pk[1], False))
        s.pending.clear()
        if s.status == "admitted":
            self._drop_from_order(s)
        s.status = "failed"

    def poll(self, wait: bool = False):
        """Completions of the ticks finished now (all in flight if wait)."""
        out = []
        while self.inflight:
            token, recs = self.inflight[0]
            if wait:
                self.device.wait(token)
            elif not self.device.ready(token):
                break
            now = time.perf_counter()
            self.inflight.popleft()
            for s, pid, arr, slot in recs:
                s.inflight -= 1
                out.append(Completion(s.sid, pid, slot, now - arr, True))
        self.done += out
        self._reap()
        return out

    def frame(self, sid, slot):
        """The session's frame in ring slot `slot` (a device tensor view)."""
        s = self.sessions[sid]
        return self.device.frame(s.frames, slot)

    def busy(self) -> int:
        return len(self.inflight)

    def close_all(self):
        self.poll(wait=True)
        for sid in list(self.sessions):
            self.close(sid)
        while self.retiring:
            self.device.wait(self.retiring[0][0])
            self._reap()
        for v in self.pool.values():
            for st, _ in v:
                self.device.destroy(st)
        self.pool.clear()
        self.used = 0
        self.device.close()
