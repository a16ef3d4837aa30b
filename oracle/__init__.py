"""FP64 serial CPU oracle of Event-based Single Integration (ESI).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package.  The GPU library never
imports or links it, and the two share no code.

The arithmetic lives in ``esi_oracle.c`` (plain C, FP64, one event at a time
in array order: Alg. 2 of the paper with the clamp of Eq. (13) per event and
the linear map of Eq. (14)); this module only loads the compiled library and
marshals numpy arrays.  ``build()`` compiles it with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "esi_oracle.c")
_LIB = os.path.join(_HERE, "libesi_oracle.so")

DECAY_THEN_ADD = 1
SNAPSHOT_LAZY = 2
DECAY_EXP = 4


def build(src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle (gcc, -O2, no fast-math, no FP contraction)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)
    return out


_lib = None


def load(path: str = _LIB) -> ctypes.CDLL:
    global _lib
    if path == _LIB and _lib is not None:
        return _lib
    if path == _LIB and not os.path.exists(path):
        build()
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, f64, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32
    lib.esi_oracle_decay.argtypes = [f64, f64, f64]
    lib.esi_oracle_decay.restype = f64
    lib.esi_oracle_decay_exp.argtypes = [f64, f64]
    lib.esi_oracle_decay_exp.restype = f64
    lib.esi_oracle_init_state.argtypes = [i64, i64, P, P, P, P]
    lib.esi_oracle_init_state.restype = None
    lib.esi_oracle_snapshot.argtypes = [i64, P, P, i64, f64, f64, f64, f64, u32, P]
    lib.esi_oracle_snapshot.restype = None
    lib.esi_oracle_u8.argtypes = [f64]
    lib.esi_oracle_u8.restype = ctypes.c_uint8
    lib.esi_oracle_integrate.argtypes = [i32, i32, f64, f64, f64, f64, f64, u32,
                                         P, P, P, P, i64, P, P, P, P, i32, P, P,
                                         P, P, P]
    lib.esi_oracle_integrate.restype = None
    lib.esi_oracle_integrate_rows.argtypes = [i32, i32, i32, i32, f64, f64, f64, f64, f64,
                                              u32, P, P, P, P, i64, P, P, P, P, i32, P, P,
                                              P, P, P]
    lib.esi_oracle_integrate_rows.restype = None
    if path == _LIB:
        _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data


@dataclass
class Params:
    """Inputs of Alg. 2: k, b, C, plus the clamp bounds of Eq. (13)."""
    C: float = 0.2
    k_per_us: float = 2e-6
    b: float = 2.0
    s_min: float = -1.0
    s_max: float = 1.0
    t0_us: int = 0
    flags: int = 0


def decay(dt, k, b, lib=None):
    """Eq. (4), scalar."""
    lib = lib or load()
    return lib.esi_oracle_decay(float(dt), float(k), float(b))


def decay_exp(dt, k, lib=None):
    """The accumulator plugin's exponential decay exp(-k dt), scalar."""
    lib = lib or load()
    return lib.esi_oracle_decay_exp(float(dt), float(k))


def u8(F, lib=None):
    """8-bit code of a normalised value (Eq. (14) times 255, rounded half up)."""
    lib = lib or load()
    F = np.asarray(F, dtype=np.float64)
    out = np.empty(F.shape, dtype=np.uint8)
    flat_in, flat_out = F.reshape(-1), out.reshape(-1)
    for i in range(flat_in.size):
        flat_out[i] = lib.esi_oracle_u8(float(flat_in[i]))
    return out


class State:
    """Per-pixel S, T (Alg. 1/2) and the counts N, P, held in host memory."""

    def __init__(self, width: int, height: int, params: Params, lib=None):
        self.W, self.H, self.params = int(width), int(height), params
        self.lib = lib or load()
        npix = self.W * self.H
        self.S = np.empty(npix, np.float64)
        self.T = np.empty(npix, np.int64)
        self.N = np.empty(npix, np.uint32)
        self.P = np.empty(npix, np.int32)
        self.dropped = 0
        self.unsorted = False
        self.lib.esi_oracle_init_state(npix, int(params.t0_us), _ptr(self.S),
                                       _ptr(self.T), _ptr(self.N), _ptr(self.P))

    def copy(self) -> "State":
        o = State.__new__(State)
        o.W, o.H, o.params, o.lib = self.W, self.H, self.params, self.lib
        o.S, o.T, o.N, o.P = self.S.copy(), self.T.copy(), self.N.copy(), self.P.copy()
        o.dropped, o.unsorted = self.dropped, self.unsorted
        return o

    def integrate(self, x, y, t, p, t_frames=None, frame_sel=None,
                  want_frames: bool = True):
        """Run Alg. 2 over the events; returns the selected frames, shape
        [n_sel, H, W] float64 (or None if want_frames is False)."""
        x = np.ascontiguousarray(x, dtype=np.uint16)
        y = np.ascontiguousarray(y, dtype=np.uint16)
        t = np.ascontiguousarray(t, dtype=np.int64)
        p = np.ascontiguousarray(p, dtype=np.int8)
        n = x.size
        assert y.size == n and t.size == n and p.size == n
        tf = (np.zeros(0, np.int64) if t_frames is None
              else np.ascontiguousarray(t_frames, dtype=np.int64))
        nf = tf.size
        sel = None
        nsel = nf
        if frame_sel is not None:
            sel = np.zeros(nf, np.uint8)
            sel[np.asarray(frame_sel, dtype=np.int64)] = 1
            nsel = int(sel.sum())
        frames = None
        if want_frames and nsel > 0:
            frames = np.empty((nsel, self.H, self.W), np.float64)
        dropped = ctypes.c_uint64(0)
        unsorted = ctypes.c_int32(0)
        pr = self.params
        self.lib.esi_oracle_integrate(
            self.W, self.H, pr.C, pr.k_per_us, pr.b, pr.s_min, pr.s_max, pr.flags,
            _ptr(self.S), _ptr(self.T), _ptr(self.N), _ptr(self.P), n,
            _ptr(x), _ptr(y), _ptr(t), _ptr(p), nf, _ptr(tf) if nf else None,
            _ptr(sel), _ptr(frames), ctypes.byref(dropped), ctypes.byref(unsorted))
        self.dropped += dropped.value
        self.unsorted = self.unsorted or bool(unsorted.value)
        return frames

    def integrate_rows(self, x, y, t, p, t_frames=None, frame_sel=None,
                       want_frames: bool = True, threads: int = 1):
        """The same result as integrate(), computed by `threads` host threads,
        each running the oracle's event loop over all events for its own band
        of rows (pixels are independent, so the bands are too).  Used to time
        the oracle on every host core; the serial loop stays the reference."""
        from concurrent.futures import ThreadPoolExecutor
        x = np.ascontiguousarray(x, dtype=np.uint16)
        y = np.ascontiguousarray(y, dtype=np.uint16)
        t = np.ascontiguousarray(t, dtype=np.int64)
        p = np.ascontiguousarray(p, dtype=np.int8)
        n = x.size
        tf = (np.zeros(0, np.int64) if t_frames is None
              else np.ascontiguousarray(t_frames, dtype=np.int64))
        nf = tf.size
        sel = None
        nsel = nf
        if frame_sel is not None:
            sel = np.zeros(nf, np.uint8)
            sel[np.asarray(frame_sel, dtype=np.int64)] = 1
            nsel = int(sel.sum())
        frames = None
        if want_frames and nsel > 0:
            frames = np.empty((nsel, self.H, self.W), np.float64)
        nb = max(1, min(int(threads), self.H))
        cuts = [self.H * i // nb for i in range(nb + 1)]
        drops = [ctypes.c_uint64(0) for _ in range(nb)]
        unsorted = [ctypes.c_int32(0) for _ in range(nb)]
        pr = self.params

        def band(i):
            # ctypes releases the interpreter lock for the duration of the call
            self.lib.esi_oracle_integrate_rows(
                self.W, self.H, cuts[i], cuts[i + 1], pr.C, pr.k_per_us, pr.b, pr.s_min,
                pr.s_max, pr.flags, _ptr(self.S), _ptr(self.T), _ptr(self.N), _ptr(self.P),
                n, _ptr(x), _ptr(y), _ptr(t), _ptr(p), nf, _ptr(tf) if nf else None,
                _ptr(sel), _ptr(frames), ctypes.byref(drops[i]), ctypes.byref(unsorted[i]))

        with ThreadPoolExecutor(max_workers=nb) as ex:
            list(ex.map(band, range(nb)))
        self.dropped += sum(d.value for d in drops)
        self.unsorted = self.unsorted or any(u.value for u in unsorted)
        return frames

    def snapshot(self, t_frame: int):
        """A frame of the current state at t_frame, shape [H, W] float64."""
        out = np.empty((self.H, self.W), np.float64)
        pr = self.params
        self.lib.esi_oracle_snapshot(self.W * self.H, _ptr(self.S), _ptr(self.T),
                                     int(t_frame), pr.k_per_us, pr.b, pr.s_min,
                                     pr.s_max, pr.flags, _ptr(out))
        return out
