"""Event-based Single Integration (ESI, arXiv 2508.02238) on MI355X (gfx950).

A thin ctypes binding of the C ABI in ``include/esi.h`` (the HIP library
``libesi.so`` built from ``csrc/``): the functions below have the C names and
only marshal arguments; every step of the method runs in the library's HIP
kernels.  PyTorch provides device memory and streams.

There is no fallback: if ``libesi.so`` is missing or fails to load, importing
the binding raises.
"""
from __future__ import annotations

import ctypes
import os

# torch first: it brings the HIP runtime its device memory and streams live
# in, and the library must bind to that same runtime
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libesi.so")

ESI_OK = 0
ESI_ERR_INVALID_ARG = 1
ESI_ERR_OUT_OF_MEMORY = 2
ESI_ERR_HIP = 3
ESI_ERR_POISONED = 4
ESI_ERR_SCRATCH_LIMIT = 5

ESI_ADD_THEN_DECAY = 0
ESI_DECAY_THEN_ADD = 1
ESI_SNAPSHOT_DECAYED = 0
ESI_SNAPSHOT_LAZY = 2
ESI_DECAY_EXP = 4

ESI_DIAG_UNSORTED = 1
ESI_DIAG_FRAMES_UNSORTED = 2
ESI_DIAG_TIME_RANGE = 4
ESI_DIAG_INTERNAL = 8


class esi_params(ctypes.Structure):
    _fields_ = [("C", ctypes.c_double), ("k_per_us", ctypes.c_double), ("b", ctypes.c_double),
                ("s_min", ctypes.c_double), ("s_max", ctypes.c_double),
                ("t0_us", ctypes.c_int64), ("flags", ctypes.c_uint32)]


class esi_events(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("t", ctypes.c_void_p),
                ("p", ctypes.c_void_p), ("n", ctypes.c_size_t)]


class esi_diag(ctypes.Structure):
    _fields_ = [("dropped", ctypes.c_uint64), ("accepted", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("poisoned", ctypes.c_uint32),
                ("calls", ctypes.c_uint64)]


# (name, restype, argtypes) for every entry point of include/esi.h
_VP = ctypes.c_void_p
_SIGNATURES = [
    ("esi_create_state", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(esi_params), _VP,
                                        ctypes.POINTER(_VP)]),
    ("esi_destroy_state", ctypes.c_int, [_VP]),
    ("esi_reset", ctypes.c_int, [_VP, _VP]),
    ("esi_integrate_window", ctypes.c_int, [_VP, ctypes.POINTER(esi_events), _VP,
                                            ctypes.c_int32, _VP, _VP, _VP]),
    ("esi_integrate_window_noalloc", ctypes.c_int, [_VP, ctypes.POINTER(esi_events), _VP,
                                                    ctypes.c_int32, _VP, _VP, _VP]),
    ("esi_snapshot_frame", ctypes.c_int, [_VP, ctypes.c_int64, _VP, _VP, _VP]),
    ("esi_read_state", ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    ("esi_state_bytes", ctypes.c_size_t, [_VP]),
    ("esi_export_state", ctypes.c_int, [_VP, _VP, ctypes.c_size_t]),
    ("esi_import_state", ctypes.c_int, [_VP, _VP, ctypes.c_size_t]),
    ("esi_get_diagnostics", ctypes.c_int, [_VP, ctypes.POINTER(esi_diag)]),
    ("esi_get_size", ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32)]),
    ("esi_profile_enable", ctypes.c_int, [_VP, ctypes.c_int]),
    ("esi_profile_read", ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_uint32),
                                        ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]),
    ("esi_batch_create", ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(_VP)]),
    ("esi_batch_destroy", ctypes.c_int, [_VP]),
    ("esi_integrate_batch", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(_VP),
                                           ctypes.POINTER(esi_events), ctypes.POINTER(_VP),
                                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_VP),
                                           ctypes.POINTER(_VP), _VP]),
    ("esi_set_tile_pixels", ctypes.c_int, [_VP, ctypes.c_int32]),
    ("esi_set_scan_run", ctypes.c_int, [_VP, ctypes.c_int32]),
    ("esi_set_chunk", ctypes.c_int, [_VP, ctypes.c_int32]),
    ("esi_scratch_bound", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_size_t,
                                         ctypes.POINTER(ctypes.c_size_t)]),
    ("esi_status_string", ctypes.c_char_p, [ctypes.c_int]),
]
EXPORTED = [s[0] for s in _SIGNATURES]


def _load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    for name, res, args in _SIGNATURES:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


class EsiError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {esi_status_string(status)}")
        self.status = status


def _check(status: int, where: str):
    if status != ESI_OK:
        raise EsiError(status, where)


# ---------------------------------------------------------------------------
# The C entry points, same names, argument marshalling only.
# ---------------------------------------------------------------------------

def esi_status_string(status: int) -> str:
    return lib.esi_status_string(int(status)).decode()


def esi_create_state(width: int, height: int, params: esi_params, stream: int = 0):
    out = _VP()
    rc = lib.esi_create_state(int(width), int(height), ctypes.byref(params), _VP(stream),
                              ctypes.byref(out))
    return rc, out.value


def esi_destroy_state(st) -> int:
    return lib.esi_destroy_state(_VP(st))


def esi_reset(st, stream: int = 0) -> int:
    return lib.esi_reset(_VP(st), _VP(stream))


def esi_integrate_window(st, x_ptr, y_ptr, t_ptr, p_ptr, n, t_frames_ptr, n_frames,
                         frames_ptr, frames_u8_ptr, stream: int = 0) -> int:
    ev = esi_events(x_ptr, y_ptr, t_ptr, p_ptr, int(n))
    return lib.esi_integrate_window(_VP(st), ctypes.byref(ev), _VP(t_frames_ptr),
                                    int(n_frames), _VP(frames_ptr), _VP(frames_u8_ptr),
                                    _VP(stream))


def esi_integrate_window_noalloc(st, x_ptr, y_ptr, t_ptr, p_ptr, n, t_frames_ptr, n_frames,
                                 frames_ptr, frames_u8_ptr, stream: int = 0) -> int:
    ev = esi_events(x_ptr, y_ptr, t_ptr, p_ptr, int(n))
    return lib.esi_integrate_window_noalloc(_VP(st), ctypes.byref(ev), _VP(t_frames_ptr),
                                            int(n_frames), _VP(frames_ptr), _VP(frames_u8_ptr),
                                            _VP(stream))


def esi_set_tile_pixels(st, tile_pixels: int) -> int:
    return lib.esi_set_tile_pixels(_VP(st), int(tile_pixels))


def esi_set_scan_run(st, scan_run: int) -> int:
    return lib.esi_set_scan_run(_VP(st), int(scan_run))


def esi_set_chunk(st, records: int) -> int:
    return lib.esi_set_chunk(_VP(st), int(records))


def esi_scratch_bound(width: int, height: int, n_events: int):
    out = ctypes.c_size_t()
    rc = lib.esi_scratch_bound(int(width), int(height), int(n_events), ctypes.byref(out))
    return rc, out.value


def esi_batch_create(max_items: int):
    out = _VP()
    rc = lib.esi_batch_create(int(max_items), ctypes.byref(out))
    return rc, out.value


def esi_batch_destroy(batch) -> int:
    return lib.esi_batch_destroy(_VP(batch))


def esi_integrate_batch(batch, states, events, t_frames=None, n_frames=None, frames=None,
                        frames_u8=None, stream: int = 0) -> int:
    """states: state handles; events: (x, y, t, p, n) pointer tuples; the
    other per-item lists hold pointers / counts, or are None for all items."""
    m = len(states)
    st = (_VP * m)(*[_VP(s) for s in states])
    ev = (esi_events * m)(*[esi_events(*e[:4], int(e[4])) for e in events])
    arr = lambda v, ty: None if v is None else (ty * m)(*v)
    return lib.esi_integrate_batch(_VP(batch), m, st, ev, arr(t_frames, _VP),
                                   arr(n_frames, ctypes.c_int32), arr(frames, _VP),
                                   arr(frames_u8, _VP), _VP(stream))


def esi_integrate_batch_arrays(batch, n: int, states, events, t_frames, n_frames, frames,
                               stream: int = 0) -> int:
    """esi_integrate_batch with its per-item arguments as numpy arrays in
    the C layout (no per-item Python objects): states, t_frames and frames
    uint64 pointer arrays of n entries, events a structured array of n
    esi_events (x, y, t, p pointers and n as uint64), n_frames int32."""
    vp = lambda a: ctypes.cast(a.ctypes.data, ctypes.POINTER(_VP))
    return lib.esi_integrate_batch(_VP(batch), int(n), vp(states),
                                   ctypes.cast(events.ctypes.data, ctypes.POINTER(esi_events)),
                                   vp(t_frames),
                                   ctypes.cast(n_frames.ctypes.data, ctypes.POINTER(ctypes.c_int32)),
                                   vp(frames), None, _VP(stream))


def esi_snapshot_frame(st, t_frame_us: int, frame_ptr, u8_ptr, stream: int = 0) -> int:
    return lib.esi_snapshot_frame(_VP(st), int(t_frame_us), _VP(frame_ptr), _VP(u8_ptr),
                                  _VP(stream))


def esi_read_state(st, S_ptr, T_ptr, N_ptr, P_ptr, stream: int = 0) -> int:
    return lib.esi_read_state(_VP(st), _VP(S_ptr), _VP(T_ptr), _VP(N_ptr), _VP(P_ptr),
                              _VP(stream))


def esi_state_bytes(st) -> int:
    return lib.esi_state_bytes(_VP(st))


def esi_export_state(st, buf_ptr, nbytes) -> int:
    return lib.esi_export_state(_VP(st), _VP(buf_ptr), int(nbytes))


def esi_import_state(st, buf_ptr, nbytes) -> int:
    return lib.esi_import_state(_VP(st), _VP(buf_ptr), int(nbytes))


def esi_get_diagnostics(st):
    d = esi_diag()
    rc = lib.esi_get_diagnostics(_VP(st), ctypes.byref(d))
    return rc, {"dropped": d.dropped, "accepted": d.accepted, "flags": d.flags,
                "poisoned": d.poisoned, "calls": d.calls}


def esi_profile_enable(st, enable: bool) -> int:
    return lib.esi_profile_enable(_VP(st), 1 if enable else 0)


def esi_profile_read(st):
    c = ctypes.c_uint32()
    b = ctypes.c_double()
    i = ctypes.c_double()
    rc = lib.esi_profile_read(_VP(st), ctypes.byref(c), ctypes.byref(b), ctypes.byref(i))
    return rc, c.value, b.value, i.value


def esi_get_size(st):
    w, h = ctypes.c_int32(), ctypes.c_int32()
    rc = lib.esi_get_size(_VP(st), ctypes.byref(w), ctypes.byref(h))
    return rc, w.value, h.value


# ---------------------------------------------------------------------------
# Convenience wrapper on torch tensors (device memory + current stream).
# ---------------------------------------------------------------------------

def make_params(C=0.2, k_per_us=2e-6, b=2.0, s_min=-1.0, s_max=1.0, t0_us=0, flags=0):
    return esi_params(float(C), float(k_per_us), float(b), float(s_min), float(s_max),
                      int(t0_us), int(flags))


class State:
    """An ESI state on the current torch CUDA (HIP) device."""

    def __init__(self, width: int, height: int, params: esi_params | None = None, **kw):
        import torch
        self._torch = torch
        self.params = params if params is not None else make_params(**kw)
        self.width, self.height = int(width), int(height)
        self.device = torch.device("cuda", torch.cuda.current_device())
        rc, h = esi_create_state(self.width, self.height, self.params, self._stream())
        _check(rc, "esi_create_state")
        self.handle = h

    def _stream(self) -> int:
        return self._torch.cuda.current_stream(self.device).cuda_stream

    def close(self):
        if getattr(self, "handle", None):
            esi_destroy_state(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _dev(t, dtype, torch, device):
        """A contiguous device tensor holding t with the bit pattern of dtype.
        16-bit coordinates travel as int16 (same bits as uint16)."""
        import numpy as np
        if dtype == torch.uint16:
            if isinstance(t, np.ndarray) or not hasattr(t, "dtype"):
                t = torch.from_numpy(np.ascontiguousarray(np.asarray(t, np.uint16)).view(np.int16))
            elif t.dtype == torch.uint16:
                t = t.view(torch.int16)
            elif t.dtype != torch.int16:
                raise TypeError("pixel coordinates must be uint16 (or int16 bit patterns)")
            dtype = torch.int16
        t = torch.as_tensor(t)
        if t.dtype != dtype:
            t = t.to(dtype=dtype)
        if t.device != device or not t.is_contiguous():
            t = t.to(device=device).contiguous()
        return t

    def integrate(self, x, y, t, p, t_frames=None, frames=None, frames_u8=None,
                  want_frames: bool = True, want_u8: bool = False):
        """Integrate events (tensors or arrays; moved to the device if needed)
        and return (frames, frames_u8) for the frame times t_frames."""
        torch, dev = self._torch, self.device
        x = self._dev(x, torch.uint16, torch, dev)
        y = self._dev(y, torch.uint16, torch, dev)
        t = self._dev(t, torch.int64, torch, dev)
        p = self._dev(p, torch.int8, torch, dev)
        n = x.numel()
        if not (y.numel() == n and t.numel() == n and p.numel() == n):
            raise ValueError("x, y, t, p must have the same length")
        nf = 0
        tf = None
        if t_frames is not None:
            tf = self._dev(t_frames, torch.int64, torch, dev)
            nf = tf.numel()
        if nf and frames is None and want_frames:
            frames = torch.empty((nf, self.height, self.width), dtype=torch.float32, device=dev)
        if nf and frames_u8 is None and want_u8:
            frames_u8 = torch.empty((nf, self.height, self.width), dtype=torch.uint8, device=dev)
        ptr = lambda a: a.data_ptr() if (a is not None and a.numel()) else None
        rc = esi_integrate_window(self.handle, ptr(x), ptr(y), ptr(t), ptr(p), n,
                                  ptr(tf) if nf else None, nf, ptr(frames) if nf else None,
                                  ptr(frames_u8) if nf else None, self._stream())
        _check(rc, "esi_integrate_window")
        self._keep = (x, y, t, p, tf)  # alive until the stream has consumed them
        return frames, frames_u8

    def snapshot(self, t_frame: int, want_u8: bool = False):
        torch = self._torch
        f = torch.empty((self.height, self.width), dtype=torch.float32, device=self.device)
        u = torch.empty((self.height, self.width), dtype=torch.uint8,
                        device=self.device) if want_u8 else None
        rc = esi_snapshot_frame(self.handle, int(t_frame), f.data_ptr(),
                                u.data_ptr() if u is not None else None, self._stream())
        _check(rc, "esi_snapshot_frame")
        return (f, u) if want_u8 else f

    def read_state(self):
        torch, dev = self._torch, self.device
        npx = self.width * self.height
        S = torch.empty(npx, dtype=torch.float32, device=dev)
        T = torch.empty(npx, dtype=torch.int64, device=dev)
        N = torch.empty(npx, dtype=torch.int32, device=dev)
        P = torch.empty(npx, dtype=torch.int32, device=dev)
        rc = esi_read_state(self.handle, S.data_ptr(), T.data_ptr(), N.data_ptr(),
                            P.data_ptr(), self._stream())
        _check(rc, "esi_read_state")
        return S, T, N, P

    def export_state(self) -> bytes:
        nbytes = esi_state_bytes(self.handle)
        buf = ctypes.create_string_buffer(nbytes)
        _check(esi_export_state(self.handle, ctypes.addressof(buf), nbytes), "esi_export_state")
        return buf.raw

    def import_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(esi_import_state(self.handle, ctypes.addressof(buf), len(blob)),
               "esi_import_state")

    def reset(self):
        _check(esi_reset(self.handle, self._stream()), "esi_reset")

    def set_tile_pixels(self, tile_pixels: int):
        _check(esi_set_tile_pixels(self.handle, tile_pixels), "esi_set_tile_pixels")

    def set_scan_run(self, scan_run: int):
        _check(esi_set_scan_run(self.handle, scan_run), "esi_set_scan_run")

    def set_chunk(self, records: int):
        _check(esi_set_chunk(self.handle, records), "esi_set_chunk")

    def diagnostics(self) -> dict:
        rc, d = esi_get_diagnostics(self.handle)
        _check(rc, "esi_get_diagnostics")
        return d


class Batch:
    """Integrate many States with one set of kernel launches per call."""

    def __init__(self, max_items: int):
        import torch
        self._torch = torch
        rc, h = esi_batch_create(int(max_items))
        _check(rc, "esi_batch_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            esi_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def integrate(self, states, events, t_frames=None, want_frames: bool = True,
                  want_u8: bool = False):
        """states: list of State; events: list of (x, y, t, p) per state;
        t_frames: list of frame-time arrays (or None entries), or None.
        Returns the list of (frames, frames_u8) per state."""
        torch = self._torch
        m = len(states)
        keep, evp, tfp, nfs, frp, u8p, outs = [], [], [], [], [], [], []
        ptr = lambda a: a.data_ptr() if (a is not None and a.numel()) else None
        for i, s in enumerate(states):
            dev = s.device
            x = State._dev(events[i][0], torch.uint16, torch, dev)
            y = State._dev(events[i][1], torch.uint16, torch, dev)
            t = State._dev(events[i][2], torch.int64, torch, dev)
            p = State._dev(events[i][3], torch.int8, torch, dev)
            n = x.numel()
            tf = None
            if t_frames is not None and t_frames[i] is not None and len(t_frames[i]):
                tf = State._dev(t_frames[i], torch.int64, torch, dev)
            nf = tf.numel() if tf is not None else 0
            fr = (torch.empty((nf, s.height, s.width), dtype=torch.float32, device=dev)
                  if nf and want_frames else None)
            u8 = (torch.empty((nf, s.height, s.width), dtype=torch.uint8, device=dev)
                  if nf and want_u8 else None)
            keep += [x, y, t, p, tf]
            evp.append((ptr(x), ptr(y), ptr(t), ptr(p), n))
            tfp.append(ptr(tf) if nf else None)
            nfs.append(nf)
            frp.append(ptr(fr) if nf else None)
            u8p.append(ptr(u8) if nf else None)
            outs.append((fr, u8))
        stream = torch.cuda.current_stream(states[0].device).cuda_stream
        rc = esi_integrate_batch(self.handle, [s.handle for s in states], evp, tfp, nfs,
                                 frp, u8p, stream)
        _check(rc, "esi_integrate_batch")
        self._keep = keep  # alive until the stream has consumed them
        return outs
