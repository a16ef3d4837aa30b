"""Helpers shared by the GPU parity tests: run one stream through the HIP
path (through the C ABI binding) and through the FP64 oracle, and compare.

Parity rule:
  N, P, T, dropped: bit-exact;
  S: |S_gpu - S_ref| <= 1e-5 * max(|S_ref|, C);
  frames F: |F_gpu - F_ref| <= 1e-5 * max(|F_ref|, C / (S_max - S_min));
  8-bit codes: equal, except +-1 where the reference 255 F + 1/2 lies within
  255 * (frame tolerance) of an integer (a rounding boundary).
The floor C is one event's contribution: relative error means nothing at a
cancellation zero of S.
"""
from __future__ import annotations

import numpy as np

import oracle

REL = 1e-5


def gpu_run(esi, stream, prm: dict, t_frames=None, calls=None, want_u8=False,
            frame_sel=None, scan_run=None):
    """Integrate on the GPU through the C ABI binding.  calls: list of
    (lo, hi) event ranges, one esi_integrate_window call each (default: one
    call).  A frame goes to the call after whose events it is complete: the
    first call c such that t_frames[j] < first time of call c+1 (the last
    call takes the rest).  Returns frames (rows frame_sel if given), u8,
    state (S, T, N, P) and the diagnostics.  scan_run: the state's
    serial-versus-scan run length (None: the library's default)."""
    import torch
    st = esi.State(stream.width, stream.height, **prm)
    if scan_run is not None:
        st.set_scan_run(scan_run)
    n = stream.n
    tf = None if t_frames is None else np.asarray(t_frames, np.int64)
    calls = calls or [(0, n)]
    frames_all, u8_all = [], []
    fj = 0
    for ci, (lo, hi) in enumerate(calls):
        sub = None
        if tf is not None:
            fk = len(tf)
            if ci + 1 < len(calls) and calls[ci + 1][0] < n:
                t_next = stream.t[calls[ci + 1][0]]
                fk = fj
                while fk < len(tf) and tf[fk] < t_next:
                    fk += 1
            sub = tf[fj:fk]
            fj = fk
        f, u = st.integrate(stream.x[lo:hi], stream.y[lo:hi], stream.t[lo:hi],
                            stream.p[lo:hi],
                            t_frames=sub if sub is not None and len(sub) else None,
                            want_u8=want_u8)
        if f is not None:
            frames_all.append(f)
        if u is not None:
            u8_all.append(u)
    torch.cuda.synchronize()
    S, T, N, P = (a.cpu().numpy() for a in st.read_state())
    diag = st.diagnostics()
    st.close()
    # copy only the frames compared (the full set can be tens of GB)
    cat = lambda xs: (xs[0] if len(xs) == 1 else torch.cat(xs)) if xs else None
    frames, u8 = cat(frames_all), cat(u8_all)
    if frame_sel is not None:
        idx = torch.as_tensor(np.asarray(frame_sel), device=frames_all[0].device if frames_all
                              else "cuda")
        frames = frames[idx] if frames is not None else None
        u8 = u8[idx] if u8 is not None else None
    frames = frames.cpu().numpy() if frames is not None else None
    u8 = u8.cpu().numpy() if u8 is not None else None
    return frames, u8, (S, T, N.view(np.uint32), P), diag


def oracle_run(stream, prm: dict, t_frames=None, frame_sel=None, want_frames=True):
    o = oracle.State(stream.width, stream.height, oracle.Params(**prm))
    f = o.integrate(stream.x, stream.y, stream.t, stream.p, t_frames=t_frames,
                    frame_sel=frame_sel, want_frames=want_frames and t_frames is not None)
    return f, o


def assert_state(state_gpu, o, C, where=""):
    S, T, N, P = state_gpu
    assert np.array_equal(N, o.N), f"{where}: N differs at {np.nonzero(N != o.N)[0][:5]}"
    assert np.array_equal(P, o.P), f"{where}: P differs at {np.nonzero(P != o.P)[0][:5]}"
    assert np.array_equal(T, o.T), f"{where}: T differs at {np.nonzero(T != o.T)[0][:5]}"
    err = np.abs(S.astype(np.float64) - o.S)
    tol = REL * np.maximum(np.abs(o.S), C)
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, (f"{where}: S off at {bad[:5]}: gpu {S[bad[:5]]} ref {o.S[bad[:5]]}")


def frame_tol(F_ref, prm):
    return REL * np.maximum(np.abs(F_ref), prm["C"] / (prm["s_max"] - prm["s_min"]))


def assert_frames(F_gpu, F_ref, prm, where=""):
    assert F_gpu.shape == F_ref.shape, (where, F_gpu.shape, F_ref.shape)
    err = np.abs(F_gpu.astype(np.float64) - F_ref)
    tol = frame_tol(F_ref, prm)
    bad = np.argwhere(err > tol)
    assert bad.shape[0] == 0, (f"{where}: {bad.shape[0]} frame values off, first {bad[:3]}: "
                               f"gpu {F_gpu[tuple(bad[0])]} ref {F_ref[tuple(bad[0])]}")


def assert_u8(U_gpu, F_ref, prm, where=""):
    U_ref = u8_codes(F_ref)
    diff = np.abs(U_gpu.astype(np.int32) - U_ref.astype(np.int32))
    a = 255.0 * F_ref + 0.5
    near = np.abs(a - np.round(a)) <= 255.0 * frame_tol(F_ref, prm) + 1e-6
    assert np.all(diff <= 1), where
    assert np.all((diff == 0) | near), f"{where}: u8 differs away from a rounding boundary"


def u8_codes(F):
    """The oracle's 8-bit code (oracle.u8), vectorised for large frames: the
    same FP32 operations, checked against oracle.u8 on a sample."""
    f = F.astype(np.float32)
    a = np.floor(np.float32(255.0) * f + np.float32(0.5))
    out = np.clip(a, 0, 255).astype(np.uint8)
    flat = F.reshape(-1)
    idx = np.linspace(0, flat.size - 1, min(flat.size, 2000)).astype(np.int64)
    assert np.array_equal(out.reshape(-1)[idx], oracle.u8(flat[idx]))
    return out
