"""HIP path vs the FP64 oracle on seeded random configurations: sensor size,
event mix (uniform pixels, hot pixels, same-time bursts, events off the
sensor, 0/1 polarity), method parameters and flags, the state's start time,
frame times (duplicates, before the first event, long after the last),
the split of the stream into calls, the integration tile size, the
serial-versus-scan run length and the chunk size are all drawn per case.  Each case compares
the state (N, P, T exact; S within 1e-5), the drop count and every frame
(and 8-bit code) with the oracle over the whole stream (Alg. 2, Eq. (14))."""
from __future__ import annotations

import numpy as np
import pytest

import evgen
from esi_parity import assert_frames, assert_state, assert_u8, oracle_run

pytestmark = pytest.mark.gpu

N_CASES = 32
SCAN_OFF = 2**31 - 1


@pytest.fixture(scope="module")
def esi():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2508_02238_amd as m
    return m


def _case(seed: int):
    rng = np.random.default_rng(9000 + seed)
    W = int(rng.choice([1, 3, int(rng.integers(2, 64)), int(rng.integers(64, 300)),
                        int(rng.integers(64, 300))]))
    H = int(rng.choice([1, 2, int(rng.integers(2, 40)), int(rng.integers(40, 200)),
                        int(rng.integers(40, 200))]))
    n = int(rng.choice([0, int(rng.integers(1, 2000)), int(rng.integers(2000, 150_000)),
                        int(rng.integers(2000, 150_000))]))
    t_lo = int(rng.integers(0, 1_000_000))
    span = int(rng.choice([1, 1000, 200_000, 3_000_000]))
    # pixels: uniform, plus a few hot pixels taking a share of the events
    q = rng.integers(0, W * H, n)
    n_hot = int(rng.integers(0, 4))
    if n_hot and n:
        hot = rng.integers(0, W * H, n_hot)
        m = rng.random(n) < rng.uniform(0.05, 0.6)
        q[m] = hot[rng.integers(0, n_hot, int(m.sum()))]
    x = (q % W).astype(np.int64)
    y = (q // W).astype(np.int64)
    t = np.sort(rng.integers(t_lo, t_lo + span, n)).astype(np.int64)
    if n > 1:  # same-time bursts
        idx = np.nonzero(rng.random(n - 1) < rng.uniform(0.0, 0.5))[0] + 1
        t[idx] = t[idx - 1]
        t = np.maximum.accumulate(t)
    if n and rng.random() < 0.3:  # a few events off the sensor
        m = rng.random(n) < 0.01
        x[m] = W + rng.integers(0, 3, int(m.sum()))
    p = rng.choice(np.array([-1, 1], np.int8), n)
    if rng.random() < 0.2:
        p = (p > 0).astype(np.int8)  # 0/1 encoding: 0 counts as negative
    s = evgen.Stream(x.astype(np.uint16), y.astype(np.uint16), t, p, W, H, span)

    flags = int(rng.integers(0, 8))
    k = float(rng.choice([0.0, 1e-7, 2e-6, 3e-5, 1e-4]))
    if rng.random() < 0.5:
        s_min, s_max = -1.0, 1.0
    else:
        s_min = float(rng.uniform(-1.0, 0.3))
        s_max = s_min + float(rng.uniform(0.2, 1.5))
    prm = dict(C=float(rng.uniform(0.05, 0.4)), k_per_us=k,
               b=float(rng.choice([0.5, 1.0, 2.0, 3.0, 4.7])), s_min=s_min, s_max=s_max,
               t0_us=int(rng.choice([0, t_lo, t_lo - 5000])), flags=flags)

    nf = int(rng.choice([0, int(rng.integers(1, 8)), int(rng.integers(8, 60)),
                         int(rng.integers(8, 60))]))
    tf = np.sort(rng.integers(t_lo - 2000, t_lo + span + 400_000, nf)).astype(np.int64)
    if nf > 2:
        tf[nf // 2] = tf[nf // 2 - 1]  # a repeated frame time
    n_calls = int(rng.integers(1, 4))
    cuts = np.sort(rng.integers(0, n + 1, n_calls - 1)) if n else np.zeros(n_calls - 1, int)
    bounds = [0, *[int(c) for c in cuts], n]
    calls = [(bounds[i], bounds[i + 1]) for i in range(n_calls)]
    tile = int(rng.choice([0, 256, 512, 1024, 2048]))
    scan = rng.choice([None, 1, 4, 16, 64, SCAN_OFF])
    want_u8 = bool(rng.random() < 0.3)
    chunk = int(rng.choice([0, 2048]))
    return s, prm, tf, calls, tile, (None if scan is None else int(scan)), want_u8, chunk


def _gpu(esi, s, prm, tf, calls, tile, scan, want_u8, chunk):
    import torch
    st = esi.State(s.width, s.height, **prm)
    if tile:
        st.set_tile_pixels(tile)
    if scan is not None:
        st.set_scan_run(scan)
    if chunk:
        st.set_chunk(chunk)
    frames, u8s = [], []
    fj = 0
    for ci, (lo, hi) in enumerate(calls):
        # a frame goes to the call after whose events it is complete
        fk = len(tf)
        if ci + 1 < len(calls) and calls[ci + 1][0] < s.n:
            t_next = s.t[calls[ci + 1][0]]
            fk = fj
            while fk < len(tf) and tf[fk] < t_next:
                fk += 1
        sub = tf[fj:fk]
        fj = fk
        f, u = st.integrate(s.x[lo:hi], s.y[lo:hi], s.t[lo:hi], s.p[lo:hi],
                            t_frames=sub if len(sub) else None, want_u8=want_u8)
        if f is not None:
            frames.append(f.cpu().numpy())
        if u is not None:
            u8s.append(u.cpu().numpy())
    torch.cuda.synchronize()
    S, T, N, P = (a.cpu().numpy() for a in st.read_state())
    diag = st.diagnostics()
    st.close()
    F = np.concatenate(frames) if frames else None
    U = np.concatenate(u8s) if u8s else None
    return F, U, (S, T, N.view(np.uint32), P), diag


@pytest.mark.parametrize("seed", range(N_CASES))
def test_random_configuration(esi, seed):
    s, prm, tf, calls, tile, scan, want_u8, chunk = _case(seed)
    where = (f"seed {seed}: {s.width}x{s.height}, n {s.n}, calls {calls}, frames {len(tf)}, "
             f"tile {tile}, scan {scan}, chunk {chunk}, params {prm}")
    print(where, flush=True)
    F, U, stg, diag = _gpu(esi, s, prm, tf, calls, tile, scan, want_u8, chunk)
    fo, o = oracle_run(s, prm, t_frames=tf if len(tf) else None)
    assert_state(stg, o, prm["C"], where)
    assert diag["dropped"] == o.dropped, (where, diag, o.dropped)
    if len(tf):
        assert F is not None and F.shape[0] == len(tf), where
        assert_frames(F, fo, prm, where)
        if want_u8:
            assert_u8(U, fo, prm, where)
