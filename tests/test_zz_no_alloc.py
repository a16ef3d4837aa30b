"""esi_integrate_window_noalloc (scratch in the library's static device
array, nothing allocated) against esi_integrate_window through the C ABI:
two calls in a row on one state, the second with a smaller input (the
static scratch keeps the first call's contents), frames and state compared
element by element, and both compared with the FP64 oracle.  Also the
host-side rejections: frame times in host memory, and a call whose scratch
exceeds the static array.
"""
from __future__ import annotations

import numpy as np
import pytest

import evgen
from esi_parity import assert_frames, assert_state, oracle_run

pytestmark = pytest.mark.gpu

PRM = dict(C=0.2, k_per_us=2e-6, b=2.0, s_min=-1.0, s_max=1.0)


@pytest.fixture(scope="module")
def esi():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    import paper_2508_02238_amd as m
    return m


def _dev(a, np_dtype=None):
    import torch
    if np_dtype is not None:
        a = a.view(np_dtype)
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _run(esi, fn, st, s, lo, hi, tf, stream):
    import torch
    x, y, t, p = (_dev(s.x[lo:hi], np.int16), _dev(s.y[lo:hi], np.int16), _dev(s.t[lo:hi]),
                  _dev(s.p[lo:hi]))
    tfd = _dev(tf)
    fr = torch.full((len(tf), s.height, s.width), -7.0, dtype=torch.float32, device="cuda")
    u8 = torch.zeros((len(tf), s.height, s.width), dtype=torch.uint8, device="cuda")
    rc = fn(st.handle, x.data_ptr(), y.data_ptr(), t.data_ptr(), p.data_ptr(), hi - lo,
            tfd.data_ptr(), len(tf), fr.data_ptr(), u8.data_ptr(), stream)
    assert rc == esi.ESI_OK, esi.esi_status_string(rc)
    torch.cuda.synchronize()
    return fr.cpu().numpy(), u8.cpu().numpy()


@pytest.mark.parametrize("W,H,n1,n2", [(640, 480, 3_000_000, 400_000),
                                       (346, 260, 700_000, 90_000)])
def test_noalloc_equals_integrate_window(esi, W, H, n1, n2):
    import torch
    s = evgen.random_stream(seed=W + n1, width=W, height=H, n=n1 + n2, t_max=600_000,
                            burst_frac=0.15, oob_frac=0.01)
    t_split = int(s.t[n1])
    tf1 = np.linspace(5_000, t_split - 1, 12).astype(np.int64)
    tf2 = np.linspace(t_split, 600_000, 7).astype(np.int64)
    stream = torch.cuda.current_stream().cuda_stream
    a = esi.State(W, H, **PRM)
    b = esi.State(W, H, **PRM)
    out_a, out_b = [], []
    for lo, hi, tf in ((0, n1, tf1), (n1, n1 + n2, tf2)):
        out_a.append(_run(esi, esi.esi_integrate_window, a, s, lo, hi, tf, stream))
        out_b.append(_run(esi, esi.esi_integrate_window_noalloc, b, s, lo, hi, tf, stream))
    for (fa, ua), (fb, ub) in zip(out_a, out_b):
        # the same kernels on the same schedule: identical results
        assert np.array_equal(fa, fb)
        assert np.array_equal(ua, ub)
    sa = [x.cpu().numpy() for x in a.read_state()]
    sb = [x.cpu().numpy() for x in b.read_state()]
    for xa, xb in zip(sa, sb):
        assert np.array_equal(xa, xb)
    assert a.diagnostics()["dropped"] == b.diagnostics()["dropped"]
    # and both against the oracle
    fo, o = oracle_run(s, PRM, t_frames=np.concatenate([tf1, tf2]))
    S, T, N, P = sb
    assert_state((S, T, N.view(np.uint32), P), o, PRM["C"], f"noalloc {W}x{H}")
    assert_frames(np.concatenate([out_b[0][0], out_b[1][0]]), fo, PRM, f"noalloc {W}x{H}")
    assert b.diagnostics()["dropped"] == o.dropped
    a.close()
    b.close()


def test_noalloc_rejections(esi):
    """Checked on the host before anything is enqueued."""
    import torch
    st = esi.State(1280, 720, **PRM)
    stream = torch.cuda.current_stream().cuda_stream
    n = 9_000_000  # about 72 MB of records: more than the 64 MiB array
    x = torch.zeros(n, dtype=torch.int16, device="cuda")
    y = torch.zeros(n, dtype=torch.int16, device="cuda")
    t = torch.arange(n, dtype=torch.int64, device="cuda")
    p = torch.ones(n, dtype=torch.int8, device="cuda")
    tf = torch.tensor([n], dtype=torch.int64, device="cuda")
    fr = torch.empty((1, 720, 1280), dtype=torch.float32, device="cuda")
    rc = esi.esi_integrate_window_noalloc(st.handle, x.data_ptr(), y.data_ptr(), t.data_ptr(),
                                          p.data_ptr(), n, tf.data_ptr(), 1, fr.data_ptr(),
                                          None, stream)
    assert rc == esi.ESI_ERR_SCRATCH_LIMIT, esi.esi_status_string(rc)
    tf_host = np.array([n], np.int64)
    rc = esi.esi_integrate_window_noalloc(st.handle, x.data_ptr(), y.data_ptr(), t.data_ptr(),
                                          p.data_ptr(), 1000, tf_host.ctypes.data, 1,
                                          fr.data_ptr(), None, stream)
    assert rc == esi.ESI_ERR_INVALID_ARG
    # nothing was enqueued: the state is untouched
    N = st.read_state()[2].cpu().numpy()
    assert int(N.sum()) == 0
    assert st.diagnostics()["poisoned"] == 0
    st.close()
