"""The oracle's row-band runner (used to time the oracle on every host core)
gives the serial oracle's result bit for bit: pixels are independent, so a
thread per band of rows changes nothing but the schedule."""
import numpy as np
import pytest

import evgen
import oracle


@pytest.mark.parametrize("threads", [1, 3, 8, 40])
@pytest.mark.parametrize("flags", [0, 1, 2, 4])
def test_bands_equal_serial(threads, flags):
    s = evgen.random_stream(seed=60 + threads, width=41, height=23, n=40_000, t_max=800_000,
                            burst_frac=0.2, oob_frac=0.03)
    s.t[5000:5003] = s.t[5000:5003][::-1].copy()   # a decreasing time: the flag
    tf = np.arange(1, 25, dtype=np.int64) * 33_000
    prm = oracle.Params(C=0.2, k_per_us=3e-6, b=2.0, s_min=-0.6, s_max=0.8, flags=flags)
    a = oracle.State(s.width, s.height, prm)
    fa = a.integrate(s.x, s.y, s.t, s.p, t_frames=tf, frame_sel=[0, 7, 23])
    b = oracle.State(s.width, s.height, prm)
    fb = b.integrate_rows(s.x, s.y, s.t, s.p, t_frames=tf, frame_sel=[0, 7, 23],
                          threads=threads)
    np.testing.assert_array_equal(fa, fb)
    for u, v in ((a.S, b.S), (a.T, b.T), (a.N, b.N), (a.P, b.P)):
        np.testing.assert_array_equal(u, v)
    assert a.dropped == b.dropped > 0
    assert a.unsorted == b.unsorted
