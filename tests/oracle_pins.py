"""Pins of the FP64 oracle to what the paper and mathematics fix.

Each ``pin_*`` function takes a loaded oracle library (ctypes) and raises
AssertionError when the oracle disagrees with a closed form, a hand-derived
worked value (tests/golden), an invariant, a special case or brute force.
They are collected by ``test_oracle_pins.py`` against the real oracle and by
``test_oracle_mutants.py`` against copies of the oracle with planted
mistakes, each of which must fail at least one pin.

None of the expected values below is computed by the oracle itself: they are
hand-derived numbers, closed forms written independently of the oracle's
event loop (Eq. (2), the geometric sum, the unrolled product of Eq. (5)),
or properties that must hold between two oracle runs.
"""
from __future__ import annotations

import itertools
import json
import math
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _params(d):
    return oracle.Params(C=d["C"], k_per_us=d["k_per_us"], b=d["b"],
                         s_min=d["s_min"], s_max=d["s_max"], t0_us=d["t0_us"],
                         flags=d["flags"])


def _run_golden_stepwise(lib, g):
    """Integrate the golden events one call per event and check S after each."""
    st = oracle.State(g["width"], g["height"], _params(g["params"]), lib=lib)
    tol = g.get("S_tolerance", 0.0)
    for ev, s_exp in zip(g["events"], g["S_after_each"]):
        x, y, t, p = ev
        st.integrate([x], [y], [t], [p], want_frames=False)
        q = y * g["width"] + x
        assert abs(st.S[q] - s_exp) <= tol, (g["cite"][:40], st.S[q], s_exp)
    fin = g["final"]
    q = g["events"][-1][1] * g["width"] + g["events"][-1][0]
    assert st.T[q] == fin["T"] and st.N[q] == fin["N"] and st.P[q] == fin["P"], \
        (st.T[q], st.N[q], st.P[q], fin)
    return st


# --------------------------------------------------------------------------
# Eq. (4) and Eq. (6)
# --------------------------------------------------------------------------

def pin_decay_values(lib):
    g = _load_golden("decay_values.json")
    for c in g["cases"]:
        d = oracle.decay(c["dt"], c["k"], c["b"], lib=lib)
        assert abs(d - c["d"]) <= 1e-15, (c, d)
    e = g["eq6_example"]
    lhs = oracle.decay(e["dt"], e["k"], e["b"], lib=lib) ** e["n"]
    rhs = oracle.decay(e["n"] * e["dt"], e["k"], e["b"], lib=lib)
    assert abs(lhs - e["lhs"]) <= 1e-15 and abs(rhs - e["rhs"]) <= 1e-15
    assert lhs > rhs


def pin_decay_shape(lib):
    """d(0) = 1, d = 0 on [1/k, inf), b = 1 is the line 1 - k t, and d is
    non-increasing in t with values in [0, 1]."""
    rng = np.random.default_rng(11)
    for _ in range(40):
        k = 10 ** rng.uniform(-8, -3)
        b = rng.uniform(0.3, 6.0)
        assert oracle.decay(0, k, b, lib=lib) == 1.0
        cut = float(np.ceil(1.0 / k)) + 1.0       # integer us just past 1/k
        assert oracle.decay(cut, k, b, lib=lib) == 0.0
        assert oracle.decay(3.7 / k, k, b, lib=lib) == 0.0
        assert oracle.decay(cut - 2.0, k, b, lib=lib) > 0.0
        ts = np.sort(rng.uniform(0, 1.0 / k, 16))
        ds = [oracle.decay(t, k, b, lib=lib) for t in ts]
        assert all(0.0 <= v <= 1.0 for v in ds)
        assert all(a >= c for a, c in zip(ds, ds[1:]))
        t1 = float(rng.uniform(0, 1.0 / k))
        lin = oracle.decay(t1, k, 1.0, lib=lib)
        assert abs(lin - (1.0 - k * t1)) <= 1e-15


def pin_eq6_inequality(lib):
    """Eq. (6): d(t)^n > d(nt) for n >= 2, t in (0, 1/(nk))."""
    rng = np.random.default_rng(12)
    for _ in range(200):
        k = 10 ** rng.uniform(-7, -4)
        b = rng.uniform(0.5, 5.0)
        n = int(rng.integers(2, 9))
        t = rng.uniform(0.05, 0.95) / (n * k)
        lhs = oracle.decay(t, k, b, lib=lib) ** n
        rhs = oracle.decay(n * t, k, b, lib=lib)
        assert lhs > rhs, (k, b, n, t, lhs, rhs)


# --------------------------------------------------------------------------
# Worked values (hand-derived, tests/golden)
# --------------------------------------------------------------------------

def pin_golden_add_then_decay(lib):
    g = _load_golden("dyadic_add_then_decay.json")
    st = _run_golden_stepwise(lib, g)
    fr = g["frame"]
    F = st.snapshot(fr["t_us"])[0, 0]
    assert F == fr["F"], F
    assert int(oracle.u8([F], lib=lib)[0]) == fr["u8"]
    lazy = st.copy()
    lazy.params = oracle.Params(**{**st.params.__dict__,
                                   "flags": oracle.SNAPSHOT_LAZY})
    assert lazy.snapshot(fr["t_us"])[0, 0] == fr["F_lazy"]


def pin_golden_decay_then_add(lib):
    _run_golden_stepwise(lib, _load_golden("dyadic_decay_then_add.json"))


def pin_golden_alternating(lib):
    _run_golden_stepwise(lib, _load_golden("alternating_polarity.json"))


def pin_golden_clamp_per_event(lib):
    _run_golden_stepwise(lib, _load_golden("clamp_per_event.json"))


def pin_golden_support_cutoff(lib):
    _run_golden_stepwise(lib, _load_golden("support_cutoff.json"))


# --------------------------------------------------------------------------
# Special cases and closed forms
# --------------------------------------------------------------------------

def _random_stream(rng, W, H, n, t_max, pol01=False):
    x = rng.integers(0, W, n).astype(np.uint16)
    y = rng.integers(0, H, n).astype(np.uint16)
    t = np.sort(rng.integers(0, t_max, n)).astype(np.int64)
    p = rng.choice(np.array([-1, 1], np.int8), n)
    if pol01:
        p = (p > 0).astype(np.int8)
    return x, y, t, p


def pin_k0_is_eq2(lib):
    """k = 0 turns Alg. 2 into Eq. (2): S = C * (signed event count), exactly
    for a dyadic C, with N the count and T the last event time per pixel."""
    rng = np.random.default_rng(13)
    W, H = 7, 5
    x, y, t, p = _random_stream(rng, W, H, 3000, 10**6)
    prm = oracle.Params(C=0.25, k_per_us=0.0, b=2.0, s_min=-1e30, s_max=1e30)
    st = oracle.State(W, H, prm, lib=lib)
    st.integrate(x, y, t, p, want_frames=False)
    q = y.astype(np.int64) * W + x
    sgn = np.where(p > 0, 1, -1)
    Pexp = np.bincount(q, weights=sgn, minlength=W * H).astype(np.int64)
    Nexp = np.bincount(q, minlength=W * H)
    Texp = np.zeros(W * H, np.int64)
    np.maximum.at(Texp, q, t)
    assert np.array_equal(st.P, Pexp) and np.array_equal(st.N, Nexp)
    assert np.array_equal(st.T, Texp)
    assert np.array_equal(st.S, 0.25 * Pexp)


def pin_polarity_encodings(lib):
    """p in {+1,-1} and p in {1,0} describe the same stream."""
    rng = np.random.default_rng(14)
    W, H = 4, 3
    x, y, t, p = _random_stream(rng, W, H, 500, 4 * 10**6)
    prm = oracle.Params(C=0.2, k_per_us=2e-6, b=2.0)
    a = oracle.State(W, H, prm, lib=lib)
    a.integrate(x, y, t, p, want_frames=False)
    b = oracle.State(W, H, prm, lib=lib)
    b.integrate(x, y, t, (p > 0).astype(np.int8), want_frames=False)
    assert np.array_equal(a.S, b.S) and np.array_equal(a.P, b.P)


def pin_constant_rate_geometric(lib):
    """One pixel, n events of polarity +1 every D us, q = d(D):
    add-then-decay S_n = C q (1 - q^n) / (1 - q); decay-then-add
    S_n = C (1 - q^n) / (1 - q); with a clamp at S_max the sequence is
    min(S_n, S_max) (the partial sums increase monotonically)."""
    for (k, b, D, n, C) in [(2e-6, 2.0, 10_000, 300, 0.2),
                            (1e-5, 0.5, 3_000, 200, 0.25),
                            (1e-7, 4.7, 50_000, 150, 0.15)]:
        q = max(1.0 - k * D, 0.0) ** b
        t = np.arange(1, n + 1, dtype=np.int64) * D
        ones = np.ones(n, np.int8)
        zeros = np.zeros(n, np.uint16)
        for flags, geo in [(0, C * q * (1 - q ** n) / (1 - q)),
                           (oracle.DECAY_THEN_ADD, C * (1 - q ** n) / (1 - q))]:
            st = oracle.State(1, 1, oracle.Params(C=C, k_per_us=k, b=b,
                                                  s_min=-1e30, s_max=1e30,
                                                  flags=flags), lib=lib)
            st.integrate(zeros, zeros, t, ones, want_frames=False)
            assert abs(st.S[0] - geo) <= 1e-12 * abs(geo), (k, b, flags, st.S[0], geo)
            smax = 0.5 * geo
            st = oracle.State(1, 1, oracle.Params(C=C, k_per_us=k, b=b,
                                                  s_min=-1e30, s_max=smax,
                                                  flags=flags), lib=lib)
            st.integrate(zeros, zeros, t, ones, want_frames=False)
            assert st.S[0] == smax


def _closed_form_eq5(C, k, b, pols, times, t0, decay_then_add):
    """The unrolled recurrence under Eq. (5) without clamping:
    add-then-decay S_n = C sum_i p_i prod_{j=i..n} d(t_j - t_{j-1}),
    decay-then-add uses prod_{j=i+1..n}; t_0 is the initial T."""
    dl = [max(1.0 - k * (times[j] - (times[j - 1] if j else t0)), 0.0) ** b
          for j in range(len(times))]
    s = 0.0
    for i in range(len(times)):
        prod = 1.0
        for j in range(i + 1 if decay_then_add else i, len(times)):
            prod *= dl[j]
        s += C * pols[i] * prod
    return s


def pin_brute_force_eq5(lib):
    """Every polarity sequence of length 1..4 with every gap from
    {0, 1/(4k), 1/(2k), 1/k, 2/k}: one run per pixel of one sensor, checked
    against the closed form of Eq. (5) (both orders, no clamp hit)."""
    k, b, C = 4e-6, 2.0, 0.25
    gaps = [0, 62_500, 125_000, 250_000, 500_000]
    runs = []
    for L in range(1, 5):
        for pols in itertools.product([1, -1], repeat=L):
            for gs in itertools.product(gaps, repeat=L):
                runs.append((pols, np.cumsum(gs) + 1000))
    npx = len(runs)
    W = 64
    H = (npx + W - 1) // W
    xs, ys, ts, ps = [], [], [], []
    for r, (pols, times) in enumerate(runs):
        for pol, tt in zip(pols, times):
            xs.append(r % W)
            ys.append(r // W)
            ts.append(int(tt))
            ps.append(pol)
    order = np.argsort(np.array(ts), kind="stable")
    x = np.array(xs, np.uint16)[order]
    y = np.array(ys, np.uint16)[order]
    t = np.array(ts, np.int64)[order]
    p = np.array(ps, np.int8)[order]
    for flags in (0, oracle.DECAY_THEN_ADD):
        st = oracle.State(W, H, oracle.Params(C=C, k_per_us=k, b=b, s_min=-1e30,
                                              s_max=1e30, flags=flags), lib=lib)
        st.integrate(x, y, t, p, want_frames=False)
        for r, (pols, times) in enumerate(runs):
            ref = _closed_form_eq5(C, k, b, pols, times, 0, flags != 0)
            assert abs(st.S[r] - ref) <= 1e-13, (pols, times, flags, st.S[r], ref)
            assert st.N[r] == len(pols) and st.P[r] == sum(pols)
            assert st.T[r] == times[-1]


def pin_clamp_saturation(lib):
    """Closed forms of the per-event clamp (Eq. (13) inside Alg. 2's loop),
    independent of any history: a burst of m same-time +1 events with
    m C >= S_max - S_min leaves S at exactly S_max (d(0) = 1: every add is
    followed by the clamp), a -1 burst at exactly S_min; from that saturated
    state a run that stays inside the bounds follows the unrolled sum of
    Eq. (5) started at S_max (add then decay: S_n = S_max prod d_j +
    C sum p_i prod_{j >= i} d_j; decay then add: S_max prod d_j +
    C sum p_i prod_{j > i} d_j).  Dyadic values (C = 1/4, bounds -1/2 and
    3/4, kD in {0, 1/4, 1/2}, b = 2): exact equality.  A clamp applied at
    the output only, or before the add, leaves S outside the bounds after
    the burst."""
    rng = np.random.default_rng(15)
    C, lo, hi, k = 0.25, -0.5, 0.75, 1e-6
    m = 6                                   # 6 C = 1.5 >= hi - lo = 1.25
    gaps = [0, 250_000, 500_000]            # k D in {0, 1/4, 1/2}
    for flags in (0, 1):
        for sign in (1, -1):
            W, H = 3, 2
            xs, ys, ts, ps = [], [], [], []
            expect = {}
            for q in range(W * H):
                x, y = q % W, q // W
                t = int(rng.integers(1_000, 50_000))
                # history: a few random events before the burst
                for _ in range(int(rng.integers(0, 4))):
                    t += int(rng.integers(0, 300_000))
                    xs.append(x); ys.append(y); ts.append(t)
                    ps.append(int(rng.choice([-1, 1])))
                t += int(rng.integers(1, 100_000))
                for _ in range(m):                      # the saturating burst
                    xs.append(x); ys.append(y); ts.append(t); ps.append(sign)
                S = hi if sign > 0 else lo
                # a run inside the bounds: polarities back towards 0 first
                seq = [-sign, sign, -sign, -sign, sign][:int(rng.integers(0, 6))]
                prods, terms = [], []
                for pol in seq:
                    t += gaps[int(rng.integers(0, 3))]
                    xs.append(x); ys.append(y); ts.append(t); ps.append(pol)
                run_t = ts[len(ts) - len(seq) - 1:]        # burst time, then the run
                d = [(1.0 - k * (run_t[j + 1] - run_t[j])) ** 2 for j in range(len(seq))]
                # Eq. (5) from the saturated state, both orders, exact
                tot = S
                for j in range(len(seq)):
                    tot *= d[j]
                for i, pol in enumerate(seq):
                    w = 1.0
                    for j in range(i if flags == 0 else i + 1, len(seq)):
                        w *= d[j]
                    tot += C * pol * w
                # the run must stay within the bounds (the clamp a no-op) for the form to hold
                part = S
                for i, pol in enumerate(seq):
                    part = (part + C * pol) * d[i] if flags == 0 else part * d[i] + C * pol
                    assert lo <= part <= hi
                expect[q] = tot
            order = np.argsort(np.array(ts), kind="stable")
            st = oracle.State(W, H, oracle.Params(C=C, k_per_us=k, b=2.0, s_min=lo, s_max=hi,
                                                  flags=flags), lib=lib)
            st.integrate(np.array(xs, np.uint16)[order], np.array(ys, np.uint16)[order],
                         np.array(ts, np.int64)[order], np.array(ps, np.int8)[order],
                         want_frames=False)
            for q, v in expect.items():
                assert st.S[q] == v, (flags, sign, q, st.S[q], v)


def pin_linearity_symmetry(lib):
    """With no clamp hit, S is linear in C (doubling C doubles S exactly)
    and flipping every polarity negates S exactly."""
    rng = np.random.default_rng(16)
    W, H = 5, 4
    x, y, t, p = _random_stream(rng, W, H, 2000, 3 * 10**6)
    base = dict(k_per_us=3e-6, b=1.7, s_min=-1e30, s_max=1e30)
    a = oracle.State(W, H, oracle.Params(C=0.2, **base), lib=lib)
    a.integrate(x, y, t, p, want_frames=False)
    b2 = oracle.State(W, H, oracle.Params(C=0.4, **base), lib=lib)
    b2.integrate(x, y, t, p, want_frames=False)
    neg = oracle.State(W, H, oracle.Params(C=0.2, **base), lib=lib)
    neg.integrate(x, y, t, (-p).astype(np.int8), want_frames=False)
    assert np.array_equal(b2.S, 2.0 * a.S)
    assert np.array_equal(neg.S, -a.S)
    assert np.array_equal(neg.P, -a.P)


def pin_pixel_independence(lib):
    """Alg. 2 touches only the event's own pixel: any interleaving of the
    pixels' runs that keeps each pixel's order gives the same state."""
    rng = np.random.default_rng(17)
    W, H = 6, 6
    x, y, t, p = _random_stream(rng, W, H, 3000, 2 * 10**6)
    prm = oracle.Params(C=0.2, k_per_us=2e-6, b=2.0, s_min=-0.5, s_max=0.8)
    a = oracle.State(W, H, prm, lib=lib)
    a.integrate(x, y, t, p, want_frames=False)
    q = y.astype(np.int64) * W + x
    order = np.argsort(q, kind="stable")          # pixel-major, order kept per pixel
    b = oracle.State(W, H, prm, lib=lib)
    b.integrate(x[order], y[order], t[order], p[order], want_frames=False)
    assert np.array_equal(a.S, b.S) and np.array_equal(a.T, b.T)
    assert np.array_equal(a.N, b.N) and np.array_equal(a.P, b.P)


def pin_window_split_and_fps(lib):
    """Integrating in one call or in many gives the same state, and frames at
    100 and 1000 FPS agree at the shared times (frames are read-only)."""
    rng = np.random.default_rng(18)
    W, H = 9, 7
    x, y, t, p = _random_stream(rng, W, H, 5000, 10**6)
    prm = oracle.Params(C=0.2, k_per_us=2e-6, b=2.0)
    tf100 = np.arange(1, 101, dtype=np.int64) * 10_000
    tf1000 = np.arange(1, 1001, dtype=np.int64) * 1_000
    a = oracle.State(W, H, prm, lib=lib)
    fa = a.integrate(x, y, t, p, t_frames=tf100)
    b = oracle.State(W, H, prm, lib=lib)
    fb = b.integrate(x, y, t, p, t_frames=tf1000)
    assert np.array_equal(fa, fb[9::10])
    c = oracle.State(W, H, prm, lib=lib)
    cuts = np.sort(rng.integers(0, len(t), 7))
    for lo, hi in zip(np.r_[0, cuts], np.r_[cuts, len(t)]):
        c.integrate(x[lo:hi], y[lo:hi], t[lo:hi], p[lo:hi], want_frames=False)
    assert np.array_equal(a.S, c.S) and np.array_equal(a.T, c.T)
    assert np.array_equal(a.N, c.N) and np.array_equal(a.P, c.P)


def pin_frame_membership(lib):
    """A frame at t_f holds the events with t <= t_f (Eq. (5)'s t_n <= t):
    an event exactly at t_f is in it, one at t_f + 1 is not."""
    prm = oracle.Params(C=0.25, k_per_us=0.0, b=1.0)
    st = oracle.State(2, 1, prm, lib=lib)
    f = st.integrate([0, 1], [0, 0], [100, 101], [1, 1], t_frames=[100, 101])
    assert f[0, 0, 0] == (0.25 + 1) / 2 and f[0, 0, 1] == 0.5
    assert f[1, 0, 1] == (0.25 + 1) / 2


def pin_event_free_window(lib):
    """With no event after T, a frame at t_f shows clamp(S d(t_f - T))
    (decayed snapshot; here exact dyadic values), and the lazy frame shows S."""
    prm = oracle.Params(C=0.5, k_per_us=1e-6, b=1.0, s_min=-1.0, s_max=1.0)
    st = oracle.State(1, 1, prm, lib=lib)
    frames = st.integrate([0], [0], [0], [1], t_frames=[0, 250_000, 500_000,
                                                        750_000, 10**6, 2 * 10**6])
    # S = 0.5 at T = 0; d(t) = 1 - t/1e6
    exp = [0.5, 0.375, 0.25, 0.125, 0.0, 0.0]
    assert np.array_equal(frames[:, 0, 0], (np.array(exp) + 1) / 2)
    lazy = oracle.State(1, 1, oracle.Params(**{**prm.__dict__, "flags": oracle.SNAPSHOT_LAZY}),
                        lib=lib)
    fl = lazy.integrate([0], [0], [0], [1], t_frames=[0, 10**6])
    assert np.array_equal(fl[:, 0, 0], [0.75, 0.75])


def pin_dropped_unsorted(lib):
    """Out-of-range events are dropped and counted; a decreasing time sets
    the flag and gives dt = 0 (d = 1), and T follows the event."""
    prm = oracle.Params(C=0.25, k_per_us=1e-6, b=1.0, s_min=-1.0, s_max=1.0)
    st = oracle.State(3, 2, prm, lib=lib)
    st.integrate([0, 3, 1, 0], [0, 0, 2, 0], [500_000, 500_001, 500_002, 250_000],
                 [1, 1, 1, 1], want_frames=False)
    assert st.dropped == 2 and st.unsorted
    # first: (0 + .25) * (1 - .5) = .125 ; second at an earlier time: d = 1
    assert st.S[0] == 0.375 and st.T[0] == 250_000 and st.N[0] == 2
    assert st.N.sum() == 2


def pin_u8_code(lib):
    """Eq. (14): B = 255 (S - S_min)/(S_max - S_min) as an 8-bit code,
    rounded half up."""
    F = np.array([0.0, 1.0, 0.5, 0.5546875, 1.0 / 255, 0.25 / 255, 0.75 / 255])
    assert list(oracle.u8(F, lib=lib)) == [0, 255, 128, 141, 1, 0, 1]


def pin_asymmetric_clamp_frames(lib):
    """Eq. (13)-(14) with asymmetric bounds [-0.5, 1.5]: a single event of
    C = 1 at t = 0 and k = 1e-6, b = 1 gives S = 1; frames at 0, 0.5 s and
    1 s show (v + 0.5) / 2 for v = 1, 0.5, 0; an event of C = 1 on a pixel at
    S = 1.5 stays clamped at 1.5 and shows (0.75 + 0.5) / 2 at 0.5 s (exact
    dyadic values)."""
    prm = oracle.Params(C=1.0, k_per_us=1e-6, b=1.0, s_min=-0.5, s_max=1.5)
    st = oracle.State(2, 1, prm, lib=lib)
    f = st.integrate([0, 1, 1], [0, 0, 0], [0, 0, 0], [1, 1, 1],
                     t_frames=[0, 500_000, 10**6])
    assert np.array_equal(f[:, 0, 0], [0.75, 0.5, 0.25]), f[:, 0, 0]
    assert st.S[1] == 1.5 and f[0, 0, 1] == 1.0 and f[1, 0, 1] == 0.625


def pin_stream_origin(lib):
    """T starts at the stream origin t0: with t0 = 10 s, an event at
    t0 + 0.25 s (k = 2e-6, b = 1, C = 0.25) decays by d(0.25 s) = 0.5 and
    gives S = 0.125; measured from 0 it would decay to exactly 0."""
    prm = oracle.Params(C=0.25, k_per_us=2e-6, b=1.0, t0_us=10_000_000)
    st = oracle.State(1, 1, prm, lib=lib)
    assert st.T[0] == 10_000_000
    st.integrate([0], [0], [10_250_000], [1], want_frames=False)
    assert st.S[0] == 0.125


def pin_exp_decay_values(lib):
    """The accumulator plugin's decay exp(-k t): 1 at 0, e^-1 at 1/k, e^-2 at
    2/k, a semigroup (d(a + b) = d(a) d(b)), 1 for k = 0, and no cutoff
    (still positive at 40/k, where Eq. (4) is 0)."""
    k = 2e-6
    assert oracle.decay_exp(0.0, k, lib=lib) == 1.0
    for m in (1, 2, 5):
        want = math.exp(-m)
        assert abs(oracle.decay_exp(m / k, k, lib=lib) - want) <= 1e-15 * want
    for a, b in [(1234.0, 98765.0), (5e5, 2.5e5), (0.0, 7e5)]:
        lhs = oracle.decay_exp(a + b, k, lib=lib)
        rhs = oracle.decay_exp(a, k, lib=lib) * oracle.decay_exp(b, k, lib=lib)
        assert abs(lhs - rhs) <= 4e-16 * lhs
    assert oracle.decay_exp(1e9, 0.0, lib=lib) == 1.0
    assert oracle.decay_exp(40 / k, k, lib=lib) > 0.0


def pin_exp_constant_rate_geometric(lib):
    """Exponential decay, one pixel, n events of +1 every D us: the geometric
    sums of the constant-rate pin with q = exp(-k D)."""
    for (k, D, n, C) in [(2e-6, 10_000, 300, 0.2), (1e-4, 3_000, 50, 0.25)]:
        q = math.exp(-k * D)
        t = np.arange(1, n + 1, dtype=np.int64) * D
        ones = np.ones(n, np.int8)
        zeros = np.zeros(n, np.uint16)
        for flags, geo in [(oracle.DECAY_EXP, C * q * (1 - q ** n) / (1 - q)),
                           (oracle.DECAY_EXP | oracle.DECAY_THEN_ADD, C * (1 - q ** n) / (1 - q))]:
            st = oracle.State(1, 1, oracle.Params(C=C, k_per_us=k, b=2.0, s_min=-1e30,
                                                  s_max=1e30, flags=flags), lib=lib)
            st.integrate(zeros, zeros, t, ones, want_frames=False)
            assert abs(st.S[0] - geo) <= 1e-12 * abs(geo), (k, flags, st.S[0], geo)


def pin_exp_telescoped_sum(lib):
    """With exponential decay the product in Eq. (5) telescopes: without a
    clamp, add-then-decay gives S_n = C sum_i p_i exp(-k (t_n - t_{i-1}))
    (t_0 = the initial T) and decay-then-add S_n = C sum_i p_i
    exp(-k (t_n - t_i)).  Random short runs, one per pixel, gaps including
    0; b is ignored under the flag (checked with two values)."""
    rng = np.random.default_rng(2024)
    k, C, W = 1e-5, 0.2, 40
    n_per = rng.integers(1, 9, W)
    xs, ts, ps = [], [], []
    runs = []
    for q in range(W):
        gaps = rng.choice([0, 1, 50, 20_000, 100_000, 400_000], n_per[q])
        tq = np.cumsum(gaps)
        pq = rng.choice([-1, 1], n_per[q])
        runs.append((tq, pq))
        xs += [q] * len(tq)
        ts += list(tq)
        ps += list(pq)
    order = np.argsort(np.array(ts), kind="stable")
    x = np.array(xs, np.uint16)[order]
    t = np.array(ts, np.int64)[order]
    p = np.array(ps, np.int8)[order]
    for dta in (False, True):
        for b in (2.0, 0.5):
            flags = oracle.DECAY_EXP | (oracle.DECAY_THEN_ADD if dta else 0)
            st = oracle.State(W, 1, oracle.Params(C=C, k_per_us=k, b=b, s_min=-1e30,
                                                  s_max=1e30, flags=flags), lib=lib)
            st.integrate(x, np.zeros_like(x), t, p, want_frames=False)
            for q, (tq, pq) in enumerate(runs):
                tn = float(tq[-1])
                prev = np.concatenate([[0.0], tq[:-1].astype(np.float64)])
                ref = tq.astype(np.float64) if dta else prev
                want = C * float(np.sum(pq * np.exp(-k * (tn - ref))))
                assert abs(st.S[q] - want) <= 1e-12 * max(abs(want), C), (q, dta, st.S[q], want)


def pin_exp_event_free_window(lib):
    """Exponential decay: a frame at t_f with no event after T shows
    S exp(-k (t_f - T)), mapped by Eq. (14)."""
    k = 3e-6
    prm = oracle.Params(C=0.5, k_per_us=k, b=1.0, s_min=-1.0, s_max=1.0,
                        flags=oracle.DECAY_EXP)
    st = oracle.State(1, 1, prm, lib=lib)
    tf = [0, 100_000, 333_333, 10**6, 10**7]
    frames = st.integrate([0], [0], [0], [1], t_frames=tf)
    for j, tj in enumerate(tf):
        want = (0.5 * math.exp(-k * tj) + 1.0) / 2.0
        assert abs(frames[j, 0, 0] - want) <= 1e-15, (tj, frames[j, 0, 0], want)


PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]


def main(argv):
    """Run every pin against the oracle library at argv[1]; print the names of
    the pins that fail and exit with status 3 if any did (used to test
    planted mistakes in a separate process)."""
    lib = oracle.load(argv[1])
    failed = []
    for pin in PINS:
        try:
            pin(lib)
        except (AssertionError, ValueError, OverflowError, ZeroDivisionError):
            failed.append(pin.__name__)
    print("FAILED:", " ".join(failed))
    return 3 if failed else 0


if __name__ == "__main__":
    import sys
    sys.exit(main(sys.argv))
