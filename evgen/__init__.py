"""Seeded synthetic event streams (inputs for both the GPU path and the oracle).

This package holds no part of the integration method: only an ideal
event-camera forward model (``evgen.c``) and small numpy generators for
adversarial test streams.  Streams are structure-of-arrays numpy arrays
``x`` (uint16), ``y`` (uint16), ``t`` (int64 microseconds), ``p`` (int8,
+1/-1), time-sorted unless a generator says otherwise.

Workloads (sizes, rates, structure):
  c1  346x260, 1 s, drifting sinusoidal grating (period 40 px, 200 px/s),
      C = 0.2, about 0.95M scene events plus 5% uniform noise, seed 1.
  c2  640x480, 10 s, random-walk translating texture (8 random 2-D
      sinusoids in log intensity), per-pixel C ~ N(0.2, 0.02) clipped to
      [0.15, 0.25], about 18M scene events plus 10% Poisson noise, seed 2.
  c3  1280x720, 5 s, rotating radial spokes (20 rev/s, 4 spokes, 1 px
      edges), C = 0.2, about 150M events, seed 3.
  c3hot  c3 plus hot pixels: 0.01% of pixels firing at 10-100 kHz.
Frame times: every 10 ms (100 FPS) or 1 ms (1000 FPS), t_f = (j+1) * period.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "evgen.c")
_LIB = os.path.join(_HERE, "libevgen.so")


def build(out: str = _LIB) -> str:
    cmd = ["gcc", "-O3", "-std=gnu99", "-mavx2", "-mfma", "-fPIC", "-shared", "-pthread",
           "-Wall", "-ffp-contract=off", "-o", out, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("scene", ctypes.c_int32), ("W", ctypes.c_int32), ("H", ctypes.c_int32),
        ("threads", ctypes.c_int32), ("duration_us", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
        ("C_mean", ctypes.c_double), ("C_sigma", ctypes.c_double),
        ("C_lo", ctypes.c_double), ("C_hi", ctypes.c_double),
        ("target_scene_events", ctypes.c_double), ("amplitude", ctypes.c_double),
        ("noise_fraction", ctypes.c_double), ("step_us", ctypes.c_double),
        ("grating_period_px", ctypes.c_double), ("grating_speed_px_s", ctypes.c_double),
        ("tex_speed_px_s", ctypes.c_double), ("tex_vel_tau_s", ctypes.c_double),
        ("tex_lambda_lo", ctypes.c_double), ("tex_lambda_hi", ctypes.c_double),
        ("spoke_rev_s", ctypes.c_double), ("spoke_radius_frac", ctypes.c_double),
        ("spoke_edge_px", ctypes.c_double), ("spoke_count", ctypes.c_int32),
        ("hot_fraction", ctypes.c_double), ("hot_rate_hz", ctypes.c_double),
        ("hot_rate_hi_hz", ctypes.c_double), ("tune", ctypes.c_int32),
    ]


SCENES = {"grating": 0, "texture": 1, "spokes": 2, "none": 3}


@dataclass
class StreamSpec:
    scene: str = "grating"
    width: int = 346
    height: int = 260
    duration_us: int = 1_000_000
    seed: int = 1
    C_mean: float = 0.2
    C_sigma: float = 0.0
    C_lo: float = 0.15
    C_hi: float = 0.25
    target_scene_events: float = 0.95e6
    amplitude: float = 0.15
    noise_fraction: float = 0.0
    step_us: float = 100.0
    grating_period_px: float = 40.0
    grating_speed_px_s: float = 200.0
    tex_speed_px_s: float = 150.0
    tex_vel_tau_s: float = 0.5
    tex_lambda_lo: float = 24.0
    tex_lambda_hi: float = 160.0
    spoke_rev_s: float = 20.0
    spoke_radius_frac: float = 0.45
    spoke_edge_px: float = 1.0
    spoke_count: int = 4
    hot_fraction: float = 0.0
    hot_rate_hz: float = 0.0
    hot_rate_hi_hz: float = 0.0
    tune: bool = False


PRESETS = {
    # One scene parameter was tuned (tune=True) to hit target_scene_events and
    # is stored here: the grating amplitude, the texture speed (rms px/s per
    # axis; amplitude 1.5 fixed), the spoke disc radius (amplitude 0.16: one
    # event per edge passage).  tests/test_evgen.py re-tunes and checks.
    "c1": StreamSpec(scene="grating", width=346, height=260, duration_us=1_000_000,
                     seed=1, amplitude=0.2012, target_scene_events=0.95e6,
                     noise_fraction=0.05),
    "c2": StreamSpec(scene="texture", width=640, height=480, duration_us=10_000_000,
                     seed=2, amplitude=1.5, tex_speed_px_s=19.9459, C_sigma=0.02,
                     target_scene_events=18e6, noise_fraction=0.10, step_us=500.0),
    "c3": StreamSpec(scene="spokes", width=1280, height=720, duration_us=5_000_000,
                     seed=3, amplitude=0.16, spoke_radius_frac=349.5185 / 720,
                     target_scene_events=150e6, noise_fraction=0.0),
}
# The stress variant of c3 (not a measured configuration of its own): the same
# stream plus hot pixels, 0.01% of the sensor firing at 10-100 kHz each
# (log-uniform), which gives runs of 10^4 and more events at one pixel.
PRESETS["c3hot"] = StreamSpec(**{**PRESETS["c3"].__dict__, "hot_fraction": 1e-4,
                                 "hot_rate_hz": 10e3, "hot_rate_hi_hz": 100e3})

# Integrator parameters used with these workloads (the paper gives C only).
DEFAULT_PARAMS = dict(C=0.2, k_per_us=2e-6, b=2.0, s_min=-1.0, s_max=1.0, t0_us=0, flags=0)


@dataclass
class Stream:
    x: np.ndarray
    y: np.ndarray
    t: np.ndarray
    p: np.ndarray
    width: int
    height: int
    duration_us: int
    tuned: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.size)

    def frame_times(self, fps: float = 100.0) -> np.ndarray:
        period = int(round(1e6 / fps))
        nf = self.duration_us // period
        return (np.arange(1, nf + 1, dtype=np.int64) * period)

    def slice(self, lo: int, hi: int) -> "Stream":
        return Stream(self.x[lo:hi], self.y[lo:hi], self.t[lo:hi], self.p[lo:hi],
                      self.width, self.height, self.duration_us, self.tuned,
                      dict(self.meta))


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.evgen_generate.argtypes = [ctypes.POINTER(_Cfg), ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_double)]
        lib.evgen_generate.restype = ctypes.c_void_p
        lib.evgen_fetch.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 4
        lib.evgen_fetch.restype = None
        _lib = lib
    return _lib


def default_threads() -> int:
    env = os.environ.get("EVGEN_THREADS")
    if env:
        return max(1, int(env))
    return max(1, min(os.cpu_count() or 1, 16))


def generate(spec: StreamSpec, threads: int | None = None) -> Stream:
    lib = _load()
    c = _Cfg()
    c.scene = SCENES[spec.scene]
    c.W, c.H = spec.width, spec.height
    c.threads = threads or default_threads()
    c.duration_us, c.seed = spec.duration_us, spec.seed
    for name in ("C_mean", "C_sigma", "C_lo", "C_hi", "target_scene_events",
                 "amplitude", "noise_fraction", "step_us", "grating_period_px",
                 "grating_speed_px_s", "tex_speed_px_s", "tex_vel_tau_s",
                 "tex_lambda_lo", "tex_lambda_hi", "spoke_rev_s",
                 "spoke_radius_frac", "spoke_edge_px", "hot_fraction", "hot_rate_hz",
                 "hot_rate_hi_hz"):
        setattr(c, name, float(getattr(spec, name)))
    c.spoke_count = int(spec.spoke_count)
    c.tune = 1 if spec.tune else 0
    n = ctypes.c_int64(0)
    amp = ctypes.c_double(0.0)
    h = lib.evgen_generate(ctypes.byref(c), ctypes.byref(n), ctypes.byref(amp))
    if not h:
        raise RuntimeError("evgen_generate failed")
    N = n.value
    x = np.empty(N, np.uint16)
    y = np.empty(N, np.uint16)
    t = np.empty(N, np.int64)
    p = np.empty(N, np.int8)
    lib.evgen_fetch(h, x.ctypes.data, y.ctypes.data, t.ctypes.data, p.ctypes.data)
    return Stream(x, y, t, p, spec.width, spec.height, spec.duration_us, amp.value,
                  {"scene": spec.scene, "seed": spec.seed})


def preset(name: str, **overrides) -> Stream:
    spec = PRESETS[name]
    if overrides:
        spec = StreamSpec(**{**spec.__dict__, **overrides})
    return generate(spec)


# ---------------------------------------------------------------------------
# Many independent streams (batched workload)
# ---------------------------------------------------------------------------

# Per resolution: the scene of the single-stream workload of that size, its
# event rate at the stored parameters (events/s), and the scene parameter
# that the rate scales with (event counts grow linearly with it).
_BATCH_SCENES = {
    (346, 260): ("c1", 1.0e6, "grating_speed_px_s"),
    (640, 480): ("c2", 1.99e6, "tex_speed_px_s"),
    (1280, 720): ("c3", 30.6e6, "spoke_rev_s"),
}


def preset_batch(name: str = "c4", duration_us: int = 200_000, n_streams: int | None = None,
                 threads: int | None = None) -> list[Stream]:
    """The batched and served workloads: independent streams, resolution
    drawn uniformly from 346x260, 640x480 and 1280x720, event rate lognormal
    with median 1.41 Mevents/s and sigma 1.03 (0.1 and 20 Mevents/s at the
    0.5% and 99.5% points), clipped to [0.1, 20] Mevents/s; each stream is
    the scene of the single-stream workload of its size with its speed scaled
    to the drawn rate (not re-tuned: rates land near the target).  c4: 64
    streams, stream s with seed 4000 + s; c5: 256 sessions, seed 5000 + s."""
    if name not in ("c4", "c5"):
        raise KeyError(name)
    wl = 4 if name == "c4" else 5
    if n_streams is None:
        n_streams = 64 if wl == 4 else 256
    rng = np.random.default_rng(wl)
    sizes = list(_BATCH_SCENES)
    out = []
    for s in range(n_streams):
        W, H = sizes[int(rng.integers(0, len(sizes)))]
        rate = float(np.clip(rng.lognormal(np.log(1.41e6), 1.03), 0.1e6, 20e6))
        base, base_rate, knob = _BATCH_SCENES[(W, H)]
        spec = PRESETS[base]
        # the noise share is taken of target_scene_events: scaled to this
        # stream's scene events
        scene_events = rate * duration_us * 1e-6 * (1.0 - spec.noise_fraction)
        spec = StreamSpec(**{**spec.__dict__, "duration_us": int(duration_us),
                             "seed": 1000 * wl + s, "target_scene_events": scene_events,
                             knob: getattr(spec, knob) * rate / base_rate})
        st = generate(spec, threads=threads)
        st.meta.update({"target_rate": rate, "base": base})
        out.append(st)
    return out


# ---------------------------------------------------------------------------
# The paper's qualitative scenes (Sec. III-A, Fig. 2; Sec. III-B, Fig. 4)
# ---------------------------------------------------------------------------

def moving_circle(width: int = 200, height: int = 120, radius: float = 20.0,
                  x0: float = 140.0, speed_px_s: float = 400.0, t_start_us: int = 100_000,
                  duration_us: int = 400_000, reflectivity: float = 0.3,
                  C: float = 0.2) -> Stream:
    """Fig. 2's simulation: intensity rising linearly along x, a disc of the
    given reflectivity starting at (x0, height / 2), still until t_start, then
    moving along -x.  The ramp is static, so only the disc's edge emits
    events: a pixel the disc enters sees its log intensity drop by
    log(1 / reflectivity), i.e. floor(that / C) negative events at the entry
    time (floored to us), and as many positive events when the disc leaves
    it.  Pixels inside the disc at the start only see it leave (the ghost of
    the initial position)."""
    steps = int(np.floor(np.log(1.0 / reflectivity) / C + 1e-9))
    yc = height / 2.0
    xs, ys, ts, ps = [], [], [], []
    for y in range(height):
        dy = y + 0.5 - yc
        if abs(dy) >= radius:
            continue
        h = np.sqrt(radius * radius - dy * dy)
        for x in range(width):
            cx = x + 0.5
            t_in = t_start_us + (x0 - cx - h) / speed_px_s * 1e6
            t_out = t_start_us + (x0 - cx + h) / speed_px_s * 1e6
            if t_in > t_start_us and t_in < duration_us:
                for _ in range(steps):
                    xs.append(x), ys.append(y), ts.append(int(t_in)), ps.append(-1)
            if t_out > t_start_us and t_out < duration_us:
                for _ in range(steps):
                    xs.append(x), ys.append(y), ts.append(int(t_out)), ps.append(1)
    order = np.argsort(np.array(ts, np.int64), kind="stable")
    return Stream(np.array(xs, np.uint16)[order], np.array(ys, np.uint16)[order],
                  np.array(ts, np.int64)[order], np.array(ps, np.int8)[order],
                  width, height, duration_us,
                  meta={"scene": "moving_circle", "steps": steps, "radius": radius, "x0": x0,
                        "speed_px_s": speed_px_s, "t_start_us": t_start_us})


def noise_only(seed: int = 6, width: int = 346, height: int = 260, rate_hz_px: float = 2.0,
               duration_us: int = 2_000_000, hot_pixels: int = 3,
               hot_rate_hz: float = 2000.0) -> Stream:
    """Fig. 4's setting without the thrown object: a static scene, so every
    event is noise.  Per-pixel Poisson noise of random polarity at
    rate_hz_px, plus a few hot pixels firing at hot_rate_hz with random
    polarity; the intensity at the end equals the one at the start."""
    rng = np.random.default_rng(seed)
    npix = width * height
    n = rng.poisson(rate_hz_px * npix * duration_us * 1e-6)
    q = rng.integers(0, npix, n)
    t = rng.integers(0, duration_us, n)
    hq = rng.choice(npix, hot_pixels, replace=False)
    nh = int(hot_rate_hz * duration_us * 1e-6)
    q = np.concatenate([q, np.repeat(hq, nh)])
    t = np.concatenate([t, np.tile(np.linspace(0, duration_us - 1, nh).astype(np.int64),
                                   hot_pixels)])
    p = rng.choice(np.array([-1, 1], np.int8), q.size)
    order = np.argsort(t, kind="stable")
    q, t, p = q[order], t[order], p[order]
    return Stream((q % width).astype(np.uint16), (q // width).astype(np.uint16),
                  t.astype(np.int64), p, width, height, duration_us,
                  meta={"scene": "noise_only", "hot": hq.tolist()})


# ---------------------------------------------------------------------------
# Small adversarial streams for tests (numpy, seeded)
# ---------------------------------------------------------------------------

def random_stream(seed: int, width: int, height: int, n: int, t_max: int,
                  t_min: int = 0, sorted_: bool = True, pol01: bool = False,
                  burst_frac: float = 0.0, oob_frac: float = 0.0) -> Stream:
    """Uniform random pixels and times.  burst_frac of the events are copied
    onto the time of their predecessor (same-t bursts); oob_frac get an
    out-of-range x or y."""
    rng = np.random.default_rng(seed)
    x = rng.integers(0, width, n).astype(np.int64)
    y = rng.integers(0, height, n).astype(np.int64)
    t = rng.integers(t_min, t_max, n).astype(np.int64)
    if sorted_:
        t = np.sort(t)
    if burst_frac > 0 and n > 1:
        idx = np.nonzero(rng.random(n - 1) < burst_frac)[0] + 1
        t[idx] = t[idx - 1]
        if sorted_:
            t = np.maximum.accumulate(t)
    if oob_frac > 0:
        m = rng.random(n) < oob_frac
        half = rng.random(n) < 0.5
        x[m & half] = width + rng.integers(0, 5, int((m & half).sum()))
        y[m & ~half] = height + rng.integers(0, 5, int((m & ~half).sum()))
    p = rng.choice(np.array([-1, 1], np.int8), n)
    if pol01:
        p = (p > 0).astype(np.int8)
    return Stream(x.astype(np.uint16), y.astype(np.uint16), t, p, width, height,
                  int(t_max), meta={"seed": seed})


def hot_pixel_stream(seed: int, width: int, height: int, n_bg: int, t_max: int,
                     hot: list[tuple[int, int]], hot_period_us: int) -> Stream:
    """Background uniform events plus hot pixels firing +1 every
    hot_period_us (long runs at one pixel, all inside one window)."""
    bg = random_stream(seed, width, height, n_bg, t_max)
    xs, ys, ts, ps = [bg.x], [bg.y], [bg.t], [bg.p]
    for (hx, hy) in hot:
        th = np.arange(0, t_max, hot_period_us, dtype=np.int64)
        xs.append(np.full(th.size, hx, np.uint16))
        ys.append(np.full(th.size, hy, np.uint16))
        ts.append(th)
        ps.append(np.ones(th.size, np.int8))
    x = np.concatenate(xs)
    y = np.concatenate(ys)
    t = np.concatenate(ts)
    p = np.concatenate(ps)
    o = np.argsort(t, kind="stable")
    return Stream(x[o], y[o], t[o], p[o], width, height, t_max, meta={"seed": seed})
