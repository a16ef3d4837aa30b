"""The paper's qualitative claims on its two illustrative scenes, checked
with the oracle: Fig. 2's moving disc (Eq. (2) leaves a reversed "ghost" at
the disc's initial position; the decay removes it within 1/k while the disc
stays visible) and Fig. 4's noise-only accumulation (Eq. (2) accumulates
noise; the decay keeps the estimate near its true value, zero change)."""
from __future__ import annotations

import numpy as np

import evgen
import oracle


def _frames(s, prm, tf):
    o = oracle.State(s.width, s.height, oracle.Params(**prm))
    f = o.integrate(s.x, s.y, s.t, s.p, t_frames=np.asarray(tf, np.int64))
    return f, o


def _disc_masks(s, t_us):
    m = s.meta
    yy, xx = np.mgrid[0:s.height, 0:s.width] + 0.5
    yc = s.height / 2.0
    x_now = m["x0"] - m["speed_px_s"] * max(t_us - m["t_start_us"], 0) * 1e-6
    r2 = m["radius"] ** 2
    start = (xx - m["x0"]) ** 2 + (yy - yc) ** 2 < r2
    now = (xx - x_now) ** 2 + (yy - yc) ** 2 < r2
    return start, now


def test_fig2_still_disc_gives_uniform_image():
    s = evgen.moving_circle()
    f, _ = _frames(s, dict(C=0.2, k_per_us=0.0, b=2.0, s_min=-10.0, s_max=10.0), [50_000])
    assert np.all(f[0] == f[0, 0, 0])


def test_fig2_ghost_persists_without_decay():
    """Eq. (2) (k = 0): once the disc has left its initial position, those
    pixels show +floor(log(1/0.3)/C) C (brighter than the background the
    disc passed over, which returns to 0), the disc itself the opposite."""
    s = evgen.moving_circle()
    C, steps = 0.2, s.meta["steps"]
    prm = dict(C=C, k_per_us=0.0, b=2.0, s_min=-10.0, s_max=10.0)
    t_end = 350_000
    f, _ = _frames(s, prm, [t_end])
    S = f[0] * (prm["s_max"] - prm["s_min"]) + prm["s_min"]   # the state at t_end
    start, now = _disc_masks(s, t_end)
    ghost = start & ~now
    assert ghost.sum() > 100 and now.sum() > 100
    core_g = ghost & _shrink(ghost)
    core_n = now & _shrink(now)
    assert np.allclose(S[core_g], steps * C, atol=1e-12)
    assert np.allclose(S[core_n], -steps * C, atol=1e-12)
    assert np.allclose(S[~start & ~now & _shrink(~start & ~now)], 0.0, atol=1e-12)


def test_fig2_decay_removes_the_ghost():
    """With the decay (k = 1 / 120 ms, longer than the 100 ms the disc takes
    to cross a pixel) a decayed frame taken 1/k after the disc left a pixel
    shows exactly the background there (Eq. (4) is 0 for k dt >= 1), while
    the moving disc is still darker than its surround."""
    s = evgen.moving_circle()
    k = 1.0 / 120_000
    prm = dict(C=0.2, k_per_us=k, b=2.0, s_min=-10.0, s_max=10.0)
    m = s.meta
    # the disc has left every initial pixel by t_start + 2R / v
    t_left = m["t_start_us"] + 2 * m["radius"] / m["speed_px_s"] * 1e6
    t_f = int(t_left + 1.0 / k) + 1
    f, o = _frames(s, prm, [t_f])
    F = f[0]
    bg = (0.0 - prm["s_min"]) / (prm["s_max"] - prm["s_min"])
    start, now = _disc_masks(s, t_f)
    ghost = start & ~now
    assert ghost.sum() > 100
    assert np.all(F[ghost] == bg)
    core_n = now & _shrink(now)
    assert np.all(F[core_n] < bg)


def _shrink(mask):
    """Pixels whose 4-neighbours are all in the mask (drops the rim, where a
    disc edge through a pixel centre is ambiguous)."""
    m = mask.copy()
    m[1:, :] &= mask[:-1, :]
    m[:-1, :] &= mask[1:, :]
    m[:, 1:] &= mask[:, :-1]
    m[:, :-1] &= mask[:, 1:]
    m[0, :] = m[-1, :] = False
    m[:, 0] = m[:, -1] = False
    return m


def test_fig4_noise_accumulates_without_decay_and_not_with_it():
    """Noise only for 2 s (the true change is 0 everywhere): log(|S| + 1) of
    Eq. (2)'s estimate is nonzero at most pixels and large at hot pixels;
    with the decay (k = 1 / 100 ms) the decayed estimate at 2 s is zero at
    most pixels and far smaller on average."""
    s = evgen.noise_only()
    wide = dict(C=0.2, b=2.0, s_min=-1e6, s_max=1e6)
    _, o0 = _frames(s, dict(wide, k_per_us=0.0), [])
    f1, o1 = _frames(s, dict(wide, k_per_us=1e-5), [s.duration_us])
    img0 = np.log(np.abs(o0.S) + 1.0)
    S1 = f1[0].reshape(-1) * (wide["s_max"] - wide["s_min"]) + wide["s_min"]
    img1 = np.log(np.abs(S1) + 1.0)
    assert (img0 > 0).mean() > 0.7
    assert (np.abs(S1) > 1e-6).mean() < 0.3
    assert img1.mean() < 0.25 * img0.mean()
    hot = np.array(s.meta["hot"])
    assert img0[hot].min() > 1.0
