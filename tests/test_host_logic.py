"""Host-side logic that needs no GPU: the autotuner's workload key and the
server's per-session memory cost."""
from __future__ import annotations

import pytest


def test_workload_key_mix_and_rate_bucket():
    from paper_2508_02238_amd.tune import workload_key
    sizes = [(640, 480), (346, 260), (640, 480), (1280, 720)]
    mix, bucket = workload_key(sizes, [3000.0, 5000.0])
    assert mix == ((346, 260), (640, 480), (1280, 720))   # sorted, duplicates merged
    assert bucket == 11                                     # mean 4000: floor(log2) = 11
    # powers of two of the mean share a bucket boundary
    assert workload_key(sizes, [4096.0])[1] == 12
    assert workload_key(sizes, [4095.0])[1] == 11
    # empty or tiny windows fall into bucket 0
    assert workload_key(sizes, [])[1] == 0
    assert workload_key(sizes, [0.0, 0.0])[1] == 0
    # with the method parameters: different methods never share a choice
    a = dict(C=0.2, k_per_us=2e-6, b=2.0, s_min=-1.0, s_max=1.0, flags=0)
    b = dict(a, flags=4)
    ka, kb = workload_key(sizes, [4000.0], a), workload_key(sizes, [4000.0], b)
    assert ka != kb and ka[0] == kb[0] and ka[2] == kb[2] == 11
    assert workload_key(sizes, [4000.0], [a, a]) == ka
    assert workload_key(sizes, [4000.0], [a, b]) == workload_key(sizes, [4000.0], [b, a])


def test_session_cost():
    """A session costs its state (24 B/px), its frame ring (4 B/px per slot)
    and the library's scratch bound for its largest packet."""
    import paper_2508_02238_amd as esi
    from paper_2508_02238_amd import serve
    assert serve.STATE_BYTES_PER_PIXEL == 24   # S (f32 pair), T (i64), N, P (i32)
    dev = serve.HipDevice.__new__(serve.HipDevice)   # no GPU needed for the cost
    dev._scratch = {}
    dev.max_packet_events = 1 << 14
    rc, bound = esi.esi_scratch_bound(640, 480, 1 << 14)
    assert rc == esi.ESI_OK
    assert dev.cost(640, 480, 3) == (24 + 4 * 3) * 640 * 480 + bound


def test_scratch_bound():
    """The bound covers the records (8 B per event and a spare), the tile
    histogram of every bucketing range, and the growth margin; it grows with
    the events; invalid sizes are refused."""
    import paper_2508_02238_amd as esi
    rc, b0 = esi.esi_scratch_bound(1280, 720, 0)
    assert rc == esi.ESI_OK and b0 == 0
    rc, b1 = esi.esi_scratch_bound(1280, 720, 100_000)
    rc2, b2 = esi.esi_scratch_bound(1280, 720, 1_000_000)
    assert rc == rc2 == esi.ESI_OK
    assert b1 >= 1.25 * (8 * 100_001) and b2 >= 1.25 * (8 * 1_000_001) and b2 > b1
    assert esi.esi_scratch_bound(0, 720, 10)[0] == esi.ESI_ERR_INVALID_ARG
    assert esi.esi_scratch_bound(1280, 65537, 10)[0] == esi.ESI_ERR_INVALID_ARG
    assert esi.esi_scratch_bound(1280, 720, 1 << 31)[0] == esi.ESI_ERR_INVALID_ARG


@pytest.mark.parametrize("tile", [0, 256, 2048, 100, 4096])
def test_set_tile_pixels_null_state(tile):
    """A null state is refused with ESI_ERR_INVALID_ARG whatever the tile
    size, before any device work."""
    import paper_2508_02238_amd as esi
    assert esi.esi_set_tile_pixels(None, tile) == esi.ESI_ERR_INVALID_ARG
