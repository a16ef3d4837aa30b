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


def test_session_cost():
    from paper_2508_02238_amd import serve
    assert serve.STATE_BYTES_PER_PIXEL == 24   # S (f32 pair), T (i64), N, P (i32)
    srv = serve.Server.__new__(serve.Server)   # no device needed for the cost
    srv.scratch_per_event = 16
    srv.max_packet_events = 1 << 14
    assert srv._cost(640, 480) == 24 * 640 * 480 + 16 * (1 << 14)


@pytest.mark.parametrize("tile", [0, 256, 2048, 100, 4096])
def test_set_tile_pixels_null_state(tile):
    """A null state is refused with ESI_ERR_INVALID_ARG whatever the tile
    size, before any device work."""
    import paper_2508_02238_amd as esi
    assert esi.esi_set_tile_pixels(None, tile) == esi.ESI_ERR_INVALID_ARG
