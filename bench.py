#!/usr/bin/env python3
"""Benchmark of the ESI hot path on one MI355X.

One step = the whole hot path over one batch: reset the per-pixel state,
then one esi_integrate_window call that integrates the workload's whole
event stream (Alg. 2 event loop with the clamp of Eq. (13)) and writes all
of its frames (Eq. (14), decayed snapshots, FP32).  Inputs are resident in
HBM before timing starts.

Default workload (c3, the largest single-stream one): 1280x720 sensor, 5 s
of a seeded rotating radial-spoke pattern at 20 rev/s, about 153M events,
frames at 100 FPS (500 frames).

Prints one JSON line on stdout: Gevents/s integrated (value), frames/s,
the roofline of the call (its algorithmic bytes over the GPU time of the
call, measured with HIP events the library records on its stream, with the
bucketing and integration kernels also reported on their own bytes), the
parity of this run's output against the FP64 oracle, and the oracle itself
timed on the host, on one core and on every core, as a CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(n: int, npix: int, nf: int, u8: bool, f32: bool = True) -> int:
    """Bytes the method itself must move in one whole-stream call: the events
    read once (x, y u16, t i64, p i8 = 13 B), the per-pixel state read and
    written once (S f32, T i64, N u32, P i32 = 20 B each way), every frame
    written once (4 B per pixel as FP32, 1 B as 8-bit codes)."""
    return 13 * n + 40 * npix + ((4 if f32 else 0) + (1 if u8 else 0)) * nf * npix


def measured_traffic(workload: str, fps: float):
    """HBM bytes per call of the call's kernels (bucketing and integration)
    from the committed counter summary (FETCH_SIZE and WRITE_SIZE, each
    scaled by the reading of a plain copy of known size), or None when no
    summary exists for this workload or the kernel sources changed since it
    was taken.  Returns (total, {kernel group: bytes})."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{fps:g}fps.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if _sources_hash(rec["sources"]) != rec["sources_sha256_16"]:
        return None
    groups = {g: int(v["read_bytes"]) + int(v["write_bytes"]) for g, v in rec["groups"].items()}
    return sum(groups.values()), groups


def cpu_baseline(s, tf, prm, sample_s: float, min_s: float, threads: int):
    """The oracle timed on the host over a bounded sample of the workload (its
    first `sample_s` seconds of events and the frames in them): whole passes
    from a fresh state until about min_s seconds, on one core (the serial
    loop) and on `threads` cores (one band of rows per thread, every thread
    scanning all events)."""
    import numpy as np

    import oracle
    m = int(np.searchsorted(s.t, int(sample_s * 1e6), side="left"))
    tf_s = tf[tf <= int(sample_s * 1e6)]
    W, H = s.width, s.height

    def timed(run):
        el, reps = 0.0, 0
        while reps == 0 or (el < min_s and reps < 16):
            o = oracle.State(W, H, oracle.Params(**prm))
            h0 = time.perf_counter()
            run(o)
            el += time.perf_counter() - h0
            reps += 1
        return el, reps

    el1, r1 = timed(lambda o: o.integrate(s.x[:m], s.y[:m], s.t[:m], s.p[:m], t_frames=tf_s))
    elN, rN = timed(lambda o: o.integrate_rows(s.x[:m], s.y[:m], s.t[:m], s.p[:m],
                                                t_frames=tf_s, threads=threads))
    return {"value": round(r1 * m / el1 / 1e9, 6), "unit": "Gevents/s", "cores": 1,
            "kind": "oracle",
            "frames_per_s": round(r1 * len(tf_s) / el1, 2),
            "all_cores": {"value": round(rN * m / elN / 1e9, 6), "unit": "Gevents/s",
                          "cores": threads, "frames_per_s": round(rN * len(tf_s) / elN, 2),
                          "method": "one band of rows per thread, each scanning all events",
                          "seconds": round(elN, 2), "passes": rN},
            "sample": (f"the first {sample_s:g} s of the workload ({m} events, {len(tf_s)} "
                       f"frames), serial FP64 oracle, {r1} pass(es) in {el1:.1f} s on one core"),
            "cpu_model": _cpu_model()}


TRAFFIC_SOURCES = ["paper_2508_02238_amd/csrc/bucket.hip", "paper_2508_02238_amd/csrc/integrate.hip",
                   "paper_2508_02238_amd/csrc/esi_device.hpp",
                   "paper_2508_02238_amd/csrc/esi_internal.hpp"]


def _sources_hash(sources) -> str:
    import hashlib
    h = hashlib.sha256()
    for src in sources:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _short_kernel_name(name: str) -> str:
    """k_bucket<8192, 8> from 'void esi::(anonymous namespace)::k_bucket<8192, 8>(...)'."""
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0].replace("esi::", "")


def _counter_means(path: str) -> dict:
    """Mean counter value (KiB) per kernel name over its dispatches, from a
    rocprofv3 counter_collection CSV; the copy probe's dispatches kept apart."""
    import csv
    import collections
    vals = collections.defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return vals


def write_traffic(workload: str, fps: float, fetch_csv: str, write_csv: str, probe_mb: int):
    """The bucketing and integration kernels' HBM bytes per call from two
    rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each
    scaled by what the counter reads for the plain copy of probe_mb MiB the
    run ended with: written to profiles/traffic_<workload>_<fps>fps.json
    with the hash of the kernel sources (bench.py reports null once they
    change); returns the per-kernel table."""
    fetch, write = _counter_means(fetch_csv), _counter_means(write_csv)
    copy = "__amd_rocclr_copyBuffer"
    probe_kib = probe_mb * 1024.0
    f_scale = probe_kib / max(fetch[copy])
    w_scale = probe_kib / max(write[copy])
    groups = {"bucketing": ("k_hist", "k_seg_sum", "k_seg_down", "k_order", "k_bucket"),
              "integration": ("k_integrate",)}
    out = {"workload": workload, "fps": fps, "fetch_scale": round(f_scale, 4),
           "write_scale": round(w_scale, 4), "groups": {}, "kernels": {},
           "sources": TRAFFIC_SOURCES, "sources_sha256_16": _sources_hash(TRAFFIC_SOURCES)}
    for name in fetch:
        short = _short_kernel_name(name)
        if not short.startswith(("k_", "kb_")):
            continue   # the copy probe and torch's own kernels
        rb = sum(fetch[name]) / len(fetch[name]) * 1024 * f_scale
        wb = sum(write.get(name, [0.0])) / max(1, len(write.get(name, []))) * 1024 * w_scale
        out["kernels"][short] = {"read_bytes": int(rb), "write_bytes": int(wb),
                                 "dispatches": len(fetch[name])}
        for g, members in groups.items():
            if any(short.startswith(m) for m in members):
                acc = out["groups"].setdefault(g, {"read_bytes": 0, "write_bytes": 0})
                acc["read_bytes"] += int(rb)
                acc["write_bytes"] += int(wb)
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{fps:g}fps.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    return out


def kernel_stats_table(stats_csv: str) -> str:
    """Markdown table of a rocprofv3 --stats kernel summary."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    lines = ["| kernel | calls | average (us) | min (us) | max (us) | share of GPU time |",
             "|---|---|---|---|---|---|"]
    for r in rows:
        name = _short_kernel_name(r["Name"])
        lines.append(f"| {name} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.1f}% |")
    return "\n".join(lines)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3",
                    choices=["c1", "c2", "c3", "c3hot", "c4", "c5"])
    ap.add_argument("--fps", type=float, default=100.0)
    ap.add_argument("--u8", action="store_true", help="also write 8-bit frames")
    ap.add_argument("--u8-only", action="store_true", help="write 8-bit frames only")
    ap.add_argument("--tile-pixels", type=int, default=0,
                    help="integration tile size (256-2048; 0: the library's default)")
    ap.add_argument("--scan-run", type=int, default=0,
                    help="runs longer than this (per chunk) take the wave's scan of the "
                         "per-event maps (0: the library's default)")
    ap.add_argument("--chunk", type=int, default=0,
                    help="records per integration chunk for 512-pixel tiles: 1536 (default) "
                         "or 2048 (esi_set_chunk)")
    ap.add_argument("--flags", type=int, default=0,
                    help="method flags: 1 decay then add, 2 lazy (undecayed) snapshots, "
                         "4 exponential decay")
    ap.add_argument("--cpu-sample-s", type=float, default=0.0,
                    help="seconds of the workload the CPU oracle is timed on (0: a sample "
                         "of about 15M events)")
    ap.add_argument("--cpu-min-s", type=float, default=8.0,
                    help="repeat each CPU oracle pass over the sample until this many seconds")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="host threads of the all-core CPU baseline (0: the host's share, "
                         "at most 16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--loads", type=float, nargs="+", default=[0.5, 1.0, 2.0, 3.0],
                    help="served workload: offered loads in Gevents/s")
    ap.add_argument("--serve-s", type=float, default=2.0,
                    help="served workload: seconds of arrivals per offered load")
    ap.add_argument("--budget-gb", type=float, default=4.0,
                    help="served workload: HBM budget for admitted sessions (GiB)")
    ap.add_argument("--max-batch", type=int, default=256,
                    help="served workload: sessions per tick")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after timing, run one plain device copy of this many MiB (a "
                         "known-size reference for hardware byte counters)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_<workload>_<fps>fps.json from two rocprofv3 "
                         "counter runs (FETCH_SIZE, WRITE_SIZE) that ended with "
                         "--copy-probe-mb 256, and exit")
    ap.add_argument("--kernel-stats", metavar="STATS_CSV",
                    help="print a rocprofv3 kernel_stats CSV as a markdown table, and exit")
    args = ap.parse_args()
    if args.write_traffic:
        out = write_traffic(args.workload, args.fps, args.write_traffic[0],
                            args.write_traffic[1], 256)
        print(json.dumps(out, indent=1))
        return 0
    if args.kernel_stats:
        print(kernel_stats_table(args.kernel_stats))
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE "
              f"{world}): this library measures the single-GPU path; sharding across GPUs "
              "(whole streams per GPU, or row bands with an event exchange) is not built.",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import evgen
    import paper_2508_02238_amd as esi

    torch.cuda.set_device(0)
    if args.workload == "c4":
        return bench_batched(args)
    if args.workload == "c5":
        return bench_served(args)
    t0 = time.time()
    log(f"[bench] generating workload {args.workload}")
    s = evgen.preset(args.workload)
    tf = s.frame_times(args.fps)
    n, W, H, nf = s.n, s.width, s.height, len(tf)
    npix = W * H
    log(f"[bench] workload {args.workload}: {W}x{H}, {n} events, {nf} frames "
        f"(generated in {time.time() - t0:.1f} s)")
    prm = dict(evgen.DEFAULT_PARAMS)
    prm["flags"] = args.flags
    want_f32 = not args.u8_only
    want_u8 = args.u8 or args.u8_only

    dev = torch.device("cuda", 0)
    x_d = torch.from_numpy(s.x.view(np.int16)).to(dev)
    y_d = torch.from_numpy(s.y.view(np.int16)).to(dev)
    t_d = torch.from_numpy(s.t).to(dev)
    p_d = torch.from_numpy(s.p).to(dev)
    tf_d = torch.from_numpy(tf).to(dev)
    frames = torch.empty((nf, H, W), dtype=torch.float32, device=dev) if want_f32 else None
    frames_u8 = torch.empty((nf, H, W), dtype=torch.uint8, device=dev) if want_u8 else None
    st = esi.State(W, H, **prm)
    if args.tile_pixels:
        st.set_tile_pixels(args.tile_pixels)
    if args.scan_run:
        st.set_scan_run(args.scan_run)
    if args.chunk:
        st.set_chunk(args.chunk)
    stream = torch.cuda.current_stream(dev).cuda_stream

    def step():
        rc = esi.esi_reset(st.handle, stream)
        assert rc == esi.ESI_OK, esi.esi_status_string(rc)
        rc = esi.esi_integrate_window(
            st.handle, x_d.data_ptr(), y_d.data_ptr(), t_d.data_ptr(), p_d.data_ptr(), n,
            tf_d.data_ptr(), nf, frames.data_ptr() if frames is not None else None,
            frames_u8.data_ptr() if frames_u8 is not None else None, stream)
        assert rc == esi.ESI_OK, esi.esi_status_string(rc)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} steps done")

    assert esi.esi_profile_enable(st.handle, True) == esi.ESI_OK
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    h0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    host_ms = (time.perf_counter() - h0) * 1e3
    gpu_ms = ev0.elapsed_time(ev1)
    rc, calls, bucket_ms, integ_ms = esi.esi_profile_read(st.handle)
    assert rc == esi.ESI_OK and calls == args.steps
    esi.esi_profile_enable(st.handle, False)
    ms_per_step = gpu_ms / args.steps
    bucket_avg, integ_avg = bucket_ms / calls, integ_ms / calls
    call_ms = bucket_avg + integ_avg
    log(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step (host {host_ms / args.steps:.3f}), "
        f"call {call_ms:.3f} ms = bucketing {bucket_avg:.3f} + integration {integ_avg:.3f}")

    if args.copy_probe_mb:
        a = torch.ones(args.copy_probe_mb << 18, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {args.copy_probe_mb} MiB read + {args.copy_probe_mb} MiB written")
        del a, b

    # algorithmic bytes: the whole call, and each phase on the bytes it must
    # move itself (bucketing: the events; integration: state and frames)
    alg = algorithmic_bytes(n, npix, nf, want_u8, want_f32)
    alg_bucket = 13 * n
    alg_integ = alg - alg_bucket
    gbs = lambda nbytes, ms: nbytes / (ms * 1e-3) / 1e9
    default_form = (want_f32 and not want_u8 and args.flags == 0 and not args.tile_pixels
                    and not args.scan_run and not args.chunk)
    meas = measured_traffic(args.workload, args.fps) if default_form else None
    roofline = {
        "scope": "one esi_integrate_window call: bucketing (k_hist, k_seg_sum, k_seg_down, "
                 "k_bucket) and integration (k_integrate), timed with HIP events the "
                 "library records on its stream",
        "bound": "hbm",
        "achieved": round(gbs(alg, call_ms), 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(gbs(alg, call_ms) / HBM_PEAK_GBS, 4),
        "traffic": meas[0] if meas else None,
        "algorithmic_bytes": alg,
        "call_ms": round(call_ms, 4),
        "kernels": {
            "bucketing": {"kernels": "k_hist, k_seg_sum, k_seg_down, k_bucket",
                          "algorithmic_bytes": alg_bucket, "avg_ms": round(bucket_avg, 4),
                          "achieved": round(gbs(alg_bucket, bucket_avg), 1),
                          "frac": round(gbs(alg_bucket, bucket_avg) / HBM_PEAK_GBS, 4),
                          "traffic": meas[1].get("bucketing") if meas else None},
            "integration": {"kernels": "k_integrate",
                            "algorithmic_bytes": alg_integ, "avg_ms": round(integ_avg, 4),
                            "achieved": round(gbs(alg_integ, integ_avg), 1),
                            "frac": round(gbs(alg_integ, integ_avg) / HBM_PEAK_GBS, 4),
                            "traffic": meas[1].get("integration") if meas else None},
        },
    }

    parity = None
    if not args.no_parity:
        import oracle
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from esi_parity import REL, u8_codes
        sel = sorted(set([0, nf // 3, nf // 2, nf - 1]))
        log(f"[bench] parity: oracle over the whole workload, frames {sel}")
        h0 = time.time()
        o = oracle.State(W, H, oracle.Params(**prm))
        fo = o.integrate(s.x, s.y, s.t, s.p, t_frames=tf, frame_sel=sel)
        S, T, N, P = (a.cpu().numpy() for a in st.read_state())
        floor_f = prm["C"] / (prm["s_max"] - prm["s_min"])
        s_err = np.abs(S.astype(np.float64) - o.S) / np.maximum(np.abs(o.S), prm["C"])
        f_max = 0.0
        if frames is not None:
            fg = frames[sel].cpu().numpy()
            f_max = float((np.abs(fg.astype(np.float64) - fo) / np.maximum(np.abs(fo), floor_f)).max())
        u8_max = 0
        if frames_u8 is not None:
            ug = frames_u8[sel].cpu().numpy()
            u8_max = int(np.abs(ug.astype(np.int32) - u8_codes(fo).astype(np.int32)).max())
        exact = (np.array_equal(N.view(np.uint32), o.N) and np.array_equal(P, o.P)
                 and np.array_equal(T, o.T))
        ok = exact and s_err.max() <= REL and f_max <= REL and u8_max <= 1
        parity = {"ok": bool(ok), "max_rel_S": float(s_err.max()),
                  "max_rel_frame": f_max, "max_u8_code_diff": u8_max, "frames_checked": sel,
                  "exact_N_P_T": bool(exact)}
        log(f"[bench] parity vs oracle: {parity} ({time.time() - h0:.1f} s)")

    cpu = None
    if not args.no_cpu_baseline:
        span_s = args.cpu_sample_s
        if span_s <= 0:
            # about 15M events (c1 and c2 whole; c3 its first half second)
            span_s = min(s.duration_us / 1e6, 15e6 / max(n / (s.duration_us / 1e6), 1.0))
        threads = args.cpu_threads or max(1, min(os.cpu_count() or 1, 16))
        log(f"[bench] cpu baseline: first {span_s:g} s, 1 and {threads} threads")
        cpu = cpu_baseline(s, tf, prm, span_s, args.cpu_min_s, threads)
        log(f"[bench] cpu baseline: {cpu}")

    value = n / (ms_per_step * 1e-3) / 1e9
    out = {
        "metric": "Gevents/s integrated + frames/s at 1e-5 rel err",
        "value": round(value, 3),
        "unit": "Gevents/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "frames_per_s": round(nf / (ms_per_step * 1e-3), 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {W}x{H}, {s.duration_us / 1e6:g} s, "
                               f"{n} events, {nf} frames at {args.fps:g} FPS"
                               + (", 8-bit frames only" if args.u8_only
                                  else ", +u8 frames" if args.u8 else "")
                               + (f", flags {args.flags}" if args.flags else "")
                               + (f", scan_run {args.scan_run}" if args.scan_run else "")
                               + (f", chunk {args.chunk}" if args.chunk else ""),
                   "events": n, "frames": nf, "width": W, "height": H,
                   "params": prm,
                   "frame_dtype": "u8" if args.u8_only else ("f32+u8" if args.u8 else "f32")},
        "roofline": roofline,
        "parity": parity,
        "cpu_baseline": cpu,
    }
    st.close()
    print(json.dumps(out), flush=True)
    return 0


def bench_batched(args) -> int:
    """Workload c4: 64 independent streams of mixed size and rate, integrated
    window by window (10 ms of events and one frame per stream per window),
    once with one batched call per window and once with one plain call per
    stream per window.  A step is the whole sample (all windows); states are
    reset before each step, outside the timed region."""
    import numpy as np
    import torch

    import evgen
    import paper_2508_02238_amd as esi

    win_us = 10_000
    dur_us = 200_000
    t0 = time.time()
    streams = evgen.preset_batch("c4", duration_us=dur_us)
    nwin = dur_us // win_us
    n_all = sum(s.n for s in streams)
    px_all = sum(s.width * s.height for s in streams)
    log(f"[bench] workload c4: {len(streams)} streams, {px_all} pixels, {n_all} events in "
        f"{nwin} windows of {win_us / 1000:g} ms (generated in {time.time() - t0:.1f} s)")
    prm = dict(evgen.DEFAULT_PARAMS)
    prm["flags"] = args.flags
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev).cuda_stream
    ev_d, bounds, frames, tfs = [], [], [], []
    for s in streams:
        ev_d.append((torch.from_numpy(s.x.view(np.int16)).to(dev),
                     torch.from_numpy(s.y.view(np.int16)).to(dev),
                     torch.from_numpy(s.t).to(dev), torch.from_numpy(s.p).to(dev)))
        bounds.append(np.searchsorted(s.t, np.arange(nwin + 1) * win_us, side="left"))
        frames.append(torch.empty((1, s.height, s.width), dtype=torch.float32, device=dev))
    tf_d = torch.tensor([(w + 1) * win_us - 1 for w in range(nwin)], dtype=torch.int64,
                        device=dev)
    states = [esi.State(s.width, s.height, **prm) for s in streams]
    batch = esi.Batch(len(streams))

    def items(w):
        evs, tfp = [], []
        for i, (x, y, t, p) in enumerate(ev_d):
            lo, hi = int(bounds[i][w]), int(bounds[i][w + 1])
            n = hi - lo
            evs.append((x.data_ptr() + 2 * lo, y.data_ptr() + 2 * lo, t.data_ptr() + 8 * lo,
                        p.data_ptr() + lo, n) if n else (None, None, None, None, 0))
        return evs

    win_items = [items(w) for w in range(nwin)]
    handles = [s.handle for s in states]
    frp = [f.data_ptr() for f in frames]

    def run_batched():
        for w in range(nwin):
            rc = esi.esi_integrate_batch(batch.handle, handles, win_items[w],
                                         [tf_d.data_ptr() + 8 * w] * len(states),
                                         [1] * len(states), frp, None, stream)
            assert rc == esi.ESI_OK, esi.esi_status_string(rc)

    def run_plain():
        for w in range(nwin):
            for i, h in enumerate(handles):
                e = win_items[w][i]
                rc = esi.esi_integrate_window(h, *e, tf_d.data_ptr() + 8 * w, 1, frp[i], None,
                                              stream)
                assert rc == esi.ESI_OK, esi.esi_status_string(rc)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            for s in states:
                s.reset()
            fn()
        torch.cuda.synchronize()
        total = 0.0
        for _ in range(steps):
            for s in states:
                s.reset()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            total += e0.elapsed_time(e1)
        return total / steps

    ms_default = timed(run_batched, args.steps, args.warmup)
    ms_plain = timed(run_plain, args.steps, args.warmup)
    # tile sizes per sensor size and the scan threshold from the autotuner
    # (throwaway states, the first three windows); tuning is not timed
    from paper_2508_02238_amd.tune import tune
    h0 = time.time()
    sample = []
    for w in range(3):
        evs = []
        for i, (x, y, t, p) in enumerate(ev_d):
            lo, hi = int(bounds[i][w]), int(bounds[i][w + 1])
            evs.append((x[lo:hi], y[lo:hi], t[lo:hi], p[lo:hi]))
        sample.append((evs, [tf_d[w:w + 1]] * len(streams)))
    sizes = [(s.width, s.height) for s in streams]
    tuned = tune(sizes, prm, sample)
    choice = tuned["tile_pixels"]
    for st, sz in zip(states, sizes):
        st.set_tile_pixels(choice[sz])
        st.set_scan_run(tuned["scan_run"])
        st.set_chunk(tuned["chunk"])
    log(f"[bench] tuned tile pixels {choice}, scan run {tuned['scan_run']}, "
        f"chunk {tuned['chunk']} ({time.time() - h0:.1f} s)")
    ms_batch = timed(run_batched, args.steps, args.warmup)
    log(f"[bench] per window: batched {ms_batch / nwin * 1e3:.1f} us (default tiles "
        f"{ms_default / nwin * 1e3:.1f} us), plain {ms_plain / nwin * 1e3:.1f} us "
        f"({len(streams)} calls)")

    parity = None
    if not args.no_parity:
        import oracle
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from esi_parity import REL
        for s in states:
            s.reset()
        run_batched()
        torch.cuda.synchronize()
        worst_s = worst_f = 0.0
        exact = True
        pick = sorted(set([0, len(streams) // 2, len(streams) - 1]))
        floor_f = prm["C"] / (prm["s_max"] - prm["s_min"])
        for i in pick:
            s = streams[i]
            o = oracle.State(s.width, s.height, oracle.Params(**prm))
            fo = o.integrate(s.x, s.y, s.t, s.p, t_frames=np.array([dur_us - 1], np.int64))
            S, T, N, P = (a.cpu().numpy() for a in states[i].read_state())
            exact &= (np.array_equal(N.view(np.uint32), o.N) and np.array_equal(P, o.P)
                      and np.array_equal(T, o.T))
            worst_s = max(worst_s, float((np.abs(S.astype(np.float64) - o.S)
                                          / np.maximum(np.abs(o.S), prm["C"])).max()))
            fg = frames[i].cpu().numpy()
            worst_f = max(worst_f, float((np.abs(fg.astype(np.float64) - fo)
                                          / np.maximum(np.abs(fo), floor_f)).max()))
        parity = {"ok": bool(exact and worst_s <= REL and worst_f <= REL),
                  "streams_checked": pick, "max_rel_S": worst_s, "max_rel_frame": worst_f,
                  "exact_N_P_T": bool(exact)}
        log(f"[bench] parity vs oracle: {parity}")

    # per window: events read, S and T of
    # every pixel read for the frame, the full state of the active pixels
    # read and written (N, P read; S, T, N, P written), one FP32 frame
    active = 0
    for i, s in enumerate(streams):
        q = s.y.astype(np.int64) * s.width + s.x
        for w in range(nwin):
            active += np.unique(q[bounds[i][w]:bounds[i][w + 1]]).size
    alg = 13 * n_all + nwin * (12 + 4) * px_all + 28 * active
    out = {
        "metric": "Gevents/s integrated + frames/s at 1e-5 rel err (batched streams)",
        "value": round(n_all / (ms_batch * 1e-3) / 1e9, 3),
        "unit": "Gevents/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_batch, 4),
        "us_per_window": round(ms_batch / nwin * 1e3, 1),
        "plain_us_per_window": round(ms_plain / nwin * 1e3, 1),
        "default_tiles_us_per_window": round(ms_default / nwin * 1e3, 1),
        "tuned_tile_pixels": {f"{w}x{h}": v for (w, h), v in choice.items()},
        "tuned_scan_run": tuned["scan_run"],
        "tuned_chunk": tuned["chunk"],
        "batched_over_plain": round(ms_plain / ms_batch, 3),
        "frames_per_s": round(len(streams) * nwin / (ms_batch * 1e-3), 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"c4: {len(streams)} streams (346x260, 640x480, 1280x720), "
                               f"{n_all} events in {nwin} windows of 10 ms, one frame per "
                               f"stream per window",
                   "streams": len(streams), "pixels": px_all, "events": n_all,
                   "windows": nwin, "params": prm},
        "roofline_path": {"achieved": round(alg / (ms_batch * 1e-3) / 1e9, 1),
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(alg / (ms_batch * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "algorithmic_bytes": alg},
        "parity": parity,
    }
    batch.close()
    for s in states:
        s.close()
    print(json.dumps(out), flush=True)
    return 0


def bench_served(args) -> int:
    """Workload c5: 256 sessions with the resolution and rate mix of c4 (256
    distinct streams, seeds 5000 + s), 10 ms packets with Poisson arrivals,
    each session's state resident in HBM, sessions admitted against an HBM
    budget (--budget-gb), two ticks in flight.  Each stream is replayed as
    back-to-back sessions (one per pass over its 20 packets: a session closes
    when its last packet completes and the next pass opens a new one), so
    sessions keep arriving and leaving.  The packets are resident in device
    memory before timing (as the other workloads' inputs are); the offered
    load is set by compressing the arrival clock (1x: every stream in real
    time, about 0.56 Gevents/s) and swept over --loads; each load runs for
    --serve-s seconds of arrivals, then drains.  Reports per load:
    throughput (completed events / wall time), p50/p99 packet-to-frame
    latency (arrival to the poll that sees the packet's frame ready)."""
    import numpy as np
    import torch

    import evgen
    from paper_2508_02238_amd.serve import Server

    win_us, dur_us = 10_000, 200_000
    nwin = dur_us // win_us
    t0 = time.time()
    streams = evgen.preset_batch("c5", duration_us=dur_us)
    n_sess = len(streams)
    dev = torch.device("cuda", 0)
    # every stream's events on the device, packets as (offset, n) views
    xs = torch.from_numpy(np.concatenate([s.x for s in streams]).view(np.int16)).to(dev)
    ys = torch.from_numpy(np.concatenate([s.y for s in streams]).view(np.int16)).to(dev)
    ts = torch.from_numpy(np.concatenate([s.t for s in streams])).to(dev)
    ps = torch.from_numpy(np.concatenate([s.p for s in streams])).to(dev)
    base = np.cumsum([0] + [s.n for s in streams])
    pk_off = np.zeros((n_sess, nwin), np.int64)
    pk_n = np.zeros((n_sess, nwin), np.int64)
    for i, s in enumerate(streams):
        b = np.searchsorted(s.t, np.arange(nwin + 1) * win_us, side="left")
        pk_off[i] = base[i] + b[:-1]
        pk_n[i] = np.diff(b)
    n_total = int(base[-1])
    rate_1x = n_total / (dur_us * 1e-6)
    max_pk = int(pk_n.max())
    log(f"[bench] workload c5: {n_sess} sessions, {nwin} packets of 10 ms per pass, "
        f"{n_total} events per pass of all streams ({rate_1x / 1e9:.3f} Gev/s in real time), "
        f"largest packet {max_pk} (generated in {time.time() - t0:.1f} s)")
    prm = dict(evgen.DEFAULT_PARAMS)
    px, py, pt, pp = (a.data_ptr() for a in (xs, ys, ts, ps))
    results = []
    budget = int(args.budget_gb * (1 << 30))
    # tile sizes per sensor size and the scan threshold from the autotuner
    # over the first two packets of every stream (throwaway states; not
    # timed), applied to every state the server creates
    from paper_2508_02238_amd.serve import HipDevice
    from paper_2508_02238_amd.tune import tune
    h0 = time.time()
    sample = []
    for k in range(2):
        evs = []
        for i in range(n_sess):
            lo, hi = int(pk_off[i, k]), int(pk_off[i, k] + pk_n[i, k])
            evs.append((xs[lo:hi], ys[lo:hi], ts[lo:hi], ps[lo:hi]))
        tfk = torch.tensor([(k + 1) * win_us - 1], dtype=torch.int64, device=dev)
        sample.append((evs, [tfk] * n_sess))
    tuned = tune([(s.width, s.height) for s in streams], prm, sample)
    log(f"[bench] tuned tile pixels {tuned['tile_pixels']}, scan run {tuned['scan_run']}, "
        f"chunk {tuned['chunk']} ({time.time() - h0:.1f} s)")
    for load in args.loads:
        f = load * 1e9 / rate_1x
        rng = np.random.default_rng(5)
        # arrivals: stream s starts at a random offset; packet j of its
        # replay (pass j // nwin, packet j % nwin) after j exponential gaps
        per = int(np.ceil(args.serve_s * f * 1e6 / win_us)) + 2
        start = rng.uniform(0, win_us * 1e-6 / f, n_sess)
        gaps = rng.exponential(win_us * 1e-6 / f, (n_sess, per))
        at = start[:, None] + np.cumsum(gaps, axis=1)
        sel = at < args.serve_s
        order = np.argsort(at[sel], kind="stable")
        s_idx = np.broadcast_to(np.arange(n_sess)[:, None], at.shape)[sel][order]
        j_idx = np.broadcast_to(np.arange(per)[None, :], at.shape)[sel][order]
        a_t = at[sel][order]
        device = HipDevice(args.max_batch, max_pk, tile_pixels=tuned["tile_pixels"],
                           scan_run=tuned["scan_run"], chunk=tuned["chunk"])
        srv = Server(budget_bytes=budget, max_batch=args.max_batch, max_packet_events=max_pk,
                     ring=3, max_inflight=2, device=device)
        remaining = {}
        done_events = 0
        n_arr = len(a_t)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        i = 0
        n_done = 0
        admitted_sum = ticks = 0
        tick_host = 0.0   # host seconds inside the ticks that launched
        host = dict(open=0.0, submit=0.0, tick=0.0, poll=0.0, close=0.0)  # host seconds per call kind
        while n_done < n_arr:
            now = time.perf_counter() - t_start
            if now > args.serve_s + 120.0:
                log(f"[bench] served {load:g} Gev/s: {n_arr - n_done} packets not done "
                    f"after {now:.0f} s; stopping")
                return 1
            while i < n_arr and a_t[i] <= now:
                s, j = int(s_idx[i]), int(j_idx[i])
                r, k = divmod(j, nwin)
                sid = (s, r)
                if k == 0:
                    st = streams[s]
                    th = time.perf_counter()
                    if srv.open(sid, st.width, st.height, **prm) == "rejected":
                        raise RuntimeError(f"session of {st.width}x{st.height} exceeds the "
                                           f"{args.budget_gb:g} GiB budget")
                    host["open"] += time.perf_counter() - th
                    remaining[sid] = nwin
                o, n = int(pk_off[s, k]), int(pk_n[s, k])
                th = time.perf_counter()
                srv.submit_device(sid, px + 2 * o, py + 2 * o, pt + 8 * o, pp + o, n,
                                  (k + 1) * win_us - 1, pid=k, arrival=t_start + a_t[i])
                host["submit"] += time.perf_counter() - th
                i += 1
            th = time.perf_counter()
            if srv.tick():
                ticks += 1
                admitted_sum += len(srv.order)
                tick_host += time.perf_counter() - th
            host["tick"] += time.perf_counter() - th
            th = time.perf_counter()
            polled = srv.poll()
            host["poll"] += time.perf_counter() - th
            for c in polled:
                n_done += 1
                s, r = c.sid
                done_events += int(pk_n[s, c.pid])
                remaining[c.sid] -= 1
                if remaining[c.sid] == 0:
                    th = time.perf_counter()
                    srv.close(c.sid)
                    host["close"] += time.perf_counter() - th
            if i >= n_arr:
                # arrivals over: sessions cut short by the window close once drained
                for sid, left in list(remaining.items()):
                    ss = srv.sessions.get(sid)
                    if ss is not None and left > 0 and not ss.pending and ss.inflight == 0 \
                            and ss.status == "admitted":
                        remaining[sid] = 0
                        srv.close(sid)
            if srv.busy() == 0 and i < n_arr and a_t[i] > now:
                time.sleep(min(1e-4, a_t[i] - now))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        lat = np.array([c.latency_s for c in srv.done if c.ok]) * 1e3
        srv.close_all()
        r = {"offered_gev_s": round(load, 3),
             "throughput_gev_s": round(done_events / wall / 1e9, 3),
             "p50_ms": round(float(np.percentile(lat, 50)), 3),
             "p99_ms": round(float(np.percentile(lat, 99)), 3),
             "packets": int(lat.size), "wall_s": round(wall, 3),
             "mean_admitted_sessions": round(admitted_sum / max(ticks, 1), 1),
             "mean_packets_per_tick": round(n_arr / max(ticks, 1), 1),
             "ticks_per_s": round(ticks / wall, 1),
             "host_ms_per_tick": round(tick_host / max(ticks, 1) * 1e3, 3),
             "host_s": {k: round(v, 3) for k, v in host.items()},
             "states_created": getattr(srv, "created", None),
             "states_destroyed": getattr(srv, "destroyed", None)}
        log(f"[bench] served {load:g} Gev/s offered: {r}")
        results.append(r)
    out = {
        "metric": "p50/p99 packet->frame latency and throughput (served sessions)",
        "value": results[-1]["throughput_gev_s"],
        "unit": "Gevents/s served at the highest offered load",
        "n_gpus": 1,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"c5: {n_sess} sessions (distinct seeded streams), 10 ms "
                               f"packets, Poisson arrivals, {args.budget_gb:g} GiB HBM budget, "
                               f"packets resident in device memory",
                   "sessions": n_sess, "packets_per_pass": nwin, "params": prm,
                   "budget_gib": args.budget_gb, "max_batch": args.max_batch,
                   "tile_pixels": {f"{w}x{h}": t for (w, h), t in tuned["tile_pixels"].items()},
                   "scan_run": tuned["scan_run"], "chunk": tuned["chunk"]},
        "loads": results,
    }
    print(json.dumps(out), flush=True)
    return 0


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip() + f" ({os.cpu_count()} logical CPUs)"
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    sys.exit(main())
