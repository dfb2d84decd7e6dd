"""Benchmark of the Onesweep sort on one MI355X.

A step is one whole sort (clear + all-place histogram + exclusive sums +
every binning pass + final copy check) of a fixed synthetic input already
resident in HBM. Default workload: 2^28 uniform uint32 keys, keys only,
8-bit digits (4 passes). Prints ONE JSON line on stdout; a per-kernel
breakdown goes to stderr.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GKeys/s + % HBM roofline, 256M u32 keys; batched/learned vs plain Onesweep"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "binning_u32_keys_2p28_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2206_01784_amd", "csrc", f)
                  for f in ("binning.hip", "device_common.hpp")]

WORKLOADS = {
    # name: (key_bits, values, distribution, log2 n)
    "u32_keys_uniform": (32, False, "uniform", 28),
    "u32_keys_and2": (32, False, "and2", 28),
    "u32_keys_and3": (32, False, "and3", 28),
    "u32_keys_and4": (32, False, "and4", 28),
    "u32_keys_equal": (32, False, "equal", 28),
    "u32_keys_and8": (32, False, "and8", 28),
    "u32_keys_and16": (32, False, "and16", 28),
    "u64_keys_uniform": (64, False, "uniform", 27),
    "f32_keys_mixed": (32, False, "float", 28),
    "u32_keys_uniform_descending": (32, False, "uniform", 28),
    "u32_pairs_uniform": (32, True, "uniform", 28),
    "u64_pairs_uniform": (64, True, "uniform", 27),
    "u32_keys_uniform_2p20": (32, False, "uniform", 20),
    "u32_keys_uniform_2p30": (32, False, "uniform", 30),
    "u32_keys_uniform_2p31": (32, False, "uniform", 31),
}
# Batched segmented workload: S segments with log-normal lengths (median 2000,
# sigma 1.5, cap 2^22) scaled to 2^26 keys in total; uniform uint32 keys,
# values = index within the segment.
LOOP_GRAPH_SEGMENTS = 500
SEGMENT_WORKLOADS = {
    # name: (segments, log2 total keys)
    "segments_lognormal_20000": (20000, 26),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(workload: str):
    """HBM traffic per binning launch from the committed rocprofv3 counter
    summary, or None when it is missing, covers another workload, or the
    kernel source changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.lstrip().startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if kv.get("workload") != workload:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _read_counters(path):
    """{kernel name: [counter value per dispatch]} from a rocprofv3 counter CSV."""
    import csv
    out = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            name = row.get("Kernel_Name") or row.get("Kernel-Name") or ""
            val = row.get("Counter_Value") or row.get("Counter-Value")
            if val is None:
                continue
            out.setdefault(name, []).append(float(val))
    return out


def summarize_counters(fetch_csv, write_csv, workload="u32_keys_uniform"):
    """Write the binning kernel's measured HBM traffic per launch.

    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of each binning launch are
    scaled by bytes / counter of the plain copy kernel in the same run, whose
    true traffic is known (n * key bytes read and written).
    """
    import statistics as st
    key_bits, has_vals, dist, log2n = WORKLOADS[workload]
    n = 1 << log2n
    copy_bytes = n * (key_bits // 8 + (4 if has_vals else 0))
    fetch, write = _read_counters(fetch_csv), _read_counters(write_csv)

    def pick(d, pattern):
        vals = [v for k, vs in d.items() if re.search(pattern, k) for v in vs]
        if not vals:
            raise SystemExit(f"no dispatches of {pattern} in the counter file")
        return vals

    # the chained-scan binning kernel: template mode argument 0 (then the key
    # order flag and the element position type)
    binning = r"binning_kernel<[^<>]*, 0, (false|true), unsigned (int|long)>"
    copy_f = max(pick(fetch, "copy_kernel")) * 1024
    copy_w = max(pick(write, "copy_kernel")) * 1024
    bin_f = st.mean(pick(fetch, binning)) * 1024
    bin_w = st.mean(pick(write, binning)) * 1024
    f_scale, w_scale = copy_bytes / copy_f, copy_bytes / copy_w
    traffic = bin_f * f_scale + bin_w * w_scale
    alg = n * 2 * (key_bits // 8 + (4 if has_vals else 0))
    lines = [
        "# HBM traffic of one binning launch, from two rocprofv3 --pmc runs of bench.py",
        f"# workload: {workload} (n = 2^{log2n})",
        f"# fetch csv: {os.path.basename(fetch_csv)}; write csv: {os.path.basename(write_csv)}",
        "# scale = bytes the plain copy kernel must move / its counter reading",
        "# commands (repo root; run from /tmp with TMPDIR=/tmp):",
        "#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o pmc -- "
        f"python bench.py --workload {workload} --steps 2 --warmup 0 --no-rts-baseline "
        "--no-cpu-baseline --no-segments --calibrate-copy",
        "#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o pmc -- "
        f"python bench.py --workload {workload} --steps 2 --warmup 0 --no-rts-baseline "
        "--no-cpu-baseline --no-segments --calibrate-copy",
        "#   python bench.py --workload " + workload + " --counters-summary <fetch csv> <write csv>",
        f"kernel_source_sha256_16: {kernel_source_hash()}",
        f"workload: {workload}",
        f"copy_fetch_kib: {copy_f / 1024:.1f}",
        f"copy_write_kib: {copy_w / 1024:.1f}",
        f"copy_true_bytes_each_way: {copy_bytes}",
        f"fetch_scale: {f_scale:.4f}",
        f"write_scale: {w_scale:.4f}",
        f"binning_fetch_kib_per_launch: {bin_f / 1024:.1f}",
        f"binning_write_kib_per_launch: {bin_w / 1024:.1f}",
        f"hbm_bytes_per_launch: {traffic:.0f}",
        f"algorithmic_bytes_per_launch: {alg}",
        f"traffic_over_algorithmic: {traffic / alg:.3f}",
    ]
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


# Key type and direction of the workloads that are not unsigned ascending.
WORKLOAD_ORDER = {
    "f32_keys_mixed": ("float", False),
    "u32_keys_uniform_descending": ("unsigned", True),
}


def make_keys(dist, n, key_bits, seed=2):
    import workload as W
    if dist == "float":
        return W.float_bits(seed, n, key_bits)
    if dist == "uniform":
        return W.uniform(seed, n, key_bits)
    if dist == "equal":
        return W.all_equal(seed, n, key_bits)
    return W.make_keys(dist, seed, n, key_bits)


def cpu_model():
    """CPU model name and the number of logical CPUs this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(keys, vals, max_s=40.0):
    """The CPU oracle, single-threaded, on the whole input (median of up to
    three runs, fewer when one run takes longer than max_s / 3)."""
    import oracle
    model, cpus = cpu_model()
    times = []
    while len(times) < 3 and sum(times) < max_s:
        t0 = time.perf_counter()
        oracle.sort(keys, vals)
        times.append(time.perf_counter() - t0)
    med = statistics.median(times)
    n = keys.size
    return {"value": round(n / med / 1e9, 4), "unit": "GKeys/s", "cores": 1,
            "kind": "oracle", "cpu": model, "host_cpus": cpus,
            "sample": f"the whole timed input (2^{n.bit_length() - 1} keys), median of "
                      f"{len(times)} single-threaded runs of the oracle"}


def cpu_parallel_baseline(keys, vals, max_s=30.0):
    """A multithreaded LSD radix sort (OpenMP, every core this process may
    use) on the whole input: the secondary CPU baseline, checked against the
    oracle in tests/test_cpu_baseline.py. Median of up to three runs."""
    import numpy as np
    import cpu_baseline
    model, cpus = cpu_model()
    threads = cpu_baseline.threads_used()
    times = []
    while len(times) < 3 and sum(times) < max_s:
        t0 = time.perf_counter()
        k, _ = cpu_baseline.sort(keys, vals)
        times.append(time.perf_counter() - t0)
    if keys.dtype == np.uint32 and vals is None and not np.array_equal(k, np.sort(keys)):
        log("[bench] ERROR: the multithreaded CPU sort differs from numpy's sort")
        sys.exit(1)
    med = statistics.median(times)
    n = keys.size
    return {"value": round(n / med / 1e9, 4), "unit": "GKeys/s", "cores": threads,
            "kind": "multithreaded LSD radix sort (OpenMP)", "cpu": model, "host_cpus": cpus,
            "sample": f"the whole timed input (2^{n.bit_length() - 1} keys), median of "
                      f"{len(times)} runs on {threads} threads"}


def segment_inputs(num_segments, log2n, seed=4):
    import numpy as np
    import workload as W
    lengths = W.lognormal_segment_lengths(num_segments=num_segments, total=1 << log2n, seed=seed)
    off = W.offsets_from_lengths(lengths)
    n = int(off[-1])
    keys = W.uniform(seed, n)
    seg_of = np.repeat(np.arange(num_segments), lengths)
    vals = (np.arange(n, dtype=np.int64) - off[seg_of]).astype(np.uint32)
    return lengths, off, keys, vals


def cpu_baseline_segments(keys, vals, off, target_s=10.0):
    """The CPU oracle on the first segments holding about 2^24 keys."""
    import numpy as np
    import oracle
    last = int(np.searchsorted(off, 1 << 24, side="right")) - 1
    last = max(last, 1)
    cut = int(off[last])
    o = off[: last + 1]
    ks, vs = np.ascontiguousarray(keys[:cut]), np.ascontiguousarray(vals[:cut])
    times = []
    t_start = time.perf_counter()
    while len(times) < 3 or (time.perf_counter() - t_start < target_s and len(times) < 10):
        t0 = time.perf_counter()
        oracle.sort_segments(ks, o, vs)
        times.append(time.perf_counter() - t0)
    med = statistics.median(times)
    return {"value": round(cut / med / 1e9, 4), "unit": "GKeys/s", "cores": 1, "kind": "oracle",
            "sample": f"first {last} segments ({cut} pairs) of the same input, median of "
                      f"{len(times)} single-threaded runs"}


def segments_leg(args, S, log2n, tune=False, with_loops=True):
    """The batched segmented sort, one captured graph replayed `steps` times
    (configuration: the command line's, or the autotuner's pick on this data
    when `tune`), its output spot-checked, per-kernel durations from eager
    traced runs, and the per-segment loops of plain pair sorts as baselines.
    Returns a dict of the measurements."""
    import numpy as np
    import torch
    import paper_2206_01784_amd as ow

    log(f"[bench] segments: {S} log-normal segments, 2^{log2n} pairs, generating input")
    lengths, off, keys, vals = segment_inputs(S, log2n)
    n = int(off[-1])
    stream = torch.cuda.current_stream()
    d_keys = torch.from_numpy(keys).cuda()
    d_vals = torch.from_numpy(vals).cuda()
    d_off = torch.from_numpy(off.astype(np.uint32)).cuda()
    d_kout = torch.empty_like(d_keys)
    d_vout = torch.empty_like(d_vals)
    if tune:
        t0 = time.perf_counter()
        tuned = ow.tune_segments(d_keys, d_off, d_vals, keys_out=d_kout, values_out=d_vout,
                                 repetitions=3)
        torch.cuda.synchronize()
        block, ipt = tuned.block_threads, tuned.items_per_thread
        limits = tuple(tuned.segment_limits)
        log(f"[bench] segments: autotuner picked tile {block} x {ipt}, class limits {limits} "
            f"({time.perf_counter() - t0:.1f} s)")
    else:
        block, ipt, limits = args.block, args.ipt, tuple(args.segment_limits)
    cfg = ow.make_config(block, ipt, rank_algorithm=args.rank, segment_limits=limits,
                         segment_streams=args.segment_streams)
    temp = torch.empty(ow.sort_segments_temp_bytes(n, S, 32, True, config=cfg),
                       dtype=torch.uint8, device="cuda")

    def batched(cfg_, s=stream):
        ow.sort_segments(d_keys, d_off, d_vals, keys_out=d_kout, values_out=d_vout, temp=temp,
                         config=cfg_, stream=s)

    for _ in range(max(args.warmup, 1)):
        batched(cfg)
    torch.cuda.synchronize()
    # Per-kernel durations from eager traced runs (events around each launch).
    launches = 16
    per_kind = {}
    for _ in range(3):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * launches)]
        for e in evs:
            e.record(stream)
        arr = (ctypes.c_void_p * len(evs))(*[e.cuda_event for e in evs])
        tr = ow.Trace()
        tr.events = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
        tr.capacity = launches
        cfg_t = ow.make_config(block, ipt, rank_algorithm=args.rank, segment_limits=limits,
                               trace=tr)
        batched(cfg_t)
        torch.cuda.synchronize()
        for i in range(tr.count):
            per_kind.setdefault((i, tr.kinds[i]), []).append(evs[2 * i].elapsed_time(evs[2 * i + 1]))
    for (i, kind), ts in sorted(per_kind.items()):
        log(f"[bench]   launch {i:2d} {ow.KERNEL_NAMES[kind]:9s} avg={statistics.mean(ts) * 1e3:9.2f} us")

    # Timed: replays of one captured graph of the whole batched sort.
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    with torch.cuda.stream(cap):
        with torch.cuda.graph(g, stream=cap):
            batched(cfg, cap)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        g.replay()
    end.record()
    torch.cuda.synchronize()
    ms_per_step = start.elapsed_time(end) / args.steps
    value = n / (ms_per_step * 1e-3) / 1e9
    log(f"[bench] batched graph: {ms_per_step:.3f} ms per sort, {value:.2f} GKeys/s")
    if int(temp[:4].cpu().numpy().view(np.uint32)[0]) != 0:
        log("[bench] ERROR: offsets reported invalid")
        sys.exit(1)
    # spot check of a few segments by properties that fix a stable sort: the
    # keys are ascending, the values (indices within the segment) are a
    # permutation that maps each output key to its input, and equal keys
    # keep increasing indices (full checks live in tests/)
    out_k, out_v = d_kout.cpu().numpy(), d_vout.cpu().numpy()
    for s_ in (0, S // 2, int(np.argmax(lengths)), S - 1):
        a, b = int(off[s_]), int(off[s_ + 1])
        k_, v_ = out_k[a:b].astype(np.int64), out_v[a:b].astype(np.int64)
        ok = (np.all(k_[1:] >= k_[:-1]) and np.array_equal(np.sort(v_), np.arange(b - a))
              and np.array_equal(keys[a:b][v_], out_k[a:b])
              and np.all((k_[1:] > k_[:-1]) | (v_[1:] > v_[:-1])))
        if not ok:
            log(f"[bench] ERROR: segment {s_} is not a stable sort of its input")
            sys.exit(1)
    baselines = None
    if with_loops:
        baselines = loop_baselines(ow, off, n, S, d_keys, d_vals, d_kout, d_vout, stream, cap,
                                   ms_per_step)
    return {"n": n, "lengths": lengths, "off": off, "keys": keys, "vals": vals,
            "ms_per_step": ms_per_step, "value": value, "block": block, "ipt": ipt,
            "limits": limits, "tuned": tune,
            # tile_items reports the plain sort's table; segments have their own
            "tile": ow.tile_items(32, True, cfg, n) if block else "segmented default",
            "per_kind": per_kind, "baselines": baselines}


def run_segments(args):
    """Batched segmented sort under a captured graph, against per-segment
    loops of the plain pair sort (eager, and captured in graphs)."""
    import paper_2206_01784_amd as ow

    S, log2n = SEGMENT_WORKLOADS[args.workload]
    leg = segments_leg(args, S, log2n, tune=args.tune_segments,
                       with_loops=not args.no_loop_baseline)
    n, lengths = leg["n"], leg["lengths"]
    bins = per_kind_summary(leg["per_kind"], ow, lengths, leg["limits"])
    dom_kind, dom_us, dom_launches = bins["dominant"]
    result = {
        "metric": METRIC,
        "value": round(leg["value"], 3),
        "unit": "GKeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(leg["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": f"batched stable sort of {S} segments (log-normal lengths, median 2000, "
                        f"sigma 1.5, scaled to 2^{log2n} uint32 key/value pairs), one graph replay",
            "n": n, "segments": S, "key_bits": 32, "values": True,
            "segment_limits": list(leg["limits"]),
            "segment_streams": 1 if args.segment_streams == 1 else 2,
            "tile": leg["tile"],
            "autotuned": leg["tuned"],
        },
        "baselines": leg["baselines"],
        "kernels_us": bins["table"],
        "roofline": bins["roofline"] if dom_kind is not None else None,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        result["cpu_baseline"] = cpu_baseline_segments(leg["keys"], leg["vals"], leg["off"])
    print(json.dumps(result), flush=True)


def loop_baselines(ow, off, n, S, d_keys, d_vals, d_kout, d_vout, stream, cap, ms_per_step):
    """The per-segment loop of plain pair sorts over every segment: eager, and
    captured in graphs of LOOP_GRAPH_SEGMENTS segments each (all of them
    replayed back to back). One graph holding the whole loop (about 8 launches
    per segment, ~160,000 kernel nodes) ended the process with a segmentation
    fault on the host during capture; graphs of 500 segments (~4,000 nodes)
    capture and replay normally, so the loop is cut into such graphs."""
    import torch
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lengths = off[1:] - off[:-1]
    seg_temp = torch.empty(ow.sort_temp_bytes(int(lengths.max()), 32, True), dtype=torch.uint8,
                           device="cuda")
    bounds = [(int(off[i]), int(off[i + 1])) for i in range(S) if off[i + 1] > off[i]]

    def loop(segs, s):
        for a, b in segs:
            ow.sort_pairs(d_keys[a:b], d_vals[a:b], keys_out=d_kout[a:b], values_out=d_vout[a:b],
                          temp=seg_temp, stream=s)

    # Baseline 1: eager loop.
    loop(bounds, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    loop(bounds, stream)
    end.record(stream)
    torch.cuda.synchronize()
    loop_ms = (time.perf_counter() - t0) * 1e3
    loop_gpu_ms = start.elapsed_time(end)
    log(f"[bench] per-segment loop (eager): {loop_ms:.1f} ms wall, {loop_gpu_ms:.1f} ms on the stream")
    # Baseline 2: the same loop as consecutive graphs of LOOP_GRAPH_SEGMENTS
    # segments each, every graph replayed once per timed run.
    chunks = [bounds[i:i + LOOP_GRAPH_SEGMENTS] for i in range(0, len(bounds), LOOP_GRAPH_SEGMENTS)]
    graphs = []
    t0 = time.perf_counter()
    for ch in chunks:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(cap):
            with torch.cuda.graph(g, stream=cap):
                loop(ch, cap)
        graphs.append(g)
    torch.cuda.synchronize()
    log(f"[bench] per-segment loop captured as {len(graphs)} graphs of up to "
        f"{LOOP_GRAPH_SEGMENTS} segments ({time.perf_counter() - t0:.1f} s)")
    for g in graphs:
        g.replay()
    torch.cuda.synchronize()
    runs = []
    for _ in range(3):
        start.record()
        for g in graphs:
            g.replay()
        end.record()
        torch.cuda.synchronize()
        runs.append(start.elapsed_time(end))
    loop_graph_ms = statistics.median(runs)
    log(f"[bench] per-segment loop (graphs): {loop_graph_ms:.1f} ms (runs {runs})")
    del graphs
    return {
        "per_segment_loop_ms": round(loop_gpu_ms, 2),
        "per_segment_loop_wall_ms": round(loop_ms, 2),
        "per_segment_loop_graph_ms": round(loop_graph_ms, 2),
        "per_segment_loop_graph_chunks": f"{len(chunks)} graphs of up to {LOOP_GRAPH_SEGMENTS} "
                                         f"segments, {len(bounds)} segments in all",
        "speedup_vs_loop": round(loop_gpu_ms / ms_per_step, 1),
        "speedup_vs_loop_graph": round(loop_graph_ms / ms_per_step, 1),
    }


SEGMENT_CLASS_CAPACITY = (512, 2048, 8192)


def segment_class_keys(lengths, limits):
    """Keys per LDS class and in large segments, with the library's rule:
    class c takes lengths in (limit[c-1], limit[c]]; -1 = class unused,
    0 = the class's capacity."""
    import numpy as np
    eff, prev = [], 0
    for c, v in enumerate(limits):
        if v != -1:
            prev = max(prev, SEGMENT_CLASS_CAPACITY[c] if v == 0 else v)
        eff.append(prev)
    lengths = np.asarray(lengths)
    keys, lo = [], 0
    for hi in eff:
        keys.append(int(lengths[(lengths > lo) & (lengths <= hi)].sum()) if hi > lo else 0)
        lo = hi
    large = int(lengths[lengths > lo].sum())
    return keys, large


def per_kind_summary(per_kind, ow, lengths, limits, pair_bytes=8):
    """Average duration of every launch of the batched sort, and the roofline
    of the kernel kind that takes the most time per sort. Algorithmic bytes
    of a launch: one read and one write of every key and value it moves (LDS
    sort: the keys of its class; binning: the keys of the large segments)."""
    table, totals = {}, {}
    class_keys, large_keys = segment_class_keys(lengths, limits)
    lds_index = 0
    for (i, kind), ts in sorted(per_kind.items()):
        us = statistics.mean(ts) * 1e3
        table[f"{i}:{ow.KERNEL_NAMES[kind]}"] = round(us, 2)
        if kind == ow.KERNEL_LDS_SORT:
            moved = class_keys[lds_index] if lds_index < 3 else 0
            lds_index += 1
        elif kind == ow.KERNEL_BINNING:
            moved = large_keys
        else:
            continue
        t = totals.setdefault(kind, [0.0, 0, 0])
        t[0] += us
        t[1] += 1
        t[2] += 2 * pair_bytes * moved
    if not totals:
        return {"table": table, "dominant": (None, 0.0, 0), "roofline": None}
    kind = max(totals, key=lambda k: totals[k][0])
    us, launches, nbytes = totals[kind]
    per_launch_bytes = nbytes / launches
    avg_us = us / launches
    achieved = per_launch_bytes / (avg_us * 1e-6) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": ow.KERNEL_NAMES[kind], "algorithmic_bytes_per_launch": int(per_launch_bytes),
            "avg_launch_us": round(avg_us, 2)}
    return {"table": table, "dominant": (kind, avg_us, launches), "roofline": roof}


def ordered_bits_np(keys, key_kind, descending, np):
    """Raw key bits mapped onto unsigned order (signed: sign bit flipped;
    floating point: negative values fully complemented, others sign flipped;
    descending: complemented), a bijection on the bit patterns."""
    w = keys.dtype.itemsize * 8
    top = keys.dtype.type(1 << (w - 1))
    x = keys.copy()
    if key_kind == "signed":
        x ^= top
    elif key_kind == "float":
        neg = (x & top) != 0
        x[neg] = ~x[neg]
        x[~neg] ^= top
    if descending:
        x = ~x
    return x


def verify_output(keys, vals, d_kout, d_vout, key_kind, descending, np):
    """Checks the timed sort's output exactly, outside the timed region,
    with numpy only. Keys only: the stable result of a full-width sort is the
    sorted multiset, which numpy's sort gives. Pairs (values = input index):
    keys sorted as numpy sorts them, every value a distinct input index whose
    key sits at that position, and values increasing within runs of equal
    keys, which together fix the stable result uniquely. Returns an error
    message or None."""
    t0 = time.perf_counter()
    kout = d_kout.cpu().numpy()
    want = np.sort(ordered_bits_np(keys, key_kind, descending, np))
    if not np.array_equal(ordered_bits_np(kout, key_kind, descending, np), want):
        return "keys differ from the sorted input"
    del want
    if vals is not None:
        vout = d_vout.cpu().numpy()
        n = keys.size
        if int(vout.max(initial=0)) >= n:
            return "a value is not an input index"
        if np.count_nonzero(np.bincount(vout, minlength=n) != 1):
            return "values are not a permutation of the input indices"
        if not np.array_equal(keys[vout], kout):
            return "a value does not point at its key"
        tie = kout[1:] == kout[:-1]
        if np.any(vout[1:][tie] <= vout[:-1][tie]):
            return "equal keys out of input order (unstable)"
    log(f"[bench] output verified exactly against numpy ({time.perf_counter() - t0:.1f} s)")
    return None


def rts_baseline(ow, step, places, n, steps, stream, traced_configs, per_kind_times,
                 plain_config, check):
    """The reduce-then-scan baseline (Section 2: upsweep, tile scan and
    downsweep per place, ~3pn memory operations against Onesweep's
    ~(2p+1)n) timed on the same input, tile shape and buffers, right after
    the Onesweep steps. The speedup compares untraced sorts of both
    algorithms timed back to back: HIP events around every launch cost more
    for reduce-then-scan, which launches about twice as many kernels. A
    separate traced run gives the per-kernel averages."""
    import torch
    k = max(3, min(steps, 10))
    plain = {alg: plain_config(alg) for alg in (ow.ALGORITHM_ONESWEEP,
                                                ow.ALGORITHM_REDUCE_THEN_SCAN)}

    def timed(cfgs):
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        for cfg in cfgs:
            step(cfg)
        end.record(stream)
        torch.cuda.synchronize()
        return start.elapsed_time(end) / len(cfgs)

    step(plain[ow.ALGORITHM_REDUCE_THEN_SCAN])  # warm-up
    os_ms, rts_ms = [], []
    for _ in range(2):  # alternate, so clock drift touches both alike
        os_ms.append(timed([plain[ow.ALGORITHM_ONESWEEP]] * k))
        rts_ms.append(timed([plain[ow.ALGORITHM_REDUCE_THEN_SCAN]] * k))
    ms, onesweep_ms = min(rts_ms), min(os_ms)
    err = check()
    if err:
        log(f"[bench] ERROR: reduce-then-scan output: {err}")
        sys.exit(1)
    cfgs, holders = traced_configs(ow.ALGORITHM_REDUCE_THEN_SCAN, k)
    traced_ms = timed(cfgs)
    per_kind = per_kind_times(holders)
    avg = {ow.KERNEL_NAMES[kind]: round(statistics.mean(ts) * 1e3, 2)
           for kind, ts in sorted(per_kind.items())}
    log(f"[bench] reduce-then-scan: {ms:.3f} ms per sort ({n / (ms * 1e-3) / 1e9:.2f} GKeys/s), "
        f"Onesweep {onesweep_ms:.3f} ms, both untraced; traced {traced_ms:.3f} ms; "
        f"per-kernel avg us {avg}")
    return {
        "ms_per_step": round(ms, 4),
        "value": round(n / (ms * 1e-3) / 1e9, 3),
        "unit": "GKeys/s",
        "steps": k,
        "onesweep_ms_untraced": round(onesweep_ms, 4),
        "onesweep_speedup": round(ms / onesweep_ms, 3),
        "memory_ops_ratio": round(3 * places / (2 * places + 1), 3),
        "traced_ms_per_step": round(traced_ms, 4),
        "per_kernel_avg_us": avg,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="u32_keys_uniform",
                    choices=sorted(WORKLOADS) + sorted(SEGMENT_WORKLOADS))
    ap.add_argument("--segment-limits", type=int, nargs=3, default=(0, 0, 0))
    ap.add_argument("--segment-streams", type=int, default=0,
                    help="segmented workload: 0 two streams (default), 1 one stream")
    ap.add_argument("--no-loop-baseline", action="store_true",
                    help="segmented workload: skip the per-segment loop baselines")
    ap.add_argument("--no-segments", action="store_true",
                    help="default workload: skip the batched segmented sort beside it")
    ap.add_argument("--tune-segments", action="store_true",
                    help="segmented workload: time the configuration the autotuner picks on "
                         "this data instead of the command line's")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--ipt", type=int, default=0)
    ap.add_argument("--hist-blocks-per-cu", type=int, default=0)
    ap.add_argument("--rank", type=int, default=0, help="0 default, 1 ballot, 2 presence")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--algorithm", choices=("onesweep", "reduce-then-scan"), default="onesweep",
                    help="algorithm of the timed sort (reduce-then-scan: the Section 2 "
                         "baseline, for profiling it on its own)")
    ap.add_argument("--no-rts-baseline", action="store_true",
                    help="skip timing the reduce-then-scan baseline beside Onesweep")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run the library's plain copy kernel once on the input first "
                         "(known size: n keys read and written), for counter scaling")
    ap.add_argument("--counters-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="offline: summarise two rocprofv3 --pmc runs (FETCH_SIZE, "
                         "WRITE_SIZE) of this script into the traffic file and exit")
    args = ap.parse_args()

    if args.counters_summary:
        summarize_counters(*args.counters_summary, workload=args.workload)
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the sort is single-GPU; see DESIGN.md for how it would shard)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2206_01784_amd as ow

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload in SEGMENT_WORKLOADS:
        run_segments(args)
        return
    key_bits, has_vals, dist, log2n = WORKLOADS[args.workload]
    key_kind, descending = WORKLOAD_ORDER.get(args.workload, ("unsigned", False))
    key_type = {"unsigned": ow.KEY_UNSIGNED, "signed": ow.KEY_SIGNED,
                "float": ow.KEY_FLOAT}[key_kind]
    n = 1 << log2n
    log(f"[bench] workload={args.workload} n=2^{log2n} generating input")
    keys = make_keys(dist, n, key_bits)
    vals = np.arange(n, dtype=np.uint32) if has_vals else None
    d_keys = torch.from_numpy(keys).cuda()
    d_vals = torch.from_numpy(vals).cuda() if has_vals else None
    d_kout = torch.empty_like(d_keys)
    d_vout = torch.empty_like(d_vals) if has_vals else None

    places = key_bits // 8
    steps = args.steps
    stream = torch.cuda.current_stream()
    algorithm = (ow.ALGORITHM_REDUCE_THEN_SCAN if args.algorithm == "reduce-then-scan"
                 else ow.ALGORITHM_ONESWEEP)

    # Onesweep bins inputs above 2^29 keys in strips: one launch per strip
    # and place (each strip at most 2^29 keys, whole tiles).
    tile = ow.tile_items(key_bits, has_vals, ow.make_config(args.block, args.ipt,
                                                           rank_algorithm=args.rank), n)
    tiles = -(-n // tile)
    strips = -(-tiles // max(1, (1 << 29) // tile))

    def traced_configs(alg, count):
        """`count` configs, each recording HIP events around every launch on
        the stream the kernels run on."""
        rts_alg = alg == ow.ALGORITHM_REDUCE_THEN_SCAN
        # from 2^31 keys the histogram runs over portions of at most 2^30 keys
        portions = -(-n // (1 << 30)) if n >= (1 << 31) else 1
        launches = min(ow.TRACE_MAX, 2 + portions + places * (3 if rts_alg else strips) + 1)
        cfgs, holders = [], []
        for _ in range(count):
            evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * launches)]
            for e in evs:
                e.record(stream)
            arr = (ctypes.c_void_p * len(evs))(*[e.cuda_event for e in evs])
            tr = ow.Trace()
            tr.events = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
            tr.capacity = launches
            cfgs.append(ow.make_config(args.block, args.ipt, args.hist_blocks_per_cu,
                                       rank_algorithm=args.rank, algorithm=alg,
                                       key_type=key_type, descending=descending, trace=tr))
            holders.append((tr, evs, arr))
        return cfgs, holders

    def per_kind_times(holders):
        per_kind = {}
        for tr, evs, _ in holders:
            for i in range(tr.count):
                per_kind.setdefault(tr.kinds[i], []).append(
                    evs[2 * i].elapsed_time(evs[2 * i + 1]))
        return per_kind

    cfg_plain = ow.make_config(args.block, args.ipt, args.hist_blocks_per_cu,
                               rank_algorithm=args.rank, algorithm=algorithm,
                               key_type=key_type, descending=descending)
    cfgs, holders = traced_configs(algorithm, steps)
    temp_bytes = ow.sort_temp_bytes(n, key_bits, has_vals, config=cfg_plain)
    if not args.no_rts_baseline:
        temp_bytes = max(temp_bytes, ow.sort_temp_bytes(
            n, key_bits, has_vals, config=ow.make_config(
                args.block, args.ipt, args.hist_blocks_per_cu, rank_algorithm=args.rank,
                algorithm=ow.ALGORITHM_REDUCE_THEN_SCAN)))
    temp = torch.empty(temp_bytes, dtype=torch.uint8, device="cuda")

    def step(cfg):
        if has_vals:
            ow.sort_pairs(d_keys, d_vals, keys_out=d_kout, values_out=d_vout, temp=temp,
                          config=cfg, stream=stream)
        else:
            ow.sort_keys(d_keys, out=d_kout, temp=temp, config=cfg, stream=stream)

    if args.calibrate_copy:
        # An empty bit range makes the sort a plain copy: one launch of the
        # copy kernel reading and writing n keys (and values).
        if has_vals:
            ow.sort_pairs(d_keys, d_vals, 0, 0, keys_out=d_kout, values_out=d_vout,
                          stream=stream)
        else:
            ow.sort_keys(d_keys, 0, 0, out=d_kout, stream=stream)
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        step(cfg_plain)
    torch.cuda.synchronize()

    # The timed region: `steps` whole sorts back to back, with events only at
    # its two ends (nothing else on the stream).
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record(stream)
    for k in range(steps):
        step(cfg_plain)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = start.elapsed_time(end)
    ms_per_step = ms_total / steps
    value = n / (ms_per_step * 1e-3) / 1e9
    log(f"[bench] {steps} steps in {ms_total:.3f} ms (wall {wall * 1e3:.1f} ms)")
    # The same steps again with HIP events around every launch, on the stream
    # the kernels run on: per-kernel durations and per-step spreads. The
    # events are packets of their own between the kernels, so these steps
    # run slightly longer than the timed ones.
    t0_, t1_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0_.record(stream)
    for k in range(steps):
        step(cfgs[k])
    t1_.record(stream)
    torch.cuda.synchronize()
    traced_ms = t0_.elapsed_time(t1_) / steps
    log(f"[bench] traced steps: {traced_ms:.4f} ms per step (timed, untraced: {ms_per_step:.4f} ms)")

    # Per-step durations (first launch's start to last launch's end of each
    # traced step): median, min and interquartile range.
    step_ms = sorted(evs[0].elapsed_time(evs[2 * tr.count - 1]) for tr, evs, _ in holders
                     if tr.count > 0)
    q = lambda f: step_ms[min(len(step_ms) - 1, int(f * (len(step_ms) - 1) + 0.5))]  # noqa: E731
    step_stats = {"median_ms": round(q(0.5), 4), "min_ms": round(step_ms[0], 4),
                  "iqr_ms": round(q(0.75) - q(0.25), 4)}
    log(f"[bench] per traced step: median {step_stats['median_ms']} ms, min "
        f"{step_stats['min_ms']} ms, IQR {step_stats['iqr_ms']} ms")

    # Per-kernel durations from the traced events.
    per_kind = per_kind_times(holders)
    for kind, ts in sorted(per_kind.items()):
        log(f"[bench]   {ow.KERNEL_NAMES[kind]:9s} launches={len(ts):4d} "
            f"avg={statistics.mean(ts) * 1e3:9.2f} us  total/step={sum(ts) / steps * 1e3:9.2f} us")

    # Exact check of the timed result (every step wrote the same output).
    err = verify_output(keys, vals, d_kout, d_vout, key_kind, descending, np)
    if err:
        log(f"[bench] ERROR: {err}")
        sys.exit(1)

    kb = key_bits // 8
    vb = 4 if has_vals else 0
    scatter_kind = (ow.KERNEL_DOWNSWEEP if algorithm == ow.ALGORITHM_REDUCE_THEN_SCAN
                    else ow.KERNEL_BINNING)
    bin_ts = per_kind.get(scatter_kind, [])
    binning_avg_s = statistics.mean(bin_ts) * 1e-3 if bin_ts else float("nan")
    # each binning pass reads and writes every element once, over `strips`
    # launches (the reduce-then-scan downsweep: one launch)
    pass_bytes = n * 2 * (kb + vb)
    launch_bytes = pass_bytes // (strips if algorithm == ow.ALGORITHM_ONESWEEP else 1)
    achieved = launch_bytes / binning_avg_s / 1e9
    traffic = read_traffic(args.workload) if algorithm == ow.ALGORITHM_ONESWEEP else None
    sort_bytes = n * kb + places * pass_bytes  # (2p+1)n element moves
    whole_gbs = sort_bytes / (ms_per_step * 1e-3) / 1e9
    log(f"[bench] whole sort: {whole_gbs:.1f} GB/s algorithmic = {whole_gbs / HBM_PEAK_GBS:.3f} "
        f"of peak; binning: {achieved:.1f} GB/s")
    # Context: the library's plain copy kernel on the same buffers (an empty
    # bit range sorts nothing), timed after the sort steps.
    def copy_once():
        if has_vals:
            ow.sort_pairs(d_keys, d_vals, 0, 0, keys_out=d_kout, values_out=d_vout, temp=temp,
                          stream=stream)
        else:
            ow.sort_keys(d_keys, 0, 0, out=d_kout, temp=temp, stream=stream)
    copy_once()
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(5):
        copy_once()
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * n * (kb + vb) / (c0.elapsed_time(c1) / 5 * 1e-3) / 1e9
    log(f"[bench] copy kernel: {copy_gbs:.1f} GB/s; whole sort at "
        f"{whole_gbs / copy_gbs:.3f} of it, binning at {achieved / copy_gbs:.3f}")

    result = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GKeys/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32" if key_bits == 32 else "u64",
        "data": "synthetic",
        "config": {
            "workload": f"stable {'descending ' if descending else ''}sort of 2^{log2n} {dist} "
                        f"{ {'unsigned': 'uint', 'signed': 'int', 'float': 'float'}[key_kind]}"
                        f"{key_bits} "
                        f"{'(key, uint32 value) pairs' if has_vals else 'keys (keys only)'}, "
                        f"8-bit digits, {places} binning passes",
            "n": n, "key_bits": key_bits, "values": has_vals, "distribution": dist,
            "key_type": key_kind, "descending": descending,
            "tile": ow.tile_items(key_bits, has_vals, cfg_plain, n),
            "hbm_fraction_whole_sort": round(whole_gbs / HBM_PEAK_GBS, 4),
            "copy_kernel_gbs": round(copy_gbs, 1),
            "whole_sort_over_copy": round(whole_gbs / copy_gbs, 4),
            "per_traced_step": step_stats,
            "traced_ms_per_step": round(traced_ms, 4),
            "output_verified": "exact, against numpy's sort of the input",
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": ow.KERNEL_NAMES[scatter_kind],
            "algorithmic_bytes_per_launch": launch_bytes,
            "avg_launch_us": round(binning_avg_s * 1e6, 2),
        },
        "cpu_baseline": None,
    }
    if algorithm != ow.ALGORITHM_ONESWEEP:
        result["config"]["algorithm"] = "reduce-then-scan"
    if not args.no_rts_baseline and algorithm == ow.ALGORITHM_ONESWEEP:
        def plain_config(alg):
            return ow.make_config(args.block, args.ipt, args.hist_blocks_per_cu,
                                  rank_algorithm=args.rank, algorithm=alg,
                                  key_type=key_type, descending=descending)
        result["reduce_then_scan"] = rts_baseline(
            ow, step, places, n, steps, stream, traced_configs, per_kind_times, plain_config,
            lambda: verify_output(keys, vals, d_kout, d_vout, key_kind, descending, np))
    if not args.no_segments and args.workload == "u32_keys_uniform":
        # The batched form beside the plain sort: the segmented workload in
        # the configuration the autotuner picks on it, against the
        # per-segment loop of plain pair sorts.
        S, log2n_s = SEGMENT_WORKLOADS["segments_lognormal_20000"]
        leg = segments_leg(args, S, log2n_s, tune=True, with_loops=True)
        b = leg["baselines"]
        result["segments"] = {
            "workload": f"batched stable sort of {S} segments (log-normal lengths, median 2000, "
                        f"sigma 1.5, scaled to 2^{log2n_s} uint32 key/value pairs), one graph "
                        "replay per step",
            "n": leg["n"], "ms_per_step": round(leg["ms_per_step"], 4),
            "value": round(leg["value"], 3), "unit": "GKeys/s",
            "tile": f"{leg['block']}x{leg['ipt']}", "segment_limits": list(leg["limits"]),
            "autotuned": True,
            "per_segment_loop_ms": b["per_segment_loop_ms"],
            "per_segment_loop_graph_ms": b["per_segment_loop_graph_ms"],
            "speedup_vs_loop": b["speedup_vs_loop"],
            "speedup_vs_loop_graph": b["speedup_vs_loop_graph"],
        }
        del leg
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on the whole input")
        result["cpu_baseline"] = cpu_baseline(keys, vals)
        log("[bench] timing the multithreaded CPU sort on the whole input")
        result["cpu_parallel_baseline"] = cpu_parallel_baseline(keys, vals)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
