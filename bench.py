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
    "u32_pairs_uniform": (32, True, "uniform", 28),
    "u64_pairs_uniform": (64, True, "uniform", 27),
    "u32_keys_uniform_2p20": (32, False, "uniform", 20),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(launch_bytes_alg: float):
    """HBM traffic per binning launch from the committed rocprofv3 counter
    summary, or None when it is missing or the kernel source changed since."""
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

    def pick(d, sub):
        vals = [v for k, vs in d.items() if sub in k for v in vs]
        if not vals:
            raise SystemExit(f"no dispatches of {sub} in the counter file")
        return vals

    copy_f = max(pick(fetch, "copy_kernel")) * 1024
    copy_w = max(pick(write, "copy_kernel")) * 1024
    bin_f = st.mean(pick(fetch, "binning_kernel")) * 1024
    bin_w = st.mean(pick(write, "binning_kernel")) * 1024
    f_scale, w_scale = copy_bytes / copy_f, copy_bytes / copy_w
    traffic = bin_f * f_scale + bin_w * w_scale
    alg = n * 2 * (key_bits // 8 + (4 if has_vals else 0))
    lines = [
        "# HBM traffic of one binning launch, from two rocprofv3 --pmc runs of bench.py",
        f"# workload: {workload} (n = 2^{log2n})",
        f"# fetch csv: {os.path.basename(fetch_csv)}; write csv: {os.path.basename(write_csv)}",
        "# scale = bytes the plain copy kernel must move / its counter reading",
        "# commands (repo root; run from /tmp with TMPDIR=/tmp):",
        "#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o fetch -- "
        f"python bench.py --workload {workload} --steps 2 --warmup 0 --no-cpu-baseline --calibrate-copy",
        "#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o write -- "
        f"python bench.py --workload {workload} --steps 2 --warmup 0 --no-cpu-baseline --calibrate-copy",
        "#   python bench.py --workload " + workload + " --counters-summary <fetch csv> <write csv>",
        f"kernel_source_sha256_16: {kernel_source_hash()}",
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


def make_keys(dist, n, key_bits, seed=2):
    import workload as W
    if dist == "uniform":
        return W.uniform(seed, n, key_bits)
    if dist == "equal":
        return W.all_equal(seed, n, key_bits)
    return W.make_keys(dist, seed, n, key_bits)


def cpu_baseline(keys, vals, target_s=10.0):
    """The CPU oracle, single-threaded, on a bounded sample of the same input."""
    import numpy as np
    import oracle
    sample = min(keys.size, 1 << 26)
    ks = np.ascontiguousarray(keys[:sample])
    vs = None if vals is None else np.ascontiguousarray(vals[:sample])
    times = []
    t_start = time.perf_counter()
    while len(times) < 3 or (time.perf_counter() - t_start < target_s and len(times) < 10):
        t0 = time.perf_counter()
        oracle.sort(ks, vs)
        times.append(time.perf_counter() - t0)
    med = statistics.median(times)
    return {"value": round(sample / med / 1e9, 4), "unit": "GKeys/s", "cores": 1,
            "kind": "oracle",
            "sample": f"first 2^{sample.bit_length() - 1} keys of the same input, "
                      f"median of {len(times)} single-threaded runs"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="u32_keys_uniform", choices=sorted(WORKLOADS))
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--ipt", type=int, default=0)
    ap.add_argument("--hist-blocks-per-cu", type=int, default=0)
    ap.add_argument("--rank", type=int, default=0, help="0 default, 1 ballot, 2 presence")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    key_bits, has_vals, dist, log2n = WORKLOADS[args.workload]
    n = 1 << log2n
    log(f"[bench] workload={args.workload} n=2^{log2n} generating input")
    keys = make_keys(dist, n, key_bits)
    vals = np.arange(n, dtype=np.uint32) if has_vals else None
    d_keys = torch.from_numpy(keys).cuda()
    d_vals = torch.from_numpy(vals).cuda() if has_vals else None
    d_kout = torch.empty_like(d_keys)
    d_vout = torch.empty_like(d_vals) if has_vals else None

    places = key_bits // 8
    launches_per_step = 3 + places + 1
    steps = args.steps
    stream = torch.cuda.current_stream()

    # Per-launch HIP events on the stream the kernels run on.
    traces, holders = [], []
    for _ in range(steps):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * launches_per_step)]
        for e in evs:
            e.record(stream)
        arr = (ctypes.c_void_p * len(evs))(*[e.cuda_event for e in evs])
        tr = ow.Trace()
        tr.events = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
        tr.capacity = launches_per_step
        traces.append(tr)
        holders.append((evs, arr))
    cfg_plain = ow.make_config(args.block, args.ipt, args.hist_blocks_per_cu,
                               rank_algorithm=args.rank)
    cfgs = [ow.make_config(args.block, args.ipt, args.hist_blocks_per_cu,
                           rank_algorithm=args.rank, trace=tr) for tr in traces]
    temp = torch.empty(ow.sort_temp_bytes(n, key_bits, has_vals, config=cfg_plain),
                       dtype=torch.uint8, device="cuda")

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

    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record(stream)
    for k in range(steps):
        step(cfgs[k])
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = start.elapsed_time(end)
    ms_per_step = ms_total / steps
    value = n / (ms_per_step * 1e-3) / 1e9
    log(f"[bench] {steps} steps in {ms_total:.3f} ms (wall {wall * 1e3:.1f} ms)")

    # Per-kernel durations from the traced events.
    per_kind = {}
    for tr, (evs, _) in zip(traces, holders):
        for i in range(tr.count):
            per_kind.setdefault(tr.kinds[i], []).append(evs[2 * i].elapsed_time(evs[2 * i + 1]))
    for kind, ts in sorted(per_kind.items()):
        log(f"[bench]   {ow.KERNEL_NAMES[kind]:9s} launches={len(ts):4d} "
            f"avg={statistics.mean(ts) * 1e3:9.2f} us  total/step={sum(ts) / steps * 1e3:9.2f} us")

    # Correctness spot check of the timed result (full check lives in tests/).
    out = d_kout.cpu().numpy()
    sorted_ok = bool(np.all(out[1:] >= out[:-1]))
    if not sorted_ok:
        log("[bench] ERROR: output is not sorted")
        sys.exit(1)

    kb = key_bits // 8
    vb = 4 if has_vals else 0
    bin_ts = per_kind.get(ow.KERNEL_BINNING, [])
    binning_avg_s = statistics.mean(bin_ts) * 1e-3 if bin_ts else float("nan")
    launch_bytes = n * 2 * (kb + vb)  # each binning pass reads and writes every element once
    achieved = launch_bytes / binning_avg_s / 1e9
    traffic = read_traffic(launch_bytes)
    sort_bytes = n * kb + places * launch_bytes  # (2p+1)n element moves
    whole_gbs = sort_bytes / (ms_per_step * 1e-3) / 1e9
    log(f"[bench] whole sort: {whole_gbs:.1f} GB/s algorithmic = {whole_gbs / HBM_PEAK_GBS:.3f} "
        f"of peak; binning: {achieved:.1f} GB/s")

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
            "workload": f"stable sort of 2^{log2n} {dist} uint{key_bits} "
                        f"{'(key, uint32 value) pairs' if has_vals else 'keys (keys only)'}, "
                        f"8-bit digits, {places} binning passes",
            "n": n, "key_bits": key_bits, "values": has_vals, "distribution": dist,
            "tile": ow.tile_items(key_bits, has_vals, cfg_plain),
            "hbm_fraction_whole_sort": round(whole_gbs / HBM_PEAK_GBS, 4),
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "binning",
            "algorithmic_bytes_per_launch": launch_bytes,
            "avg_launch_us": round(binning_avg_s * 1e6, 2),
        },
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        result["cpu_baseline"] = cpu_baseline(keys, vals)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
