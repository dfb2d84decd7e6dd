"""Host-side logic of bench.py (no GPU): the one-GPU contract and the
rocprofv3 counter summary that feeds roofline.traffic."""
import csv
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def write_counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Value": value})


def test_counter_summary_scales_by_the_copy_and_keeps_chained_binning_only(tmp_path,
                                                                           monkeypatch):
    bench = load_bench()
    out = tmp_path / "traffic.txt"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    n = 1 << 28
    chained = "void onesweep::binning_kernel<unsigned int, false, 1024, 8, 0, 0, false, unsigned int>(x)"
    downsweep = "void onesweep::binning_kernel<unsigned int, false, 1024, 8, 0, 2, false, unsigned int>(x)"
    copy = "onesweep::copy_kernel(onesweep::CopyArgs)"
    # FETCH_SIZE reads half the true bytes, WRITE_SIZE the true bytes (KiB)
    write_counters(tmp_path / "f.csv", [(copy, n * 4 / 2 / 1024), (chained, 600000.0),
                                        (chained, 700000.0), (downsweep, 9e9)])
    write_counters(tmp_path / "w.csv", [(copy, n * 4 / 1024), (chained, 1200000.0),
                                        (chained, 1300000.0), (downsweep, 9e9)])
    bench.summarize_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"),
                             workload="u32_keys_uniform")
    kv = dict(line.split(":", 1) for line in out.read_text().splitlines()
              if ":" in line and not line.startswith("#"))
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    assert float(kv["fetch_scale"]) == 2.0 and float(kv["write_scale"]) == 1.0
    want = (650000.0 * 2 + 1250000.0) * 1024
    assert abs(float(kv["hbm_bytes_per_launch"]) - want) < 2
    assert kv["workload"] == "u32_keys_uniform"
    assert kv["kernel_source_sha256_16"] == bench.kernel_source_hash()
    # read back only for its own workload and the current kernel sources
    assert abs(bench.read_traffic("u32_keys_uniform") - want) < 2
    assert bench.read_traffic("u32_pairs_uniform") is None


class _Host:
    """Stands in for a device tensor: .cpu().numpy() returns the array."""

    def __init__(self, a):
        self.a = a

    def cpu(self):
        return self

    def numpy(self):
        return self.a


def test_output_verification_accepts_the_stable_sort_and_rejects_wrong_ones():
    import numpy as np
    bench = load_bench()
    rng = np.random.default_rng(5)
    keys = rng.integers(0, 50, 5000).astype(np.uint32)  # many ties
    vals = np.arange(keys.size, dtype=np.uint32)
    order = np.argsort(keys, kind="stable").astype(np.uint32)
    ko, vo = keys[order], order
    check = lambda k, v, kind="unsigned", desc=False: bench.verify_output(  # noqa: E731
        keys, vals, _Host(k), None if v is None else _Host(v), kind, desc, np)
    assert check(ko, vo) is None
    assert bench.verify_output(keys, None, _Host(ko), None, "unsigned", False, np) is None
    # same byte histograms, sum, XOR and order as a sorted {0x0101, 0x0202}, yet wrong
    two = np.array([0x0101, 0x0202], dtype=np.uint32)
    bad = np.array([0x0102, 0x0201], dtype=np.uint32)
    assert bench.verify_output(two, None, _Host(bad), None, "unsigned", False, np)
    unstable = vo.copy()
    i = int(np.flatnonzero(ko[1:] == ko[:-1])[0])
    unstable[i], unstable[i + 1] = unstable[i + 1], unstable[i]
    assert "unstable" in check(ko, unstable)
    wrong = vo.copy()
    wrong[0], wrong[-1] = wrong[-1], wrong[0]
    assert check(ko, wrong)
    dup = vo.copy()
    dup[1] = dup[0]
    assert "permutation" in check(ko, dup)
    # signed and descending orders
    s = rng.integers(-100, 100, 3000).astype(np.int32)
    want = np.sort(s)[::-1].copy()
    assert bench.verify_output(s.view(np.uint32), None, _Host(want.view(np.uint32)), None,
                               "signed", True, np) is None
    assert bench.verify_output(s.view(np.uint32), None, _Host(np.sort(s).view(np.uint32)), None,
                               "signed", True, np)
