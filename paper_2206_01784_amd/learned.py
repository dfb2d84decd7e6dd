"""Training data, training and evaluation of the configuration-selection MLP.

Every number here comes from the library itself: sort times of each model
class measured with HIP events on the GPU, features from the library's
feature kernel, training steps from its HIP training kernels.

    python -m paper_2206_01784_amd.learned collect --seeds 10000:10400 --out train.npz
    python -m paper_2206_01784_amd.learned train --data train.npz --out model.bin
    python -m paper_2206_01784_amd.learned evaluate --model model.bin --seeds 1000:1200

Inputs follow the seeded sweep of the `workload` package: n = round(2^(17 + 11u)),
key widths alternating 32/64 bits, distributions cycling over AND-of-1..4,
Zipf(1.1), presorted, reverse-sorted and 16 distinct values.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import (FEATURES, MODEL_CLASSES, Config, Model, OnesweepError, features, select_config,
               sort_keys, sort_learned, sort_pairs, sort_temp_bytes, tile_items)

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)
import workload as W  # noqa: E402  (seeded input generators shared with the tests)

DEFAULT_MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config_model.bin")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sweep_keys(seed: int, device="cuda"):
    """(keys on the device, n, key_bits, distribution) of one sweep input.

    Equal to workload.make_keys for the same case; the sorting and
    inverse-CDF steps of the presorted, reverse and Zipf inputs run on the GPU
    (torch) so that inputs of 2^28 keys take seconds, not minutes.
    """
    n, kb, dist = W.sweep_case(seed)
    if dist in ("presorted", "reverse"):
        t = torch.from_numpy(W.uniform(seed, n, kb)).to(device)
        t = sort_keys(t)
        if dist == "reverse":
            signed = torch.int32 if kb == 32 else torch.int64
            t = torch.flip(t.view(signed), dims=[0]).contiguous().view(t.dtype)
    elif dist == "zipf":
        support, s = 1 << 20, 1.1
        ranks = np.arange(1, support + 1, dtype=np.float64)
        cdf = np.cumsum(ranks ** (-s))
        cdf /= cdf[-1]
        u = torch.from_numpy(W.unit_doubles(seed, 1, n)).to(device)
        k = torch.searchsorted(torch.from_numpy(cdf).to(device), u, side="left")
        k = torch.clamp(k, max=support - 1)
        t = k.to(torch.int32).view(torch.uint32) if kb == 32 else k.view(torch.uint64)
        t = t.contiguous()
    else:
        t = torch.from_numpy(W.make_keys(dist, seed, n, kb)).to(device)
    return t, n, kb, dist


def model_classes(model: Model):
    return [model.class_config(c) for c in range(MODEL_CLASSES)]


def _timed(fn, reps: int) -> float:
    """Mean milliseconds of `reps` back-to-back calls after one warm-up."""
    fn()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def reps_for(n: int) -> int:
    return int(min(50, max(3, (1 << 24) // max(n, 1))))


def time_classes(keys, kb, has_values, classes, reps):
    """Sort time (ms) of every class that applies to kb (nan elsewhere) and of
    the library default."""
    n = keys.numel()
    vals = torch.arange(n, dtype=torch.int32, device=keys.device).view(torch.uint32) \
        if has_values else None
    out = torch.empty_like(keys)
    vout = torch.empty_like(vals) if has_values else None
    cfgs = [Config()] + [c for c, _ in classes]
    need = max(sort_temp_bytes(n, kb, has_values, config=c)
               for c, m in [(Config(), 3)] + classes if m & (1 if kb == 32 else 2))
    temp = torch.empty(max(need, 1), dtype=torch.uint8, device=keys.device)

    def run(cfg):
        if has_values:
            return lambda: sort_pairs(keys, vals, keys_out=out, values_out=vout, temp=temp,
                                      config=cfg)
        return lambda: sort_keys(keys, out=out, temp=temp, config=cfg)

    times = np.full(MODEL_CLASSES, np.nan)
    for c, (cfg, mask) in enumerate(classes):
        if mask & (1 if kb == 32 else 2):
            times[c] = _timed(run(cfg), reps)
    default = _timed(run(cfgs[0]), reps)
    return times, default, (out, vout, temp)


def collect(seeds, out_path: str, pairs_every: int = 2):
    """Timing records of the model classes over sweep inputs."""
    model = Model(max_batch=1)
    classes = model_classes(model)
    feats, times, defaults, meta = [], [], [], []
    t0 = time.time()
    for i, seed in enumerate(seeds):
        keys, n, kb, dist = sweep_keys(seed)
        has_values = (seed // 8) % pairs_every == 1
        f = features(keys, 0, kb, has_values).cpu().numpy()
        t, d, _ = time_classes(keys, kb, has_values, classes, reps_for(n))
        feats.append(f)
        times.append(t)
        defaults.append(d)
        meta.append((seed, n, kb, int(has_values)))
        log(f"[collect] {i + 1}/{len(seeds)} seed={seed} n={n} kb={kb} vals={int(has_values)} "
            f"{dist}: best {np.nanmin(t):.4f} ms (class {int(np.nanargmin(t))}), default "
            f"{d:.4f} ms, {time.time() - t0:.0f} s")
        del keys
        torch.cuda.empty_cache()
        if (i + 1) % 25 == 0 or i + 1 == len(seeds):  # partial results survive a time limit
            np.savez(out_path, features=np.array(feats, dtype=np.float32),
                     times=np.array(times), default=np.array(defaults),
                     meta=np.array(meta, dtype=np.int64))


def targets(times: np.ndarray):
    """y = log(t / fastest) of the classes that were timed, mask = timed."""
    mask = np.isfinite(times).astype(np.float32)
    best = np.nanmin(times, axis=1, keepdims=True)
    y = np.where(mask > 0, np.log(np.where(mask > 0, times, 1.0) / best), 0.0)
    return y.astype(np.float32), mask


def glorot_params(seed: int) -> np.ndarray:
    """Glorot-uniform weights, zero biases (layer shapes of the library's MLP)."""
    shapes = [(256, 16), (16,), (131, 64), (64,), (64, 64), (64,), (64, 12), (12,)]
    rng = np.random.default_rng(seed)
    parts = []
    for sh in shapes:
        if len(sh) == 2:
            a = math.sqrt(6.0 / (sh[0] + sh[1]))
            parts.append(rng.uniform(-a, a, size=sh).ravel())
        else:
            parts.append(np.zeros(sh))
    return np.concatenate(parts).astype(np.float32)


def train(data_paths, out_path: str, steps: int = 3000, lr: float = 3e-3, seed: int = 0):
    feats, times = [], []
    for p in data_paths:
        d = np.load(p)
        feats.append(d["features"])
        times.append(d["times"])
    x = np.concatenate(feats).astype(np.float32)
    y, mask = targets(np.concatenate(times))
    B = x.shape[0]
    model = Model(max_batch=B)
    model.set_params(glorot_params(seed))
    dx = torch.from_numpy(x).cuda()
    split = (dx[:, : FEATURES - 3].contiguous(), dx[:, FEATURES - 3:].contiguous())
    dy = torch.from_numpy(y).cuda()
    dm = torch.from_numpy(mask).cuda()
    losses = []
    for step in range(steps):
        loss = model.train_step(dx, dy, dm, lr, split=split)
        if step % 500 == 0 or step == steps - 1:
            losses.append(float(loss.cpu()))
            log(f"[train] step {step} loss {losses[-1]:.5f}")
    model.save(out_path)
    return model, losses


def reference_sorted(keys: torch.Tensor) -> torch.Tensor:
    """The keys sorted ascending as unsigned integers, by torch's own sort
    (an implementation independent of this library): 32-bit keys widened to
    int64, 64-bit keys with the sign bit flipped so signed order is unsigned
    order."""
    if keys.dtype == torch.uint32:
        wide = keys.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        return torch.sort(wide).values.to(torch.int32).view(torch.uint32)
    top = torch.tensor(-(1 << 63), dtype=torch.int64, device=keys.device)
    flipped = keys.view(torch.int64) ^ top
    return (torch.sort(flipped).values ^ top).view(torch.uint64)


def evaluate(model_path: str | None, seeds, reps_scale: int = 1):
    """The learned sort against the library default over sweep inputs (keys
    only). Per input: the default sort, the learned sort (selection included:
    onesweep_sort_learned overlaps it with the first phases), the model's
    pick timed without selection, and every class (for regret). Every output
    of the learned sort is checked against torch's sort of the keys.

    gain = default time / learned time; regret = learned time / best class
    time - 1.
    """
    model = Model(max_batch=1, path=model_path) if model_path else None
    probe = Model(max_batch=1)
    classes = model_classes(probe)
    rows = []
    for seed in seeds:
        keys, n, kb, dist = sweep_keys(seed)
        reps = reps_for(n) * reps_scale
        t, d, (out, _, temp) = time_classes(keys, kb, False, classes, reps)
        lout, _, used = sort_learned(model, keys)
        torch.cuda.synchronize()
        want = reference_sorted(keys)
        if not torch.equal(lout.view(want.dtype), want):
            raise RuntimeError(f"seed {seed}: the learned sort's output differs from torch.sort")
        del want
        ltemp = torch.empty(max(1, temp.numel()), dtype=torch.uint8, device=keys.device)
        learned_ms = _timed(lambda: sort_learned(model, keys, out=lout), reps)
        pick_ms = _timed(lambda: sort_keys(keys, out=out, temp=temp, config=used), reps)
        best = float(np.nanmin(t))
        rows.append(dict(seed=seed, n=n, key_bits=kb, dist=dist, best_ms=best, default_ms=d,
                         learned_ms=learned_ms, pick_ms=pick_ms,
                         pick=[used.block_threads, used.items_per_thread, used.rank_algorithm]))
        log(f"[eval] seed={seed} n={n} kb={kb} {dist}: best {best:.4f} default {d:.4f} "
            f"learned {learned_ms:.4f} (pick {pick_ms:.4f}) ms, pick {rows[-1]['pick']}")
        del keys, out, temp, lout, ltemp
        torch.cuda.empty_cache()
    return summarize(rows), rows


def summarize(rows):
    best = np.array([r["best_ms"] for r in rows])
    default = np.array([r["default_ms"] for r in rows])
    learned = np.array([r["learned_ms"] for r in rows])
    pick = np.array([r["pick_ms"] for r in rows])
    n = np.array([r["n"] for r in rows])
    geo = lambda a: float(np.exp(np.mean(np.log(a))))  # noqa: E731
    sel = n >= (1 << 26)
    out = {
        "inputs": len(rows),
        "gain_geomean": geo(default / learned),
        "gain_geomean_without_selection": geo(default / pick),
        "regret_mean": float(np.mean(learned / best - 1)),
        "best_over_default_geomean": geo(default / best),
        "inputs_selected": int(sel.sum()),
    }
    if sel.any():
        out["gain_geomean_selected"] = geo(default[sel] / learned[sel])
        out["best_over_default_geomean_selected"] = geo(default[sel] / best[sel])
    return out


def _seeds(spec: str):
    a, b = spec.split(":")
    return list(range(int(a), int(b)))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--seeds", required=True)
    c.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--data", nargs="+", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--steps", type=int, default=3000)
    t.add_argument("--lr", type=float, default=3e-3)
    e = sub.add_parser("evaluate")
    e.add_argument("--model", default=DEFAULT_MODEL)
    e.add_argument("--seeds", required=True)
    e.add_argument("--out")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    if args.cmd == "collect":
        collect(_seeds(args.seeds), args.out)
    elif args.cmd == "train":
        _, losses = train(args.data, args.out, args.steps, args.lr)
        print(json.dumps({"losses": losses}))
    else:
        summary, rows = evaluate(args.model, _seeds(args.seeds))
        print(json.dumps(summary))
        if args.out:
            with open(args.out, "w") as f:
                json.dump({"summary": summary, "rows": rows}, f)


if __name__ == "__main__":
    main()
