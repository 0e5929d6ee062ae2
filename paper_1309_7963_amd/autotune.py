"""Autotuner for the persistent kernel's launch policy.

Sweeps the launch options that decide how a wave keeps its lanes busy and
where its data lives, on the caller's workload:

* launch: block size (waves per workgroup) and resident waves per CU
  (events in flight);
* thresholds: the per-state lane thresholds of the wave scheduler (how many
  lanes must wait in the kinematics, tentative-collision or flight-start
  state before the wave runs that state);
* stack_levels: how many entries of each lane's LIFO stay in LDS (the rest in
  private memory): none, 1, 2 or as many as fit;
* chunk_events: events a wave claims from the work queue at once;
* table_layout: the NN table in LDS as columns or as node pairs (one 8-byte
  read per interpolation for twice the LDS, which can cost a LIFO level).

The dimensions are swept one after another (coordinate descent): each
candidate of a dimension is timed with the best choices so far for the
others, and the dimension's fastest candidate is kept.  Each timing is a
warm-up launch, then the median of `repeats` launches (HIP events).  The
resulting policy and the library's default are then re-timed in interleaved
rounds, and the policy replaces the default only if it is faster by more than
`margin` (launch times drift by a few per cent, so a noisy winner would
otherwise make the launch slower).  The result (options {} = the library
default) is cached in a JSON file keyed by GPU architecture and workload
signature (targets, energy range), so later contexts can reuse it.  No
option changes the events, only their speed.

    from paper_1309_7963_amd import autotune
    best = autotune.tune([(16, 8), (40, 20)], T0, tidx)
    ctx = paper_1309_7963_amd.Context(targets, **best["options"])
"""
from __future__ import annotations

import json
import os
import time
from typing import Optional

import numpy as np

DEFAULT_DIMENSIONS = {
    "launch": tuple(dict(block_size=b, waves_per_cu=w) for b in (128, 256) for w in (8, 12, 16)),
    # (kinematics, tentative collision, flight start) lane thresholds
    "thresholds": tuple(dict(kin_threshold=k, tent_threshold=t, start_threshold=s)
                        for k, t, s in ((24, 24, 8), (24, 32, 8), (16, 32, 8), (16, 16, 8), (24, 12, 4), (16, 8, 8))),
    "stack_levels": tuple(dict(stack_levels=v) for v in (-1, 1, 2, 0)),
    "chunk_events": tuple(dict(chunk_events=c) for c in (32, 64, 128, 256)),
    "table_layout": tuple(dict(table_layout=v) for v in (0, 1)),
}


def cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "paper_1309_7963_amd", "autotune.json")


def signature(targets, T0) -> str:
    t = ",".join("%d-%d" % (a, z) for a, z in sorted(set(map(tuple, targets))))
    lo, hi = float(np.min(T0)), float(np.max(T0))
    return "%s|%d-%d" % (t, int(lo // 10) * 10, int(np.ceil(hi / 10)) * 10)


def _arch() -> str:
    import torch

    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _time(targets, T0_d, tidx_d, opts, repeats, mode):
    import torch

    import paper_1309_7963_amd as inc

    ctx = inc.Context(targets, **opts)
    n = int(T0_d.shape[0])
    out = inc.DeviceOutput.allocate(n, ctx.default_capacity(n))
    stream = torch.cuda.current_stream()
    ctx.simulate(T0_d, seed=1, target_idx=tidx_d, out=out, mode=mode)
    times = []
    for k in range(repeats):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        ctx.simulate(T0_d, seed=1, target_idx=tidx_d, out=out, first_event_id=(k + 1) * n, mode=mode)
        b.record(stream)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    ctx.close()
    return float(np.median(times))


def tune(targets, T0, tidx=None, dimensions: Optional[dict] = None, repeats: int = 3, use_cache: bool = True,
         verbose: bool = False, mode: str = "staged", rounds: int = 3, margin: float = 0.02) -> dict:
    """Return {"options": {...}, "ms": best, "default_ms": ..., "table": [...]}
    for the workload (T0: host float32 array, tidx: host uint8 array or
    None); options {} means the library default was kept.  dimensions:
    {name: (option dict, ...)} swept in order (DEFAULT_DIMENSIONS).  Every
    table row holds the dimension, the candidate's full options and its ms."""
    import torch

    dims = dimensions or DEFAULT_DIMENSIONS
    key = "%s|%s|%s|%d|%s" % (_arch(), mode, signature(targets, T0), len(T0), ",".join(dims))
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return cache[key]
    T0_d = torch.as_tensor(np.asarray(T0, dtype=np.float32), device="cuda")
    tidx_d = None if tidx is None else torch.as_tensor(np.asarray(tidx, dtype=np.uint8), device="cuda")
    table = []
    t0 = time.perf_counter()
    current = {}
    for name, cands in dims.items():
        best_ms, best_opts = None, current
        for c in cands:
            opts = dict(current, **c)
            ms = _time(targets, T0_d, tidx_d, opts, repeats, mode)
            table.append(dict(dimension=name, options=opts, ms=ms))
            if verbose:
                print("autotune", name, opts, "%.3f ms" % ms, flush=True)
            if best_ms is None or ms < best_ms:
                best_ms, best_opts = ms, opts
        current = best_opts
    # launch times vary by a few per cent: re-time the swept policy and the
    # library default in interleaved rounds; the policy replaces the default
    # only if it is faster by more than `margin`
    cand = dict(options=current)
    default = dict(options={})
    samples = {id(cand): [], id(default): []}
    for _ in range(rounds):
        for r in (cand, default):
            samples[id(r)].append(_time(targets, T0_d, tidx_d, r["options"], repeats, mode))
    for r in (cand, default):
        r["ms_final"] = float(np.median(samples[id(r)]))
        if verbose:
            print("autotune final", r["options"] or "library default", "%.3f ms" % r["ms_final"], flush=True)
    best = cand if cand["ms_final"] < default["ms_final"] * (1.0 - margin) else default
    result = {"options": best["options"], "ms": best["ms_final"], "default_ms": default["ms_final"],
              "swept_options": current, "swept_ms": cand["ms_final"],
              "events": int(len(T0)), "sweep_s": time.perf_counter() - t0, "table": table}
    if use_cache:
        cache[key] = result
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return result
