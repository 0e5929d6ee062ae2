#!/usr/bin/env python3
"""Benchmark: non-elastic proton-nucleus events/s on one MI355X.

Default workload (one step): 10^6 events of 200 MeV p + 16O and 10^6 events of
200 MeV p + 40Ca, synthetic inputs already resident in HBM, generated in the
staged mode: the persistent cascade kernel, then the persistent evaporation
kernel, back to back on one stream.  The timed steps are consecutive batches
(each on new event ids) with three on the device at once, each with its own
context, buffers and stream (--inflight), so that a batch's start fills the
CUs its predecessor's end frees (a launch ends waiting for its slowest
events); `value` is the whole job's events over its wall time, and
`one_batch_at_a_time` the same steps run one after another.  Prints one JSON
line (see the keys below).  Extra keys report the single-target rates, the tissue mixture
(12C/14N/16O/31P/40Ca at 20-250 MeV) and the implant mixture (48Ti/56Fe at
70-250 MeV), the fused persistent kernel and the plain two-kernel path, the
divergence ceiling, the host-inclusive rate, the fast-math build, the nuclide
tally, the ring, serving latency, and the CPU oracle timed on this host's
cores on a bounded sample.

The roofline is the VALU (FP32 lane-operation) roofline: the path is ALU
bound, not HBM bound (output is ~0.1 GB per 10^6 events).  `achieved` is the
algorithmic lane-operation count of the method per launch (per-step costs in
STEP_COST below, times the oracle's per-event step counts on the same
workload, times the events per launch) over the launch's kernel time, one
batch at a time, measured with HIP events on the stream the kernels run on.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 FP32 lanes x 2.4 GHz = one VALU lane-operation per lane
# per clock (FMA counted as one operation, no packed math).
PEAK_LANE_OPS = 256 * 64 * 2.4e9
# Algorithmic lane-operations per step of the method, counted item by item
# from the oracle's formulas.  Each entry is (what, basic, transcendental,
# wide): basic = FP32 add/sub/mul/FMA/min/max/compare/select and 32-bit
# integer operations, weight 1; transcendental = exp, log, sqrt, reciprocal,
# sin, cos (a division is a reciprocal and a multiply), weight 4, the issue
# cost of a quarter-rate instruction; wide = cbrt or a sine-cosine pair,
# weight 8.  Counting rules: a quantity is counted once per event where it is
# first formed (the collision reuses T_x, T_t, Q, s, p* and p_lab of its
# tentative step); quantities that depend only on the target or on the
# nuclide (A, Z) -- masses, separation energies, Coulomb barriers, radii,
# Fermi energies and momenta, shell radii -- are set-up tables, not per-event
# work; sigma and its majorant are read from pre-calculated tables with
# linear interpolation in log p_lab, as the paper's implementation does
# (Sec. 3); an inversion counts the mean number of Newton steps it takes
# (4 residuals, 3 updates for the spectrum) rather than the oracle's
# bisection; counters that only serve diagnostics are not counted.
STEP_OPS = {
    "draw": [  # one uniform
        ("a quarter of a Philox4x32-10 block: 10 rounds x (2 mul_lo, 2 mul_hi, 4 xor), "
         "9 key bumps x 2 adds, counter bump", 99 / 4, 0, 0),
        ("24-bit mantissa to (0, 1): shift, convert, FMA; position in the block", 4, 0, 0),
    ],
    "tau": [  # optical depth of a new flight (the uniform is a draw)
        ("-ln u", 1, 1, 0),
    ],
    "segment": [  # every flight segment inside one shell
        ("lambda = rho_n sh_n + rho_p sh_p with the sea-occupancy checks", 6, 0, 0),
        ("x.d and b^2 = |x cross d|^2", 12, 0, 0),
        ("inner-sphere test: s > 0, x.d < 0, b^2 < r_in^2", 5, 0, 0),
        ("distance: r^2 - b^2, clamp, sqrt, -x.d -/+ root, clamp; destination shell", 5, 1, 0),
        ("optical-depth test tau < lambda t; segment guard", 4, 0, 0),
    ],
    "crossing": [  # a segment that ends on a shell boundary
        ("tau -= lambda t; x += t d", 4, 0, 0),
        ("normal n = x / |x|", 6, 2, 0),
        ("T on both sides of the step (E_F of both shells, or the binding energy), outer test", 4, 0, 0),
        ("|p| = sqrt(T^2 + 2 T m); p_n = |p| d.n", 6, 1, 0),
        ("dp^2 = (T' - T)(T' + T + 2m); p_n'^2 = p_n^2 + dp^2; both tests", 7, 0, 0),
        ("p_t = p - p_n n; p_n' = +/-sqrt(p_n'^2); q = p_t + p_n' n", 11, 1, 0),
        ("d' = q / |q|; shell index", 7, 2, 0),
    ],
    "tentative": [  # a segment that ends in a tentative collision
        ("x += (tau / lambda) d", 4, 1, 0),
        ("target species: u (w_n + w_p) against w_n; its m, p_F, E_F", 6, 0, 0),
        ("Fermi momentum: p_F u^(1/3), cos = 2u - 1, sin = sqrt(1 - cos^2), phi = 2 pi u, "
         "sine-cosine pair, vector", 10, 1, 2),
        ("T_x = eps + E_F; p_x = sqrt(T_x^2 + 2 T_x m_x) d; like pair", 7, 1, 0),
        ("T_t = p_t^2 / (sqrt(p_t^2 + m_y^2) + m_y)", 4, 2, 0),
        ("Q = 2 (T_x T_t + T_x m_y + T_t m_x - p_x.p_t); s = (m_x + m_y)^2 + Q", 9, 0, 0),
        ("p_lab = sqrt(Q (Q + 4 m_x m_y) / (4 s)) sqrt(s) / m_y", 6, 3, 0),
        ("sigma from its table: GeV/c, clamp, log coordinate, node, fraction, interpolation, "
         "like/unlike, mb to fm^2", 13, 1, 0),
        ("acceptance u < sigma / sh_y", 2, 1, 0),
    ],
    "kinematics": [  # an accepted or Pauli-blocked collision
        ("P = p_x + p_t; sqrt(s) and its reciprocal", 3, 2, 0),
        ("CM velocity u = P / sqrt(s); gamma = (T_x + T_t + m_x + m_y) / sqrt(s)", 7, 0, 0),
        ("direction of x in the CM: q = p_x + (u.p_x / (g + 1) - E_x) u, normalised", 16, 3, 0),
        ("slope b at p_lab (closed form; mean of like and unlike pairs), GeV/c, clamp", 10, 0.5, 0),
        ("k = 2 b (p*/1000)^2; y = -log1p(u expm1(-2k)) / k, small-k branch, clamp", 12, 3, 0),
        ("cos = 1 - y, sin = sqrt(y (2 - y))", 4, 1, 0),
        ("rotation by (theta, phi) about the CM direction: perpendicular frame, sine-cosine pair", 23, 2, 1),
        ("q* = p* n", 3, 0, 0),
        ("boosts of both products sharing 1/(g+1) and u.u/(g+1): E* = sqrt(p*^2 + m^2), u.q, "
         "p = q + (u.q/(g+1) + E*) u, T* = p*^2 / (E* + m), T = g T* + m u.u/(g+1) + u.q", 29, 4, 0),
        ("like pairs: which product is x", 9, 0, 0),
        ("Pauli test and outcome: T' <= E_F for both, hole depth, excess energies, cutoff tests", 11, 0, 0),
    ],
    "collision": [  # an accepted collision, after its kinematics
        ("the struck nucleon leaves the sea; lowest occupancy; hole depth to E*", 3, 0, 0),
        ("unit directions of both products", 12, 4, 0),
        ("cutoff captures; stack push or pop (position, direction, eps, species, shell)", 14, 0, 0),
    ],
    "majorant": [  # every new flight: entry, after a collision, after an escape
        ("T = eps + min E_F; p = sqrt(T^2 + 2 T m); E = T + m", 4, 1, 0),
        ("per target species: p_lab,min = (p E_F,y - E p_F,max) / m_y, clamp, GeV/c", 10, 0, 0),
        ("per target species: sigma-hat from its table, like/unlike, mb to fm^2", 26, 2, 0),
    ],
    "entry": [  # every cascade pass
        ("b = R sqrt(u), azimuth (sine-cosine pair), entry point on the sphere, eps = T0 + E_B", 8, 2, 1),
        ("inward normal n = x / |x|", 7, 2, 0),
        ("inward refraction at R (the crossing's refraction items)", 31, 4, 0),
    ],
    "escape": [  # a cascade particle that leaves the nucleus
        ("|p| = sqrt(T^2 + 2 T m) outside; recoil p_res -= |p| d; escape count", 6, 1, 0),
        ("next particle from the stack, or the end of the pass", 10, 0, 0),
    ],
    "evap_channels": [  # every evaporation step, including the last (nothing open)
        ("6 channels: daughter (A - a, Z - z) and its existence test", 6 * 7, 0, 0),
        ("6 channels: U = E - S - V, open test", 6 * 3, 0, 0),
        ("6 channels: Y = 2 sqrt(a U)", 6 * 2, 6 * 1, 0),
        ("6 channels: I = [e^Y (2Y^2 - 6Y + 6) + Y^2 - 6] / (8 a^2)", 6 * 6, 6 * 1, 0),
        ("6 channels: w = g m R^2 I; running total; any channel open", 6 * 2 + 1, 0, 0),
    ],
    "evap_emit": [  # every emission
        ("channel: u x total, cumulative scan over the channels", 22, 0, 0),
        ("K(1) of the spectrum (closed form) and the target mass", 12, 1, 0),
        ("4 residuals K(s) - target (closed form e^(-Ys) Q(Ys), Q cubic)", 4 * 12, 4 * 1, 0),
        ("3 Newton updates: density s (2 - s)(1 - s) e^(-Ys), step, bracket, stop tests", 3 * 13, 3 * 1, 0),
        ("x = U s (2 - s); E_d = U - x; eps = V + x; parent and daughter masses", 7, 0, 0),
        ("p^2 = eps (eps + 2m)(eps + 2M_d)(eps + 2M_d + 2m) / (4 M_p^2); p", 9, 2, 0),
        ("isotropic direction: cos = 2u - 1, sin, phi, sine-cosine pair, q = p n", 9, 1, 1),
        ("recoil velocity u = P / M_p, g = sqrt(1 + u.u), 1/(g+1), u.u/(g+1)", 8, 3, 0),
        ("boost of the fragment: E*, u.q, p, T*, T", 14, 2, 0),
        ("unit direction of the record; P -= p; A, Z, E", 12, 2, 0),
    ],
}
OP_WEIGHTS = (1, 4, 8)


def step_cost(items) -> float:
    """Weighted lane-operations of one step from its itemised counts."""
    return float(sum(b * OP_WEIGHTS[0] + t * OP_WEIGHTS[1] + w * OP_WEIGHTS[2] for _, b, t, w in items))


STEP_COST = {k: step_cost(v) for k, v in STEP_OPS.items()}


# kernels of one step per launch mode (timed together: they run back to back
# on one stream)
KERNELS = {"plain": "k_cascade_plain+k_evap_plain", "persistent": "k_persistent",
           "staged": "k_persistent+k_evap_persistent"}


# The sources the profiled event launch is compiled from (kernels, their
# headers, the setup and start-order kernels, the launch policy); the server
# and ring front ends are not part of it.
KERNEL_SOURCES = ("api.hip", "ctx.h", "device.h", "event.h", "kernels.h", "kernels.hip", "setup.hip")


def kernel_sources_hash() -> str:
    """sha256 (first 16 hex digits) over the code of the profiled launch's
    sources: comments removed and whitespace collapsed, so that only a code
    change voids a profile."""
    import hashlib
    import re

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1309_7963_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(csrc, f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(f.encode())
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def profiled_traffic(kernel: str, events: int):
    """HBM bytes per launch from a committed counter summary under profiles/
    (FETCH_SIZE and WRITE_SIZE scaled by the copy calibration), or None when
    no summary was taken on the current kernel sources and this workload."""
    d = os.path.join(ROOT, "profiles")
    if not os.path.isdir(d):
        return None
    want = kernel_sources_hash()
    for f in sorted(os.listdir(d)):
        if not f.endswith(".md"):
            continue
        with open(os.path.join(d, f)) as fh:
            for ln in fh:
                if not ln.startswith("traffic_json:"):
                    continue
                rec = json.loads(ln.split(":", 1)[1])
                if rec["kernel"] == kernel and rec["kernel_sources"] == want and rec["events"] == events:
                    return float(rec["traffic_bytes"])
    return None


def profiled_same_stream(kernel: str):
    """The divergence-free probe's VALU counters from a committed summary
    under profiles/ (`same_stream_json:` line): every lane of a launch
    replays one event, so VALU wave-instructions x 64 / events is the
    instructions one event's history takes with every lane active.  None
    when no summary was taken on the current kernel sources."""
    d = os.path.join(ROOT, "profiles")
    if not os.path.isdir(d):
        return None
    want = kernel_sources_hash()
    for f in sorted(os.listdir(d)):
        if not f.endswith(".md"):
            continue
        with open(os.path.join(d, f)) as fh:
            for ln in fh:
                if ln.startswith("same_stream_json:"):
                    rec = json.loads(ln.split(":", 1)[1])
                    if rec["kernel"] == kernel and rec["kernel_sources"] == want:
                        return rec
    return None


def step_counts(res) -> dict:
    """Per-step totals over the events of `res` (the oracle's per-event
    counters: draws, segments, tentative, accepted and Pauli-blocked
    collisions, retried passes, emissions and records).  Every pass starts
    with an entry, a majorant and an optical depth; each null or blocked
    tentative collision draws a new optical depth; each accepted collision and
    each escape starts a new flight (majorant and optical depth) except the
    one that ends its event (an event the segment guard ends has none); a
    retried (transparent) pass records nothing."""
    n = len(res)
    tent = int(res["n_tent"].sum())
    coll = int(res["n_coll"].sum())
    evap = int(res["n_evap"].sum())
    passes = n + int(res["n_retry"].sum())
    escapes = int(res["n_sec"].sum()) - evap
    ended = n - int(np.count_nonzero(res["flags"] & 2))  # events ended by a collision or an escape
    return {"draw": int(res["n_draw"].sum()), "tau": passes + tent + escapes - ended,
            "segment": int(res["n_seg"].sum()), "crossing": int(res["n_seg"].sum()) - tent,
            "tentative": tent, "kinematics": coll + int(res["n_pauli"].sum()), "collision": coll,
            "majorant": passes + coll + escapes - ended, "entry": passes, "escape": escapes,
            "evap_channels": evap + n, "evap_emit": evap}


def algorithmic_ops_per_event(res) -> float:
    """Mean lane-operations per event: the step totals times STEP_COST."""
    c = step_counts(res)
    return sum(c[k] * STEP_COST[k] for k in STEP_COST) / len(res)


def _workloads(n_events: int):
    rng = np.random.default_rng(20130930)
    out = {}
    half = n_events // 2
    out["o16_ca40_200"] = dict(
        label="200 MeV p+16O and p+40Ca, %d events each" % half,
        targets=[(16, 8), (40, 20)],
        tidx=np.concatenate([np.zeros(half, np.uint8), np.ones(n_events - half, np.uint8)]),
        T0=np.full(n_events, 200.0, np.float32), T_max=200.0)
    out["o16_200"] = dict(label="200 MeV p+16O", targets=[(16, 8)], tidx=None,
                          T0=np.full(half, 200.0, np.float32), T_max=200.0)
    out["ca40_200"] = dict(label="200 MeV p+40Ca", targets=[(40, 20)], tidx=None,
                           T0=np.full(half, 200.0, np.float32), T_max=200.0)
    tissue = [(12, 6), (14, 7), (16, 8), (31, 15), (40, 20)]
    out["tissue_mix"] = dict(
        label="tissue mixture 12C/14N/16O/31P/40Ca (.18/.03/.65/.01/.13), T0 ~ U(20,250) MeV",
        targets=tissue,
        tidx=rng.choice(5, size=half, p=[0.18, 0.03, 0.65, 0.01, 0.13]).astype(np.uint8),
        T0=rng.uniform(20, 250, half).astype(np.float32), T_max=250.0)
    out["implant_mix"] = dict(
        label="implant mixture 48Ti/56Fe 50/50, T0 ~ U(70,250) MeV", targets=[(48, 22), (56, 26)],
        tidx=rng.choice(2, size=half).astype(np.uint8),
        T0=rng.uniform(70, 250, half).astype(np.float32), T_max=250.0)
    return out


def _time_gpu(w, mode, steps, warmup, seed=1, inflight=1, **ctx_opts):
    """Time `steps` batches of workload w (after `warmup` untimed ones, at
    least one per in-flight context), each on new event ids.  inflight = 1: one batch at a time on torch's current
    stream, launch_ms = each launch's duration (HIP events on that stream).
    inflight = k > 1: batch i goes to context, output buffers and stream
    i mod k (default priority), so up to k batches are on the device at once
    and a batch's start fills the CUs its predecessor's end frees; launch_ms
    then spans each launch's wait for the device as well."""
    import torch

    import paper_1309_7963_amd as inc

    ctxs = [inc.Context(w["targets"], **ctx_opts) for _ in range(inflight)]
    T0 = torch.as_tensor(w["T0"], device="cuda")
    tidx = None if w["tidx"] is None else torch.as_tensor(w["tidx"], device="cuda")
    n = int(T0.shape[0])
    outs = [inc.DeviceOutput.allocate(n, ctxs[0].default_capacity(n)) for _ in range(inflight)]
    streams = [torch.cuda.current_stream()] if inflight == 1 else [torch.cuda.Stream() for _ in range(inflight)]
    # with several batches in flight every context gets at least one untimed
    # launch, which allocates its start-order and hand-over buffers outside
    # the timed steps
    n_warm = warmup if inflight == 1 else max(warmup, inflight)
    for k in range(n_warm):
        i = k % inflight
        ctxs[i].simulate(T0, seed=seed, target_idx=tidx, mode=mode, out=outs[i], first_event_id=k * n,
                         stream=streams[i])
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        i = k % inflight
        starts[k].record(streams[i])
        ctxs[i].simulate(T0, seed=seed, target_idx=tidx, mode=mode, out=outs[i], first_event_id=(n_warm + k) * n,
                         stream=streams[i])
        ends[k].record(streams[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    last = outs[(steps - 1) % inflight]
    n_sec = last.n_sec()
    flagged = sum(o.n_flagged() for o in outs)
    for c in ctxs:
        c.close()
    return dict(n=n, wall_s=wall, launch_ms=launch_ms, n_sec=n_sec, flagged=flagged,
                out_bytes=n * 32 + n_sec * 22)


def _end_to_end(w, steps: int, seed: int = 1):
    """Host-inclusive rate: inputs start in pinned host memory, results end in
    pinned host memory (H2D, kernel, the secondary count, D2H of the residuals
    and of the records actually written), one batch after another."""
    import torch

    import paper_1309_7963_amd as inc

    ctx = inc.Context(w["targets"])
    n = len(w["T0"])
    T0_h = torch.from_numpy(w["T0"]).pin_memory()
    ti_h = torch.from_numpy(w["tidx"]).pin_memory()
    T0_d = torch.empty_like(T0_h, device="cuda")
    ti_d = torch.empty_like(ti_h, device="cuda")
    out = inc.DeviceOutput.allocate(n, ctx.default_capacity(n))
    names = ("sec_event", "sec_species", "sec_stage", "sec_T", "sec_ux", "sec_uy", "sec_uz")
    res_h = torch.empty(out.res.shape, dtype=out.res.dtype).pin_memory()
    sec_h = {k: torch.empty(getattr(out, k).shape, dtype=getattr(out, k).dtype).pin_memory() for k in names}
    cnt_h = torch.empty(4, dtype=torch.int64).pin_memory()

    def one(k):
        T0_d.copy_(T0_h, non_blocking=True)
        ti_d.copy_(ti_h, non_blocking=True)
        ctx.simulate(T0_d, seed=seed, target_idx=ti_d, out=out, first_event_id=k * n)
        cnt_h.copy_(out.counters, non_blocking=True)
        res_h.copy_(out.res, non_blocking=True)
        torch.cuda.current_stream().synchronize()
        m = min(int(cnt_h[0]), out.capacity)
        for name in names:
            sec_h[name][:m].copy_(getattr(out, name)[:m], non_blocking=True)
        torch.cuda.current_stream().synchronize()
        return m

    one(0)
    t0 = time.perf_counter()
    for k in range(steps):
        m = one(k + 1)
    dt = (time.perf_counter() - t0) / steps
    ctx.close()
    return dict(events_per_s=n / dt, ms_per_batch=dt * 1000.0, bytes_h2d=n * 5, bytes_d2h=n * 32 + m * 22,
                note="pinned host inputs -> device -> pinned host residuals and secondaries, serial")


def _end_to_end_pipelined(w, steps: int, seed: int = 1):
    """Host-inclusive rate with the copies overlapped: each batch's inputs go
    up and its results come down on a copy stream while the next batch runs
    on the compute stream (two sets of device and pinned host buffers used in
    turn).  The host learns a batch's secondary count from a pinned counter
    copy queued behind its kernel, then queues exactly those records."""
    import torch

    import paper_1309_7963_amd as inc

    ctx = inc.Context(w["targets"])
    n = len(w["T0"])
    comp = torch.cuda.current_stream()
    copy = torch.cuda.Stream()
    T0_h = torch.from_numpy(w["T0"]).pin_memory()
    ti_h = torch.from_numpy(w["tidx"]).pin_memory()
    names = ("sec_event", "sec_species", "sec_stage", "sec_T", "sec_ux", "sec_uy", "sec_uz")
    sets = []
    for _ in range(2):
        out = inc.DeviceOutput.allocate(n, ctx.default_capacity(n))
        sets.append(dict(
            T0=torch.empty_like(T0_h, device="cuda"), ti=torch.empty_like(ti_h, device="cuda"), out=out,
            res=torch.empty(out.res.shape, dtype=out.res.dtype).pin_memory(),
            sec={k: torch.empty(getattr(out, k).shape, dtype=getattr(out, k).dtype).pin_memory() for k in names},
            cnt=torch.empty(4, dtype=torch.int64).pin_memory(), done=torch.cuda.Event(), m=0))

    def launch(k):
        # inputs up on the copy stream, behind the results of the batch that
        # used this buffer set before (stream order), then the kernel
        b = sets[k % 2]
        with torch.cuda.stream(copy):
            b["T0"].copy_(T0_h, non_blocking=True)
            b["ti"].copy_(ti_h, non_blocking=True)
        up = torch.cuda.Event()
        up.record(copy)
        comp.wait_event(up)
        ctx.simulate(b["T0"], seed=seed, target_idx=b["ti"], out=b["out"], first_event_id=k * n, stream=comp)
        b["cnt"].copy_(b["out"].counters, non_blocking=True)
        b["done"].record(comp)

    def drain(k):
        b = sets[k % 2]
        b["done"].synchronize()
        m = min(int(b["cnt"][0]), b["out"].capacity)
        copy.wait_event(b["done"])
        with torch.cuda.stream(copy):
            b["res"].copy_(b["out"].res, non_blocking=True)
            for name in names:
                b["sec"][name][:m].copy_(getattr(b["out"], name)[:m], non_blocking=True)
        b["m"] = m

    launch(0)
    drain(0)
    copy.synchronize()
    t0 = time.perf_counter()
    launch(1)
    for k in range(1, steps + 1):
        if k < steps:
            launch(k + 1)
        drain(k)
    copy.synchronize()
    dt = (time.perf_counter() - t0) / steps
    m = sets[steps % 2]["m"]
    ctx.close()
    return dict(events_per_s=n / dt, ms_per_batch=dt * 1000.0, bytes_h2d=n * 5, bytes_d2h=n * 32 + m * 22,
                note="pinned host inputs -> device -> pinned host residuals and secondaries, "
                     "copies of one batch overlapping the next batch's kernels")


def _reaction_cross_sections(n: int = 1_000_000, T: float = 200.0, seed: int = 3):
    """Diagnostic of the transparent-pass reading (Sec. 2.1): sigma_R = pi R^2 x
    events / (events + transparent passes), from the retries every residual
    records, per target at one energy (mb; no measured value is compared)."""
    import torch

    import paper_1309_7963_amd as inc

    out = {}
    for name, AZ in (("12C", (12, 6)), ("16O", (16, 8)), ("40Ca", (40, 20)), ("56Fe", (56, 26))):
        ctx = inc.Context([AZ])
        R = float(ctx.tables()[0, 107])
        d = ctx.simulate(torch.full((n,), T, device="cuda"), seed=seed)
        retries = int((d.res.view(torch.int16).view(n, 16)[:, 15].to(torch.int64) & 0xFFFF).sum())
        ctx.close()
        out[name] = dict(sigma_R_mb=math.pi * R * R * 10.0 * n / (n + retries), transparent_per_event=retries / n)
    return dict(T0_MeV=T, events=n, **out)


def _evaporation_stage(w, reps: int = 5, seed: int = 1):
    """The two stages apart, the paper's run-time split: cascade-only launches
    (no_evaporation) of the workload, whose first supplies (A', Z', E*, p) per
    event, and the evaporation stage alone (inc_evaporate_dev) on those
    post-cascade nuclei, each timed over `reps` launches."""
    import torch

    import paper_1309_7963_amd as inc

    casc = inc.Context(w["targets"], no_evaporation=1)
    T0 = torch.as_tensor(w["T0"], device="cuda")
    tidx = None if w["tidx"] is None else torch.as_tensor(w["tidx"], device="cuda")
    n = int(T0.shape[0])
    stream = torch.cuda.current_stream()
    first = casc.simulate(T0, seed=seed, target_idx=tidx)
    # the cascade stage alone, timed on its own outputs' buffers (later ids)
    scratch = inc.DeviceOutput.allocate(n, casc.default_capacity(n))
    casc_ms = []
    for k in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        casc.simulate(T0, seed=seed, target_idx=tidx, out=scratch, first_event_id=(k + 1) * n)
        b.record(stream)
        b.synchronize()
        casc_ms.append(a.elapsed_time(b))
    del scratch
    torch.cuda.synchronize()
    casc.close()
    r16 = first.res.view(torch.int16).view(n, 16)
    r32 = first.res.view(torch.float32).view(n, 8)
    A, Z = r16[:, 0].contiguous(), r16[:, 1].contiguous()
    Ex, P = r32[:, 3].contiguous(), r32[:, 4:7].contiguous()
    del first
    ctx = inc.Context(w["targets"])
    out = inc.DeviceOutput.allocate(n, ctx.default_capacity(n))
    ctx.evaporate(A, Z, Ex, seed=seed, P=P, out=out)
    ms = []
    for k in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        ctx.evaporate(A, Z, Ex, seed=seed, P=P, out=out, first_event_id=(k + 1) * n)
        b.record(stream)
        b.synchronize()
        ms.append(a.elapsed_time(b))
    mean_steps = out.n_sec() / n
    flagged = out.n_flagged()
    ctx.close()
    med = float(np.median(ms))
    return dict(nuclei=n, ms=med, nuclei_per_s=n / (med / 1000.0), fragments_per_nucleus=mean_steps,
                not_evaporated=flagged, cascade_only_ms=float(np.median(casc_ms)))


def _tally_run(w, n_ebins: int = 23, reps: int = 5):
    """Residual-nuclide tally of one generated batch (positron-emitter
    yields per energy bin): kernel time and the main emitters' yields."""
    import torch

    import paper_1309_7963_amd as inc

    ctx = inc.Context(w["targets"])
    T0 = torch.as_tensor(w["T0"], device="cuda")
    tidx = torch.as_tensor(w["tidx"], device="cuda")
    out = ctx.simulate(T0, seed=1, target_idx=tidx)
    table = ctx.tally(T0, out, target_idx=tidx, n_ebins=n_ebins)
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        ctx.tally(T0, out, target_idx=tidx, n_ebins=n_ebins, table=table)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    n = len(w["T0"])
    once = table.cpu().numpy() // (reps + 1)
    y = inc.positron_yields(once, w["targets"])
    per_1e6 = {"%d-%d" % t: {k: round(float(v.sum()) * 1e6 / n, 1) for k, v in d.items()} for t, d in y.items()}
    ctx.close()
    return dict(events_per_s=n / (ms / 1000.0), kernel_ms=ms, n_ebins=n_ebins, yields_per_1e6_events=per_1e6)


def _vertex_run(w, steps: int = 3, windows=(16, 18, 20), plain_launches: bool = True):
    """The event-based vertex pipeline (mode vertex: in-flight window in
    device memory, one kernel per vertex type over compacted queues) on
    workload w, one batch at a time, against the staged kernels: mean ms per
    batch (HIP events on the stream) for in-flight windows of 2^16, 2^18 and
    2^20 events."""
    staged = _time_gpu(w, "staged", steps, 1)
    out = {"staged_ms": float(np.mean(staged["launch_ms"])), "vertex_ms": {}, "vertex_ms_plain_launches": {}}
    for log2w in windows:
        e = _time_gpu(w, "vertex", steps, 1, vertex_window=1 << log2w)
        out["vertex_ms"]["2^%d" % log2w] = float(np.mean(e["launch_ms"]))
        if plain_launches:
            e = _time_gpu(w, "vertex", steps, 1, vertex_window=1 << log2w, vertex_launch=1)
            out["vertex_ms_plain_launches"]["2^%d" % log2w] = float(np.mean(e["launch_ms"]))
    best = min(out["vertex_ms"].values())
    out["vertex_over_staged"] = best / out["staged_ms"]
    return out


def _ring_run(w, slots: int, reps: int = 2, placement: str = "host", chunk: int = 1 << 16):
    """Implant mixture with the secondaries streamed through a bounded ring
    (in host memory, or in device memory drained by asynchronous chunk
    copies) while the kernel runs, drained into reused host arrays (timed:
    the call, residuals copied back included)."""
    import torch

    import paper_1309_7963_amd as inc

    ctx = inc.Context(w["targets"])
    ring = inc.Ring(ctx, slots=slots, placement=placement, chunk=chunk)
    T0 = torch.as_tensor(w["T0"], device="cuda")
    tidx = torch.as_tensor(w["tidx"], device="cuda")
    buf = inc.Ring.host_buffers(ctx.default_capacity(len(w["T0"])), len(w["T0"]))  # reused host arrays
    ring.simulate(T0, seed=1, target_idx=tidx, out=buf)  # warm-up
    best = None
    for k in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = ring.simulate(T0, seed=1, target_idx=tidx, first_event_id=(k + 1) << 32, out=buf)
        dt = time.perf_counter() - t
        if best is None or dt < best[0]:
            best = (dt, r)
    dt, r = best
    out = {"label": w["label"] + ", secondaries through a %d-record ring in %s memory" % (slots, placement),
           "placement": placement, "chunk": chunk if placement == "device" else None, "events": len(w["T0"]),
           "events_per_s": len(w["T0"]) / dt, "records": r["stats"]["records"], "wraps": r["stats"]["wraps"],
           "rc": r["rc"]}
    ring.close()
    ctx.close()
    return out


TISSUE = [(12, 6), (14, 7), (16, 8), (31, 15), (40, 20)]
TISSUE_W = [0.18, 0.03, 0.65, 0.01, 0.13]


def _serving_requests(n_req: int, seed: int):
    """Requests of floor(10^U(3,5)) events, tissue targets, energies 85 %
    U(150, 250) and 15 % U(20, 150) MeV (a Bragg-curve-like spectrum)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(n_req):
        n = int(10 ** rng.uniform(3, 5))
        hi = rng.random(n) < 0.85
        reqs.append(dict(
            T0=np.where(hi, rng.uniform(150, 250, n), rng.uniform(20, 150, n)).astype(np.float32),
            target_idx=rng.choice(5, size=n, p=TISSUE_W).astype(np.uint8), seed=7, first_event_id=r << 32))
    return reqs


def _serving(n_req: int, loads, budget: int, slots: int):
    import paper_1309_7963_amd as inc

    ctx = inc.Context(TISSUE)
    srv = inc.Server(ctx, hbm_budget=budget, max_slots=slots)
    # saturated throughput: every request arrives at once
    sat_reqs = _serving_requests(max(n_req // 4, 50), seed=100)
    srv.replay(np.zeros(len(sat_reqs)), sat_reqs)
    sat = srv.stats()["events_per_s"]
    out = {"requests_per_load": n_req, "hbm_budget_bytes": budget, "slots": slots,
           "saturated_events_per_s": sat, "loads": []}
    for k, f in enumerate(loads):
        reqs = _serving_requests(n_req, seed=200 + k)
        mean_n = float(np.mean([len(q["T0"]) for q in reqs]))
        lam = f * sat / mean_n
        arrivals = np.cumsum(np.random.default_rng(300 + k).exponential(1.0 / lam, n_req))
        arrivals -= arrivals[0]
        srv.stats_reset()
        srv.replay(arrivals, reqs)
        st = srv.stats()  # the server's own latency statistics over this load's requests
        out["loads"].append({"load": f, "arrival_rate_per_s": lam, "mean_events_per_request": mean_n,
                             "p50_ms": st["latency_p50_s"] * 1e3, "p99_ms": st["latency_p99_s"] * 1e3,
                             "events_per_s": st["events_per_s"], "launches": st["launches"]})
        print("bench: serving load %.1f done" % f, file=sys.stderr, flush=True)
    srv.close()
    ctx.close()
    return out


def _host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_baseline(w, n_sample: int, threads: int):
    import oracle

    T0 = w["T0"].astype(np.float64)
    idx = np.linspace(0, len(T0) - 1, n_sample).astype(np.int64)
    tidx = None if w["tidx"] is None else w["tidx"][idx]
    t = time.perf_counter()
    out = oracle.run(w["targets"], T0[idx], seed=2, tidx=tidx, n_threads=threads)
    dt = time.perf_counter() - t
    return out, dt


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--events", type=int, default=2_000_000, help="events per step (split O/Ca)")
    ap.add_argument("--mode", default="staged", choices=["staged", "persistent", "plain"])
    ap.add_argument("--inflight", type=int, default=3,
                    help="batches on the device at once in the timed steps (each with its own context, "
                         "buffers and stream); the roofline's kernel time is always one batch at a time")
    ap.add_argument("--cpu-sample", type=int, default=1_000_000)
    ap.add_argument("--no-extra", action="store_true", help="skip the per-target and mixture rates")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--serving-requests", type=int, default=1000, help="requests per load point (0: skip)")
    ap.add_argument("--stage-split", action="store_true",
                    help="only time the cascade and evaporation stages apart on the main workload "
                         "(one JSON line; for profiling the evaporation-only launch)")
    ap.add_argument("--same-stream", action="store_true",
                    help="only run the divergence-free probe: --steps launches of the 200 MeV p+16O batch, "
                         "launch k with every lane replaying event id k x batch size (seed 1), one at a "
                         "time (one JSON line; for the VALU instruction counters)")
    ap.add_argument("--vertex", action="store_true",
                    help="only time the vertex pipeline (mode vertex, three window sizes) against the staged "
                         "kernels on the main workload (one JSON line)")
    ap.add_argument("--vertex-window", type=int, default=0,
                    help="with --vertex: only this in-flight window (log2), graph replay only")
    ap.add_argument("--rings", action="store_true",
                    help="only time the implant mixture directly and through the host and device rings "
                         "(one JSON line)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 256 MiB device to device (a plain copy kernel of known size, "
                         "to scale the HBM byte counters)")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this path runs on one GPU; the event stream shards by event id across GPUs "
              "but only --gpus 1 is measured here", file=sys.stderr)
        return 2

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    wl = _workloads(args.events)
    main_w = wl["o16_ca40_200"]
    if args.stage_split:
        print(json.dumps(dict(workload=main_w["label"], **_evaporation_stage(main_w, reps=args.steps))))
        return 0
    if args.vertex:
        kw = dict(windows=(args.vertex_window,), plain_launches=False) if args.vertex_window else {}
        print(json.dumps(dict(workload=main_w["label"], **_vertex_run(main_w, args.steps, **kw))))
        return 0
    if args.rings:
        w = wl["implant_mix"]
        e = _time_gpu(w, args.mode, 5, 1)
        rate = e["n"] / (float(np.median(e["launch_ms"])) / 1000.0)
        rings = {}
        for placement, slots, chunk in (("host", 1 << 20, 1 << 16), ("device", 1 << 20, 1 << 16),
                                        ("device", 1 << 20, 1 << 18), ("device", 1 << 22, 1 << 16),
                                        ("device", 1 << 22, 1 << 18)):
            rings["%s_%d_%d" % (placement, slots, chunk)] = _ring_run(w, slots, reps=3, placement=placement,
                                                                      chunk=chunk)
        print(json.dumps(dict(workload=w["label"], direct_events_per_s=rate, rings=rings)))
        return 0
    if args.same_stream:
        w = wl["o16_200"]
        e = _time_gpu(w, args.mode, args.steps, 0, same_stream=1)  # no warm-up: launch k replays id k n
        print(json.dumps(dict(same_stream=True, workload=w["label"], kernel=KERNELS[args.mode],
                              events_per_launch=e["n"], first_ids=[k * e["n"] for k in range(args.steps)],
                              launch_ms=e["launch_ms"])))
        return 0
    # whole-job throughput: the K batches with args.inflight of them on the
    # device at once (one context, buffer set and stream each)
    r = _time_gpu(main_w, args.mode, args.steps, args.warmup, inflight=args.inflight)
    ms_wall = r["wall_s"] * 1000.0 / args.steps
    value = r["n"] / (ms_wall / 1000.0)
    # one batch at a time: the kernels' own launch duration (roofline, profile)
    r1 = r if args.inflight == 1 else _time_gpu(main_w, args.mode, args.steps, args.warmup)
    ms = float(np.mean(r1["launch_ms"]))
    print("bench: main workload done (%.2f ms/batch, %.2f ms per launch one at a time)" % (ms_wall, ms),
          file=sys.stderr, flush=True)

    extra = {}
    if not args.no_extra:
        from paper_1309_7963_amd import autotune

        rate = lambda e: e["n"] / (float(np.median(e["launch_ms"])) / 1000.0)

        def tuner_table(tuned):
            # each swept candidate: its dimension, the options it set, ms per launch
            return [[r["dimension"], r["options"], round(r["ms"], 3)] for r in tuned["table"]]

        for key in ("o16_200", "ca40_200", "tissue_mix", "implant_mix"):
            e = _time_gpu(wl[key], args.mode, 5, 1)
            extra[key] = dict(label=wl[key]["label"], events=e["n"], events_per_s=rate(e))
            if key in ("tissue_mix", "implant_mix"):
                # autotuned launch policy (swept on the same batch)
                w = wl[key]
                tuned = autotune.tune(w["targets"], w["T0"], w["tidx"], use_cache=False)
                e = _time_gpu(w, args.mode, 5, 1, **tuned["options"])
                p = _time_gpu(w, "plain", 3, 1)
                extra[key].update(tuned_options=tuned["options"] or "library default", tuned_events_per_s=rate(e),
                                  plain_events_per_s=rate(p), autotune_sweep_s=tuned["sweep_s"],
                                  autotune=dict(swept_options=tuned["swept_options"], swept_ms=tuned["swept_ms"],
                                                default_ms=tuned["default_ms"], table=tuner_table(tuned)))
            print("bench: %s done" % key, file=sys.stderr, flush=True)
        # the tuner on the main workload itself
        tuned = autotune.tune(main_w["targets"], main_w["T0"], main_w["tidx"], use_cache=False)
        extra["main_autotune"] = dict(options=tuned["options"] or "library default", ms=tuned["ms"],
                                      default_ms=tuned["default_ms"], swept_options=tuned["swept_options"],
                                      swept_ms=tuned["swept_ms"], table=tuner_table(tuned))
        print("bench: main-workload autotune done", file=sys.stderr, flush=True)
        e = _time_gpu(main_w, "plain", 3, 1)
        extra["plain_two_kernel"] = dict(events_per_s=rate(e))
        extra["vertex_pipeline"] = _vertex_run(main_w, 2)
        e = _time_gpu(main_w, "persistent", 3, 1)
        extra["fused_persistent"] = dict(events_per_s=rate(e))
        # divergence ceiling: every lane on the same event stream (one history)
        dc = {}
        for mode in ("plain", args.mode):
            base = _time_gpu(wl["o16_200"], mode, 3, 1)
            same = _time_gpu(wl["o16_200"], mode, 3, 1, same_stream=1)
            dc[mode] = dict(events_per_s=rate(base), same_stream_events_per_s=rate(same),
                            ratio=rate(same) / rate(base))
        extra["divergence_ceiling"] = dict(workload=wl["o16_200"]["label"], **dc)
        extra["end_to_end_host"] = _end_to_end(main_w, 3)
        extra["end_to_end_host_pipelined"] = _end_to_end_pipelined(main_w, 5)
        extra["nuclide_tally"] = dict(workload=wl["tissue_mix"]["label"], **_tally_run(wl["tissue_mix"]))
        extra["evaporation_stage"] = dict(workload=main_w["label"], **_evaporation_stage(main_w))
        extra["reaction_cross_section"] = _reaction_cross_sections()
        # fast-math build of the event kernels (same workloads)
        fm = {}
        for key, w in (("o16_ca40_200", main_w), ("o16_200", wl["o16_200"]), ("ca40_200", wl["ca40_200"]),
                       ("tissue_mix", wl["tissue_mix"])):
            fm[key] = rate(_time_gpu(w, args.mode, 3, 1, fast_math=1))
        extra["fast_math"] = dict(events_per_s=fm, speedup_main=fm["o16_ca40_200"] / (r["n"] / (ms / 1000.0)))
        print("bench: divergence ceiling and end-to-end done", file=sys.stderr, flush=True)
        extra["implant_ring"] = _ring_run(wl["implant_mix"], slots=1 << 20, placement="device")
        extra["implant_ring_host"] = _ring_run(wl["implant_mix"], slots=1 << 20, placement="host")
        print("bench: implant rings done", file=sys.stderr, flush=True)

    serving = None
    if args.serving_requests > 0 and not args.no_extra:
        serving = _serving(args.serving_requests, (0.3, 0.6, 0.9), 2 << 30, 4)

    # oracle on a bounded sample of the same workload: work counts for the
    # roofline and the CPU baseline
    threads = min(os.cpu_count() or 1, 16)
    cpu = None
    ops_per_event = None
    if not args.no_cpu:
        out, dt = _cpu_baseline(main_w, args.cpu_sample, threads)
        print("bench: cpu baseline done (%.1f s)" % dt, file=sys.stderr, flush=True)
        ops_per_event = algorithmic_ops_per_event(out.results)
        n1 = max(args.cpu_sample // 10, 1000)
        _, dt1 = _cpu_baseline(main_w, n1, 1)
        cpu = {"value": args.cpu_sample / dt, "unit": "events/s", "cores": threads, "kind": "oracle",
               "sample": "%d events evenly spaced over the same 16O/40Ca 200 MeV batch, C++ float64 oracle, "
                         "%d threads, %.1f s" % (args.cpu_sample, threads, dt),
               "per_core": args.cpu_sample / dt / threads, "one_thread": n1 / dt1, "one_thread_sample": n1,
               "host_cpus": os.cpu_count(), "host_cpu_model": _host_cpu()}
    same = None
    rec = profiled_same_stream(KERNELS[args.mode])
    if rec is not None and not args.no_cpu:
        import oracle

        per = []
        for fid, valu in zip(rec["first_ids"], rec["valu_per_event"]):
            o = oracle.run([(16, 8)], np.array([200.0]), seed=1, first_id=fid)
            per.append([fid, valu, algorithmic_ops_per_event(o.results)])
        same = {"workload": rec["workload"] + ", every lane of a launch replays one event",
                "valu_instructions_per_event": float(np.mean([p[1] for p in per])),
                "algorithmic_ops_per_event": float(np.mean([p[2] for p in per])),
                "valu_utilization": rec["valu_utilization"], "per_event": per}
        same["ratio"] = same["valu_instructions_per_event"] / same["algorithmic_ops_per_event"]
    roof = None
    if ops_per_event is not None:
        achieved = ops_per_event * r["n"] / (ms / 1000.0)
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                "unit": "T lane-ops/s (FP32 VALU)", "frac": achieved / PEAK_LANE_OPS,
                "traffic": profiled_traffic(KERNELS[args.mode], r["n"]),
                "ops_per_event": ops_per_event, "same_stream": same, "kernel": KERNELS[args.mode],
                "kernel_ms": ms,
                "hbm_write_GBps": r["out_bytes"] / (ms / 1000.0) / 1e9}

    line = {
        "metric": "non-elastic events/sec, 200 MeV p+16O and mixed targets, 1 MI355X; p99 latency",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": main_w["label"], "events_per_step": r["n"], "mode": args.mode,
                   "targets": main_w["targets"], "batches_in_flight": args.inflight},
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernel_ms_per_step": ms,
        "one_batch_at_a_time": {"ms_per_step": r1["wall_s"] * 1000.0 / args.steps,
                                "events_per_s": r1["n"] / r1["wall_s"] * args.steps},
        "secondaries_per_step": r["n_sec"],
        "flagged_events": r["flagged"],
        "extra": extra,
        "p99_latency_ms": serving["loads"][1]["p99_ms"] if serving else None,
        "serving": serving,
        "paper_context": "GTX680, FP32, incl. host work: 310k events/s p+16O, 167k events/s p+40Ca at 200 MeV",
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
