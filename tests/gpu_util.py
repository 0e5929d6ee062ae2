"""Helpers for the GPU tests: run the HIP library through its C ABI and
convert the output to the float64 Events form of ledger.py."""
from __future__ import annotations

import numpy as np

import ledger


def run_gpu(targets, T0, seed, tidx=None, mode="persistent", first_id=0, capacity=None, ctx=None,
            allow_overflow=False, history=False, **opts):
    """history: also return the per-event history words (uniforms drawn,
    flight segments) as h["history"] (n x 2)."""
    import torch
    import paper_1309_7963_amd as inc

    own = ctx is None
    if own:
        ctx = inc.Context(targets, **opts)
    T0_d = torch.as_tensor(np.asarray(T0, dtype=np.float32), device="cuda")
    ti_d = None if tidx is None else torch.as_tensor(np.asarray(tidx, dtype=np.uint8), device="cuda")
    out = None
    if history:
        n = len(T0)
        out = inc.DeviceOutput.allocate(n, ctx.default_capacity(n) if capacity is None else capacity, "cuda",
                                        history=True)
    out = ctx.simulate(T0_d, seed=seed, target_idx=ti_d, first_event_id=first_id, mode=mode, capacity=capacity,
                       out=out)
    torch.cuda.synchronize()
    if out.n_sec() > out.capacity and not allow_overflow:
        raise RuntimeError("secondary buffer too small: %d records for capacity %d" % (out.n_sec(), out.capacity))
    host = out.to_numpy()
    if own:
        ctx.close()
    return host


def sort_secondaries(h):
    """Order records by (event, stage) keeping emission order inside a stage
    is not possible after compaction; sort by (event, stage, species, T)."""
    key = np.lexsort((h["sec_T"], h["sec_species"], h["sec_stage"], h["sec_event"]))
    return {k: (v[key] if k.startswith("sec_") else v) for k, v in h.items()}


def events_from_gpu(h, targets, T0, tidx=None) -> ledger.Events:
    AZ = np.array(targets, dtype=np.int64).reshape(-1, 2)
    ti = np.zeros(len(T0), dtype=np.int64) if tidx is None else np.asarray(tidx, dtype=np.int64)
    r = h["res"]
    return ledger.Events(
        A=AZ[ti, 0], Z=AZ[ti, 1], T0=np.asarray(T0, dtype=np.float32).astype(np.float64),
        A_f=r["A_f"].astype(np.int64), Z_f=r["Z_f"].astype(np.int64),
        Ex_casc=r["Ex_casc"].astype(np.float64), Ex_f=r["Ex_f"].astype(np.float64),
        p_f=r["p_f"].astype(np.float64), n_sec=r["n_sec"].astype(np.int64), flags=r["flags"].astype(np.int64),
        sec_event=h["sec_event"].astype(np.int64), sec_species=h["sec_species"].astype(np.int64),
        sec_stage=h["sec_stage"].astype(np.int64), sec_T=h["sec_T"].astype(np.float64),
        sec_u=h["sec_u"].astype(np.float64),
    )


def outcome_keys(ev: ledger.Events):
    """Per-event integer outcome: (A_f, Z_f, sorted (stage, species) list)."""
    order = np.lexsort((ev.sec_species, ev.sec_stage, ev.sec_event))
    e = ev.sec_event[order]
    code = (ev.sec_stage[order] * 32 + ev.sec_species[order]).astype(np.int64)
    bounds = np.searchsorted(e, np.arange(ev.n + 1))
    keys = []
    for i in range(ev.n):
        keys.append((int(ev.A_f[i]), int(ev.Z_f[i]), tuple(code[bounds[i]:bounds[i + 1]].tolist())))
    return keys


def events_slice(ev: ledger.Events, start: int, stop: int) -> ledger.Events:
    """Events [start, stop) of a batch with their records, indices rebased to 0."""
    sel = (ev.sec_event >= start) & (ev.sec_event < stop)
    sl = slice(start, stop)
    return ledger.Events(
        A=ev.A[sl], Z=ev.Z[sl], T0=ev.T0[sl], A_f=ev.A_f[sl], Z_f=ev.Z_f[sl], Ex_casc=ev.Ex_casc[sl],
        Ex_f=ev.Ex_f[sl], p_f=ev.p_f[sl], n_sec=ev.n_sec[sl], flags=ev.flags[sl],
        sec_event=ev.sec_event[sel] - start, sec_species=ev.sec_species[sel], sec_stage=ev.sec_stage[sel],
        sec_T=ev.sec_T[sel], sec_u=ev.sec_u[sel],
    )
