"""The staged kernel's drain-time merge (option merge_lanes): once no event is
left to start, a wave with few live cascades hands them to waves of its
workgroup with free lanes.  Every event still follows its own random stream
through the same steps, so the merge changes the schedule and not the
results: identical residual records and the same secondary records with the
merge at its default, at its most eager (64) and off (-1), in fused mode,
through the ring, with the test hooks and with the evaporation options; and
the diagnostic count shows that events did move."""
import numpy as np
import pytest

from gpu_util import run_gpu

pytestmark = pytest.mark.gpu

TISSUE = [(12, 6), (14, 7), (16, 8), (31, 15), (40, 20)]
MAIN = [(16, 8), (40, 20)]


def _batch(n, seed):
    rng = np.random.default_rng(seed)
    tidx = rng.choice(5, size=n, p=[0.18, 0.03, 0.65, 0.01, 0.13]).astype(np.uint8)
    T0 = rng.uniform(20, 250, n).astype(np.float32)
    T0[::997] = 10.0   # below the model's range: written out flagged
    T0[5::1009] = 400.0
    return tidx, T0


def _same_records(a, b):
    assert a["res"].tobytes() == b["res"].tobytes()
    assert a["n_sec_total"] == b["n_sec_total"]
    ka = np.lexsort((a["sec_T"], a["sec_species"], a["sec_stage"], a["sec_event"]))
    kb = np.lexsort((b["sec_T"], b["sec_species"], b["sec_stage"], b["sec_event"]))
    for f in ("sec_event", "sec_species", "sec_stage", "sec_T", "sec_u"):
        assert np.array_equal(a[f][ka], b[f][kb]), f


def _staged(targets, T0, tidx, seed, **opts):
    import paper_1309_7963_amd as inc

    ctx = inc.Context(targets, **opts)
    try:
        h = run_gpu(targets, T0, seed=seed, tidx=tidx, mode="staged", ctx=ctx)
        moved = ctx.moved_events()
    finally:
        ctx.close()
    return h, moved


def test_merge_changes_schedule_not_results():
    n = 200000
    tidx, T0 = _batch(n, 11)
    off, m_off = _staged(TISSUE, T0, tidx, 3, merge_lanes=-1)
    assert m_off == 0
    fused = run_gpu(TISSUE, T0, seed=3, tidx=tidx, mode="persistent")
    _same_records(off, fused)
    for lanes in (0, 64, 1):
        got, moved = _staged(TISSUE, T0, tidx, 3, merge_lanes=lanes)
        print("merge_lanes", lanes, "moved events", moved)
        _same_records(off, got)
        if lanes != 1:
            assert moved > 0


def test_merge_on_the_benchmark_batch():
    # 10^6 p+16O and 10^6 p+40Ca at 200 MeV, one staged launch
    n = 2_000_000
    tidx = np.concatenate([np.zeros(n // 2, np.uint8), np.ones(n - n // 2, np.uint8)])
    T0 = np.full(n, 200.0, np.float32)
    on, moved = _staged(MAIN, T0, tidx, 1)
    off, _ = _staged(MAIN, T0, tidx, 1, merge_lanes=-1)
    print("moved events", moved, "of", n)
    assert moved > 0
    _same_records(on, off)


@pytest.mark.parametrize("n", [1, 63, 1000, 70001])
def test_merge_small_and_ragged_batches(n):
    tidx, T0 = _batch(n, 12)
    off, _ = _staged(TISSUE, T0, tidx, 4, merge_lanes=-1)
    for lanes in (0, 64):
        got, _ = _staged(TISSUE, T0, tidx, 4, merge_lanes=lanes)
        _same_records(off, got)


def test_merge_with_hooks_and_evaporation_options():
    n = 100000
    T0 = np.full(n, 180.0, np.float32)
    for opts in (dict(no_pauli=1), dict(photon_evaporation=1, heavy_fragments=1), dict(table_layout=1),
                 dict(block_size=128), dict(fast_math=1)):
        off, _ = _staged([(40, 20)], T0, None, 8, merge_lanes=-1, **opts)
        got, moved = _staged([(40, 20)], T0, None, 8, merge_lanes=64, **opts)
        print(opts, "moved events", moved)
        _same_records(off, got)


def test_merge_through_the_ring():
    import torch

    import paper_1309_7963_amd as inc

    n = 60000
    tidx, T0 = _batch(n, 13)
    off, _ = _staged(TISSUE, T0, tidx, 6, merge_lanes=-1)
    ctx = inc.Context(TISSUE, merge_lanes=64)
    ring = inc.Ring(ctx, slots=1 << 14, chunk=1 << 11)
    try:
        r = ring.simulate(torch.as_tensor(T0, device="cuda"), seed=6, target_idx=torch.as_tensor(tidx, device="cuda"))
    finally:
        ring.close()
        ctx.close()
    assert r["rc"] == 0 and r["stats"]["producer_gave_up"] == 0
    r["sec_u"] = np.stack([r["sec_ux"], r["sec_uy"], r["sec_uz"]], 1)
    _same_records(off, r)


def test_merge_option_range():
    import paper_1309_7963_amd as inc

    for bad in (-2, 65):
        with pytest.raises(inc.IncError):
            inc.Context([(16, 8)], merge_lanes=bad)
