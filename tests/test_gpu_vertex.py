"""The event-based vertex pipeline (mode "vertex", INC_MODE_VERTEX: a window
of in-flight events in device memory, one kernel per vertex type over
compacted queues, Sec. 4.2's suggested restructuring) gives the same events
as the persistent kernel: identical residual records and the same secondary
records, for every window size, with inputs out of range in the batch, and
with the evaporation options on."""
import numpy as np
import pytest

from gpu_util import run_gpu

pytestmark = pytest.mark.gpu

TISSUE = [(12, 6), (14, 7), (16, 8), (31, 15), (40, 20)]


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


@pytest.mark.parametrize("window,launch", [(1024, 0), (1 << 16, 0), (1 << 18, 0), (1 << 16, 1)])
def test_vertex_equals_persistent(window, launch):
    # launch 0: each group of cycles replays a graph captured for the call
    # (many replays per call, host reads between them); 1: plain launches
    import paper_1309_7963_amd as inc

    n = 200000
    tidx, T0 = _batch(n, 3)
    ctx = inc.Context(TISSUE, vertex_window=window, vertex_launch=launch)
    ref = run_gpu(TISSUE, T0, seed=5, tidx=tidx, mode="persistent", ctx=ctx)
    for rep in range(2):  # the second launch reuses the pipeline's buffers
        got = run_gpu(TISSUE, T0, seed=5, tidx=tidx, mode="vertex", ctx=ctx)
        _same_records(ref, got)
    assert ((ref["res"]["flags"] & inc.FLAG_RANGE) != 0).sum() == len(range(0, n, 997)) + len(range(5, n, 1009))
    ctx.close()


def test_vertex_with_evaporation_options():
    import paper_1309_7963_amd as inc

    n = 100000
    T0 = np.full(n, 200.0, dtype=np.float32)
    ctx = inc.Context([(40, 20)], photon_evaporation=1, heavy_fragments=1, vertex_window=1 << 14)
    ref = run_gpu([(40, 20)], T0, seed=7, mode="staged", ctx=ctx)
    got = run_gpu([(40, 20)], T0, seed=7, mode="vertex", ctx=ctx)
    ctx.close()
    _same_records(ref, got)
    assert (got["sec_species"] == 6).any() and (got["sec_species"] >= 7).any()


def test_vertex_window_validated():
    import paper_1309_7963_amd as inc

    for bad in (1000, 512, 1 << 21):
        with pytest.raises(inc.IncError):
            inc.Context([(16, 8)], vertex_window=bad)
    with pytest.raises(inc.IncError):
        inc.Context([(16, 8)], vertex_launch=2)


def test_vertex_mode_is_not_offered_where_unsupported():
    # the allocation-free entry point and the ring take the three kernel
    # modes only; the vertex pipeline needs its own buffers
    import torch

    import paper_1309_7963_amd as inc

    ctx = inc.Context([(16, 8)])
    T0 = torch.full((1000,), 200.0, dtype=torch.float32, device="cuda")
    out = inc.DeviceOutput.allocate(1000, ctx.default_capacity(1000))
    with pytest.raises(inc.IncError) as e:
        ctx.simulate_noalloc(T0, seed=1, out=out, mode="vertex")
    assert e.value.code == inc.INC_ERR_ARG
    ring = inc.Ring(ctx, slots=1 << 12, chunk=1 << 10)
    with pytest.raises(inc.IncError):
        ring.simulate(T0, seed=1, mode="vertex")
    ring.close()
    ctx.close()
