"""inc_simulate_dev_noalloc (the entry point for callers that cannot allocate
device memory) against inc_simulate_dev, through the C ABI: two calls in a
row on one context, the second smaller than the first, each compared with
the allocating entry point on the same inputs; and the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TISSUE = [(12, 6), (14, 7), (16, 8), (31, 15), (40, 20)]
TISSUE_W = [0.18, 0.03, 0.65, 0.01, 0.13]
FIELDS = ("sec_event", "sec_species", "sec_stage", "sec_T", "sec_u")


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    tidx = rng.choice(len(TISSUE), size=n, p=TISSUE_W).astype(np.uint8)
    T0 = rng.uniform(20.0, 250.0, n).astype(np.float32)
    return tidx, T0


def _same(a, b):
    assert a["res"].tobytes() == b["res"].tobytes()
    assert a["n_sec_total"] == b["n_sec_total"]
    ka = np.lexsort((a["sec_T"], a["sec_event"]))
    kb = np.lexsort((b["sec_T"], b["sec_event"]))
    for f in FIELDS:
        assert np.array_equal(a[f][ka], b[f][kb]), f


@pytest.mark.parametrize("mode", ["staged", "persistent", "plain"])
def test_noalloc_equals_allocating_entry_point(mode):
    import torch
    import paper_1309_7963_amd as inc

    ctx = inc.Context(TISSUE)
    # the first call fills the workspace (start order included: >= 65536
    # events); the second, smaller, with a ragged last chunk, must not see it
    for n, seed, first_id in ((300_000, 3, 0), (70_001, 5, 1 << 33)):
        print("noalloc case: mode %s, n %d, seed %d" % (mode, n, seed), flush=True)
        tidx, T0 = _inputs(n, seed + 100)
        T0_d = torch.as_tensor(T0, device="cuda")
        ti_d = torch.as_tensor(tidx, device="cuda")
        cap = ctx.default_capacity(n)
        ref = ctx.simulate(T0_d, seed=seed, target_idx=ti_d, first_event_id=first_id, mode=mode, capacity=cap)
        out = inc.DeviceOutput.allocate(n, cap, T0_d.device)
        torch.cuda.synchronize()
        got = ctx.simulate_noalloc(T0_d, seed=seed, out=out, target_idx=ti_d, first_event_id=first_id, mode=mode)
        torch.cuda.synchronize()
        assert ref.n_sec() <= cap and got.n_sec() == ref.n_sec()
        _same(ref.to_numpy(), got.to_numpy())
    ctx.close()


def test_noalloc_rejects_batches_beyond_the_workspace():
    import torch
    import paper_1309_7963_amd as inc

    ctx = inc.Context([(16, 8)])
    n = inc.NOALLOC_MAX_EVENTS + 1
    T0_d = torch.full((n,), 200.0, dtype=torch.float32, device="cuda")
    out = inc.DeviceOutput.allocate(n, 16)
    with pytest.raises(inc.IncError) as e:
        ctx.simulate_noalloc(T0_d, seed=1, out=out)
    assert e.value.code == inc.INC_ERR_TOO_LARGE
    torch.cuda.synchronize()
    # nothing was launched: the counters keep their zeros
    assert out.n_sec() == 0
    # the largest batch it takes runs, and equals the allocating call
    n = inc.NOALLOC_MAX_EVENTS
    T0_d = T0_d[:n].contiguous()
    ref = ctx.simulate(T0_d, seed=2, capacity=ctx.default_capacity(n))
    got = ctx.simulate_noalloc(T0_d, seed=2, out=inc.DeviceOutput.allocate(n, ctx.default_capacity(n)))
    torch.cuda.synchronize()
    _same(ref.to_numpy(), got.to_numpy())
    ctx.close()
