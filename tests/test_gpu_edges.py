"""Edge cases of the GPU path against the oracle's invariants.

* ragged batch sizes (1, 63, 65, 257, 1000 events: a partial wave, one event
  past a wave, past a block) give the same events in every launch mode and
  pass the ledgers;
* the smallest and largest admissible targets (4He, A = 250) at both ends of
  the energy range, including the degenerate 250/1 (no binding: the segment
  guard ends most events, as often as in the oracle);
* a context with the maximum number of targets (16) and a mixture over all;
* every launch policy the autotuner tries gives the same events;
* the staged evaporation kernel's share (chunks of waves that took more than
  they keep) gives the same events as the cascade waves' own evaporation;
* the costliest-first start order gives the same events as input order."""
import numpy as np
import pytest

import ledger
import oracle
from gpu_util import events_from_gpu, outcome_keys, run_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 63, 65, 257, 1000])
def test_ragged_batches_same_in_every_mode(n):
    targets = [(16, 8), (40, 20)]
    rng = np.random.default_rng(n)
    tidx = rng.integers(0, 2, n).astype(np.uint8)
    T0 = rng.uniform(20, 250, n).astype(np.float32)
    runs = {m: run_gpu(targets, T0, seed=2, tidx=tidx, mode=m) for m in ("plain", "persistent", "staged")}
    ref = runs["staged"]
    ledger.assert_clean(ledger.check(events_from_gpu(ref, targets, T0, tidx)))
    for m, h in runs.items():
        assert h["res"].tobytes() == ref["res"].tobytes(), m
        assert h["n_sec_total"] == ref["n_sec_total"], m
    # the first events of a batch do not depend on its length
    whole = run_gpu(targets, np.tile(T0, 3), seed=2, tidx=np.tile(tidx, 3))
    assert whole["res"][:n].tobytes() == ref["res"].tobytes()


@pytest.mark.parametrize("target", [(4, 2), (250, 98), (250, 1)])
@pytest.mark.parametrize("T", [20.0, 250.0])
def test_extreme_targets_and_energies(target, T):
    n = 20000
    T0 = np.full(n, T, np.float32)
    h = run_gpu([target], T0, seed=3, capacity=n * (target[0] + 1))
    ev = events_from_gpu(h, [target], T0)
    if target == (250, 1):
        # ~100-250 emissions per event: the FP32 recoil momentum loses up to
        # half an ulp of |p| <= 730 MeV/c per component and emission, so the
        # momentum bar is 250 x 2^-24 x 730 MeV/c = 1.1e-2 MeV/c; measured
        # 1.3e-3 at 250 MeV, so the flat 1e-3 bar of real targets (up to ~25
        # emissions) does not hold here
        s = ledger.check(ev, tol_p=250 * 2.0 ** -24 * 730.0)
    else:
        s = ledger.check(ev)
    print("extreme target", target, T, "max |E1| %.2e MeV, max |E2| %.2e MeV, max |P| %.2e MeV/c"
          % (s["max_E1"], s["max_E2"], s["max_P"]))
    ledger.assert_clean(s)
    flags = h["res"]["flags"].astype(np.int64)
    assert ((flags & 0x8000) == 0).all()
    assert ((flags & ~7) == 0).all()
    if target == (250, 1):
        # degenerate target (no binding): most events trip the segment guard;
        # the guarded fraction matches the oracle's
        out = oracle.run([target], T0[:1000].astype(np.float64), seed=5, n_threads=16)
        f_gpu = np.mean((flags & 2) != 0)
        f_orc = np.mean((out.results["flags"] & 2) != 0)
        print("segment-guard fraction", target, T, f_gpu, f_orc)
        assert abs(f_gpu - f_orc) < 0.05


def test_sixteen_targets_in_one_context():
    targets = [(12, 6), (14, 7), (16, 8), (20, 10), (24, 12), (27, 13), (31, 15), (32, 16),
               (40, 20), (48, 22), (56, 26), (63, 29), (90, 40), (120, 50), (197, 79), (238, 92)]
    n = 64000
    rng = np.random.default_rng(16)
    tidx = rng.integers(0, 16, n).astype(np.uint8)
    T0 = rng.uniform(20, 250, n).astype(np.float32)
    h = run_gpu(targets, T0, seed=4, tidx=tidx)
    ev = events_from_gpu(h, targets, T0, tidx)
    ledger.assert_clean(ledger.check(ev))
    # each event equals the same event generated in a one-target context
    for t in (0, 7, 15):
        sel = np.nonzero(tidx == t)[0][:200]
        assert sel.size > 0
        # event identity is (seed, id): regenerate those ids one by one
        for i in sel[:5]:
            single = run_gpu([targets[t]], T0[i:i + 1], seed=4, first_id=int(i))
            assert single["res"].tobytes() == h["res"][i:i + 1].tobytes()


def test_autotuned_policy_changes_speed_not_results():
    """The autotuner picks among launch policies (block size and waves per
    CU, scheduler thresholds, LIFO levels in LDS, events per queue claim, the
    NN table's LDS layout); every candidate must produce the same events, in
    staged and in fused persistent mode."""
    from paper_1309_7963_amd import autotune

    targets = [(12, 6), (16, 8), (208, 82)]
    rng = np.random.default_rng(11)
    n = 20000
    tidx = rng.choice(3, n, p=[0.45, 0.45, 0.1]).astype(np.uint8)
    T0 = rng.uniform(20, 250, n).astype(np.float32)
    dims = {
        "launch": (dict(block_size=128, waves_per_cu=8), dict(block_size=256, waves_per_cu=12)),
        "thresholds": (dict(kin_threshold=24, tent_threshold=24, start_threshold=8),
                       dict(kin_threshold=16, tent_threshold=8, start_threshold=8)),
        "stack_levels": (dict(stack_levels=-1), dict(stack_levels=1), dict(stack_levels=0)),
        "chunk_events": (dict(chunk_events=16), dict(chunk_events=128), dict(chunk_events=1024)),
        "table_layout": (dict(table_layout=0), dict(table_layout=1)),
    }
    best = autotune.tune(targets, T0, tidx, dimensions=dims, repeats=2, use_cache=False)
    assert len(best["table"]) == 12 and best["ms"] > 0 and best["default_ms"] > 0
    swept = best["swept_options"]
    for name, cands in dims.items():
        assert any(all(swept[k] == v for k, v in c.items()) for c in cands), name
    if best["options"]:  # else the library default was kept (not clearly faster)
        assert best["options"] == swept and best["ms"] < best["default_ms"]
    for mode in ("staged", "persistent"):
        ref = run_gpu(targets, T0, seed=4, tidx=tidx, mode=mode)
        for cand in best["table"]:
            h = run_gpu(targets, T0, seed=4, tidx=tidx, mode=mode, **cand["options"])
            assert h["res"].tobytes() == ref["res"].tobytes(), (mode, cand["options"])
            assert h["n_sec_total"] == ref["n_sec_total"], (mode, cand["options"])


def test_staged_evaporation_overflow_pass():
    """In staged mode a cascade wave evaporates the events of the chunks it
    took (it keeps up to 64); a wave that took more lists the others for the
    evaporation kernel.  One wave per CU on 1.2e6 events takes that path; the
    events must equal those of the default grid."""
    targets = [(16, 8), (40, 20)]
    rng = np.random.default_rng(21)
    n = 1_200_000
    tidx = rng.integers(0, 2, n).astype(np.uint8)
    T0 = np.full(n, 200.0, np.float32)
    few = run_gpu(targets, T0, seed=8, tidx=tidx, mode="staged", waves_per_cu=1)
    ref = run_gpu(targets, T0, seed=8, tidx=tidx, mode="staged")
    assert few["res"].tobytes() == ref["res"].tobytes()
    assert few["n_sec_total"] == ref["n_sec_total"]


@pytest.mark.parametrize("mode", ["persistent", "staged"])
def test_costliest_first_start_order_changes_nothing(mode):
    """Launches of >= 65536 events on a context's own buffers start the events
    with the largest expected cost first (a device counting sort); starting
    them in input order must give the same events."""
    targets = [(12, 6), (16, 8), (40, 20)]
    rng = np.random.default_rng(31)
    n = 150_000
    tidx = rng.integers(0, 3, n).astype(np.uint8)
    T0 = rng.uniform(20, 250, n).astype(np.float32)
    T0[::997] = 300.0  # out of range: flagged, sorted last
    ordered = run_gpu(targets, T0, seed=6, tidx=tidx, mode=mode)
    inorder = run_gpu(targets, T0, seed=6, tidx=tidx, mode=mode, input_order=1)
    assert ordered["res"].tobytes() == inorder["res"].tobytes()
    assert ordered["n_sec_total"] == inorder["n_sec_total"]


def test_batches_in_flight_on_two_streams_equal_one_at_a_time():
    """Consecutive batches with two on the device at once (each with its own
    context, buffers and stream, as the benchmark runs them) give the same
    events as the same batches run one after another."""
    import torch
    import paper_1309_7963_amd as inc

    targets = [(16, 8), (40, 20)]
    n = 200_000
    rng = np.random.default_rng(31)
    tidx = rng.integers(0, 2, n).astype(np.uint8)
    T0 = np.full(n, 200.0, np.float32)
    T0_d = torch.as_tensor(T0, device="cuda")
    ti_d = torch.as_tensor(tidx, device="cuda")
    ctxs = [inc.Context(targets) for _ in range(2)]
    streams = [torch.cuda.Stream() for _ in range(2)]
    outs = [[inc.DeviceOutput.allocate(n, ctxs[0].default_capacity(n)) for _ in range(2)] for _ in range(2)]
    for k in range(4):
        i = k % 2
        ctxs[i].simulate(T0_d, seed=3, target_idx=ti_d, out=outs[i][k // 2], first_event_id=k * n, stream=streams[i])
    torch.cuda.synchronize()
    for k in range(4):
        ref = run_gpu(targets, T0, seed=3, tidx=tidx, mode="staged", first_id=k * n)
        got = outs[k % 2][k // 2].to_numpy()
        assert got["res"].tobytes() == ref["res"].tobytes(), k
        assert got["n_sec_total"] == ref["n_sec_total"], k
    for c in ctxs:
        c.close()
