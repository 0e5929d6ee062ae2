"""Parity at the benchmark's full size and launch configuration: 10^6 events
each of 200 MeV p + 16O and p + 40Ca in one staged-mode launch on a context
with the default options (what bench.py times).

* every one of the 2x10^6 events passes the float64 ledgers (properties that
  hold at any size);
* sampled outputs the oracle computes event by event: three blocks of events
  (start, the 16O/40Ca boundary, end of the batch) replayed by the oracle with
  the same seed and event ids agree in their integer outcomes (same bar as
  the small-size replay test), and value by value where their discrete
  histories agree;
* distributions: each 10^6-event half of the launch against 10^6 oracle
  events of its target with another seed (the same statistics and bars as
  the paper-scale test)."""
import numpy as np
import pytest

import elementwise
import ledger
import oracle
import stats
from gpu_util import events_from_gpu, events_slice, outcome_keys, run_gpu

pytestmark = pytest.mark.gpu

TARGETS = [(16, 8), (40, 20)]
N = 2_000_000


def test_bench_size_ledgers_and_sampled_replay():
    half = N // 2
    tidx = np.concatenate([np.zeros(half, np.uint8), np.ones(N - half, np.uint8)])
    T0 = np.full(N, 200.0, np.float32)
    h = run_gpu(TARGETS, T0, seed=1, tidx=tidx, mode="staged", history=True)
    ev = events_from_gpu(h, TARGETS, T0, tidx)
    s = ledger.check(ev)
    ledger.assert_clean(s)
    assert h["n_sec_total"] == int(h["res"]["n_sec"].sum())
    assert s["max_E1"] < 1e-3 and s["max_E2"] < 1e-3 and s["max_P"] < 1e-3
    keys = outcome_keys(ev)
    m = 3000
    for start in (0, half - m // 2, N - m):
        sl = slice(start, start + m)
        out = oracle.run(TARGETS, T0[sl].astype(np.float64), seed=1, tidx=tidx[sl], first_id=start, n_threads=16)
        o = ledger.from_oracle(out, TARGETS, T0[sl], tidx[sl])
        ko = outcome_keys(o)
        agree = np.mean([a == b for a, b in zip(keys[sl], ko)])
        print("bench-size replay block at", start, agree)
        assert agree > 0.97
        Tp, delta = elementwise.one_ulp_up(T0[sl], top=250.0)
        outp = oracle.run(TARGETS, Tp, seed=1, tidx=tidx[sl], first_id=start, n_threads=16)
        elementwise.assert_replay_close(events_slice(ev, start, start + m), o, h["res"][sl], out.results,
                                        "bench-size replay block at %d" % start, g_hist=h["history"][sl],
                                        o_pert=(ledger.from_oracle(outp, TARGETS, Tp, tidx[sl]), outp.results),
                                        delta=delta)
    # each half against the oracle's own 10^6 events of that target (seed 2)
    for t, sl in ((0, slice(0, half)), (1, slice(half, N))):
        g = events_slice(ev, sl.start, sl.stop)
        out = oracle.run([TARGETS[t]], T0[sl].astype(np.float64), seed=2, n_threads=16)
        o = ledger.from_oracle(out, [TARGETS[t]], T0[sl])
        res = stats.compare_samples(g, o, 200.0)
        print("bench-size half", TARGETS[t], {k: (round(v[0], 1), v[1], round(v[2], 4)) for k, v in res.items()})
        assert not stats.gate(res), stats.gate(res)


def test_four_times_the_bench_size():
    # 8x10^6 events of the tissue mixture (12C/14N/16O/31P/40Ca, U(20, 250) MeV)
    # in one staged launch: the work queue, the costliest-first start order
    # over many cost buckets and the hand-over buffer at four times the
    # benchmark's size; ledgers on every event and the oracle's replay of a
    # block at each end of the batch
    targets = [(12, 6), (14, 7), (16, 8), (31, 15), (40, 20)]
    n = 8_000_000
    rng = np.random.default_rng(41)
    tidx = rng.choice(5, n, p=[0.18, 0.03, 0.65, 0.01, 0.13]).astype(np.uint8)
    T0 = rng.uniform(20.0, 250.0, n).astype(np.float32)
    h = run_gpu(targets, T0, seed=2, tidx=tidx, mode="staged", history=True)
    ev = events_from_gpu(h, targets, T0, tidx)
    s = ledger.check(ev)
    print("8x10^6 events: max momentum residual %.2e MeV/c" % s["max_P"])
    ledger.assert_clean(s)
    assert h["n_sec_total"] == int(h["res"]["n_sec"].sum())
    m = 2000
    for start in (0, n - m):
        sl = slice(start, start + m)
        out = oracle.run(targets, T0[sl].astype(np.float64), seed=2, tidx=tidx[sl], first_id=start, n_threads=16)
        o = ledger.from_oracle(out, targets, T0[sl], tidx[sl])
        ko = outcome_keys(o)
        kg = outcome_keys(events_slice(ev, start, start + m))
        agree = np.mean([a == b for a, b in zip(kg, ko)])
        print("8x10^6 events: replay block at", start, agree)
        assert agree > 0.97
        Tp, delta = elementwise.one_ulp_up(T0[sl], top=250.0)
        outp = oracle.run(targets, Tp, seed=2, tidx=tidx[sl], first_id=start, n_threads=16)
        elementwise.assert_replay_close(events_slice(ev, start, start + m), o, h["res"][sl], out.results,
                                        "8x10^6 events: replay block at %d" % start, g_hist=h["history"][sl],
                                        o_pert=(ledger.from_oracle(outp, targets, Tp, tidx[sl]), outp.results),
                                        delta=delta)
