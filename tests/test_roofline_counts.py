"""The step totals behind the benchmark's algorithmic work count
(bench.step_counts: how many optical depths, majorants, crossings ... an
event's history holds, derived from the oracle's per-event counters) against
the oracle's own direct counts of the same steps, on whole events; and the
per-step operation counts (bench.STEP_OPS) summed as the benchmark weighs
them."""
import numpy as np
import pytest

import bench
import oracle


@pytest.mark.parametrize("target,T", [((16, 8), 200.0), ((40, 20), 200.0), ((12, 6), 70.0), ((56, 26), 250.0)])
def test_step_totals_equal_the_oracles_direct_counts(target, T):
    out = oracle.run([target], np.full(20000, T), seed=3, n_threads=8)
    r = out.results
    c = bench.step_counts(r)
    assert c["tau"] == int(r["n_tau"].sum())
    assert c["majorant"] == int(r["n_majorant"].sum())
    # every segment ends in a tentative collision or at a boundary
    assert c["crossing"] + c["tentative"] == c["segment"]
    assert c["entry"] >= len(r) and c["escape"] >= 0


def test_step_costs_are_the_weighted_sums_of_their_items():
    w = bench.OP_WEIGHTS
    assert w == (1, 4, 8)
    for step, items in bench.STEP_OPS.items():
        total = sum(b + 4 * t + 8 * x for _, b, t, x in items)
        assert bench.STEP_COST[step] == pytest.approx(total), step
        assert all(b >= 0 and t >= 0 and x >= 0 for _, b, t, x in items)
    # a uniform costs a quarter of a Philox4x32-10 block: 10 rounds of two
    # 32-bit products (lo and hi halves) and four xors, nine key bumps of two
    # adds, a counter bump
    assert bench.STEP_OPS["draw"][0][1] == pytest.approx((10 * (2 * 2 + 4) + 9 * 2 + 1) / 4)


def test_algorithmic_work_per_event_on_the_benchmark_targets():
    # the per-event means quoted beside the roofline (200 MeV, 16O and 40Ca)
    for target, lo, hi in (((16, 8), 24000, 28000), ((40, 20), 37000, 42000)):
        out = oracle.run([target], np.full(20000, 200.0), seed=1, n_threads=8)
        ops = bench.algorithmic_ops_per_event(out.results)
        assert lo < ops < hi, (target, ops)
