"""Fast-math build of the event kernels (Sec. 4.2: approximate
transcendentals, reciprocal division, flushed denormals) against the oracle.

The fast build follows the same random stream in the same order, so every
event must still pass the float64 ledgers and the distributions must pass the
same two-sample chi-square gate as the default build; per-event replay
agreement with the oracle is reported (the approximations flip more
comparisons than FP32 rounding alone)."""
import numpy as np
import pytest

import ledger
import oracle
import stats
from gpu_util import events_from_gpu, outcome_keys, run_gpu

pytestmark = pytest.mark.gpu

O16, CA40 = (16, 8), (40, 20)
TISSUE = [(12, 6), (14, 7), (16, 8), (31, 15), (40, 20)]
TISSUE_W = [0.18, 0.03, 0.65, 0.01, 0.13]


@pytest.mark.parametrize("mode", ["plain", "persistent"])
@pytest.mark.parametrize("target,T", [(O16, 200.0), (CA40, 200.0), ((12, 6), 20.0), ((56, 26), 250.0)])
def test_fast_ledgers_every_event(mode, target, T):
    n = 20000
    T0 = np.full(n, T, dtype=np.float32)
    h = run_gpu([target], T0, seed=1, mode=mode, fast_math=1)
    s = ledger.check(events_from_gpu(h, [target], T0))
    ledger.assert_clean(s)
    assert h["n_sec_total"] == int(h["res"]["n_sec"].sum())
    assert s["max_E1"] < 1e-3 and s["max_E2"] < 1e-3 and s["max_P"] < 1e-3


def test_fast_replay_agreement_reported():
    n = 10000
    T0 = np.full(n, 200.0, dtype=np.float32)
    g = events_from_gpu(run_gpu([O16], T0, seed=1, fast_math=1), [O16], T0)
    out = oracle.run([O16], T0.astype(np.float64), seed=1, n_threads=16)
    o = ledger.from_oracle(out, [O16], T0)
    agree = np.mean([a == b for a, b in zip(outcome_keys(g), outcome_keys(o))])
    print("fast-math replay agreement", agree)
    assert agree > 0.9


def _chi2_gate(g, o, T_max, label):
    res = stats.compare_samples(g, o, T_max)
    print(label, {k: (round(v[0], 1), v[1], round(v[2], 4)) for k, v in res.items()})
    bad = stats.gate(res)
    assert not bad, (label, bad)


def test_fast_chi2_o16_paper_scale():
    n = 1_000_000
    T0 = np.full(n, 200.0, dtype=np.float32)
    g = events_from_gpu(run_gpu([O16], T0, seed=1, fast_math=1), [O16], T0)
    o = ledger.from_oracle(oracle.run([O16], T0.astype(np.float64), seed=2, n_threads=16), [O16], T0)
    _chi2_gate(g, o, 200.0, "fast 16O 200 MeV")


def test_fast_chi2_mixed():
    n = 1_000_000
    rng = np.random.default_rng(11)
    tidx = rng.choice(len(TISSUE), size=n, p=TISSUE_W).astype(np.uint8)
    T0 = rng.uniform(20, 250, n).astype(np.float32)
    g = events_from_gpu(run_gpu(TISSUE, T0, seed=1, tidx=tidx, fast_math=1), TISSUE, T0, tidx)
    o = ledger.from_oracle(oracle.run(TISSUE, T0.astype(np.float64), seed=2, tidx=tidx, n_threads=16), TISSUE, T0,
                           tidx)
    _chi2_gate(g, o, 250.0, "fast tissue mixture")
