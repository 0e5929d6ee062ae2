"""The element-wise replay gate (tests/elementwise.py) on the CPU, with the
oracle standing in for both sides: an implementation that differs from the
oracle only by rounding-sized changes passes, and an error planted in one
value of one well-conditioned event fails."""
import dataclasses

import numpy as np
import pytest

import elementwise
import ledger
import oracle

O16 = [(16, 8)]


def _run(T0, seed=1):
    out = oracle.run(O16, T0, seed=seed, n_threads=8)
    return ledger.from_oracle(out, O16, T0), out


@pytest.fixture(scope="module")
def sides():
    n = 5000
    T0 = np.full(n, 200.0)
    o, o_out = _run(T0)
    # stand-in for a second implementation: the same events with the input
    # three FP32 ulps higher (a rounding-sized difference everywhere downstream)
    T3 = np.float32(200.0)
    for _ in range(3):
        T3 = np.nextafter(T3, np.float32(np.inf))
    g, g_out = _run(np.full(n, float(T3)))
    Tp, delta = elementwise.one_ulp_up(T0)
    p, p_out = _run(Tp)
    hist = np.stack([g_out.results["n_draw"], g_out.results["n_seg"], g_out.results["tent_shells"]], 1)
    return dict(o=o, o_out=o_out, g=g, g_out=g_out, p=p, p_out=p_out, delta=delta, hist=hist)


def _gate(s, g):
    elementwise.assert_replay_close(g, s["o"], s["g_out"].results, s["o_out"].results, "oracle stand-in",
                                    g_hist=s["hist"], o_pert=(s["p"], s["p_out"].results), delta=s["delta"])


def test_rounding_sized_differences_pass(sides):
    _gate(sides, sides["g"])


def test_planted_error_in_one_value_fails(sides):
    g, o = sides["g"], sides["o"]
    m = elementwise.same_history(g, o)
    D = elementwise.event_deviation(o, sides["p"], elementwise.same_history(o, sides["p"]))
    # a well-conditioned event with records: raise its first record's T by 1 %
    cand = np.flatnonzero(m & (D < 1e-6) & (g.n_sec > 0))
    assert cand.size > 100
    e = cand[0]
    k = np.flatnonzero(g.sec_event == e)[0]
    T = g.sec_T.copy()
    T[k] *= 1.01
    with pytest.raises(AssertionError):
        _gate(sides, dataclasses.replace(g, sec_T=T))
    # and one wrong excitation energy
    Ex = g.Ex_f.copy()
    Ex[e] += 0.05
    with pytest.raises(AssertionError):
        _gate(sides, dataclasses.replace(g, Ex_f=Ex))
