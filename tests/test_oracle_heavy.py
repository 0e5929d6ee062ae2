"""Pins of the oracle's optional heavier-fragment channels of the evaporation
(reading R20: the stable isotopes of Li to Mg, GEM's ejectiles reaching Mg,
emitted with the particles' Weisskopf-Ewing width and spectrum; off by
default, Sec. 2.4).  Pinned against widths by quadrature (tests/evap_ref.py),
spin rules of nuclear ground states, thresholds from the mass formula, and
the conservation ledgers."""
import numpy as np
import pytest
from scipy import stats

import evap_ref
import ledger
import oracle


def test_fragment_table_matches_the_ledger_and_ground_state_spin_rules():
    for j in range(27):
        f = oracle.fragment(j)
        if j == ledger.PHOTON:
            assert f is None
            continue
        a, z, g = f
        assert (a, z, g) == (ledger.FRAG_A[j], ledger.FRAG_Z[j], ledger.FRAG_G[j]), j
        if j < 7:
            continue
        n = a - z
        assert 3 <= z <= 12 and 5 < a <= 28
        # even-even ground states have spin 0; odd-A ones half-integer spin
        # (even 2s + 1); odd-odd ones integer spin >= 1 (odd 2s + 1 >= 3)
        if z % 2 == 0 and n % 2 == 0:
            assert g == 1, (a, z)
        elif a % 2 == 1:
            assert g % 2 == 0, (a, z)
        else:
            assert g % 2 == 1 and g >= 3, (a, z)
    assert oracle.fragment(27) is None and oracle.fragment(-1) is None
    # every element from Li to Mg has at least one isotope in the list
    assert set(ledger.FRAG_Z[7:]) == set(range(3, 13))


@pytest.mark.parametrize("A,Z,E", [(12, 6, 40.0), (16, 8, 50.0)])
def test_heavy_branching_matches_widths(A, Z, E):
    # first-emission frequencies of 2 x 10^4 nuclei against the 26 channels'
    # widths by quadrature
    n = 20000
    first = np.empty(n, dtype=np.int64)
    for i in range(n):
        _, s = oracle.evaporate(A, Z, E, seed=17, event_id=i, heavy_fragments=1)
        first[i] = s["species"][0]
    p = evap_ref.branching(A, Z, E, heavy=True)
    assert p[7:].sum() > 0.01  # the heavier channels matter here
    obs = np.bincount(first, minlength=27)
    exp = p * n
    keep = exp >= 5
    rest_o, rest_e = obs[~keep].sum(), exp[~keep].sum()
    chi2 = float(np.sum((obs[keep] - exp[keep]) ** 2 / exp[keep]))
    dof = int(keep.sum()) - 1
    if rest_e >= 5:
        chi2 += (rest_o - rest_e) ** 2 / rest_e
        dof += 1
    print(A, Z, E, "heavy share", p[7:].sum(), "observed", obs[7:].sum() / n, "chi2 %.1f / %d" % (chi2, dof))
    assert rest_o <= max(5.0, 5 * rest_e)
    assert stats.chi2.sf(chi2, dof) > 1e-3


def test_heavy_emission_respects_thresholds():
    # 24Mg -> 12C + 12C: the channel opens at S + V from the mass formula;
    # 10^3 nuclei just below it never emit 12C first, and the model's
    # threshold equals the one computed here from binding energies
    A, Z, j = 24, 12, 12
    thr = evap_ref.threshold(A, Z, j)
    B = oracle.binding
    V = 1.44 * 6 * 6 / (1.5 * (2 * 12 ** (1 / 3)))
    assert thr == pytest.approx(B(24, 12) - 2 * B(12, 6) + V, abs=1e-9)
    for E in (thr - 0.05, thr + 5.0):
        firsts = [oracle.evaporate(A, Z, E, seed=19, event_id=i, heavy_fragments=1)[1]["species"][0]
                  for i in range(1000)]
        if E < thr:
            assert j not in firsts
    p = evap_ref.branching(A, Z, thr + 5.0, heavy=True)
    assert p[j] > 0.0


def test_heavy_ledgers_on_cascades():
    # whole events with the heavier channels on: every ledger (A, Z, energy,
    # momentum), no channel left open, heavier fragments only in stage 1
    for target, T in (((16, 8), 200.0), ((40, 20), 150.0), ((27, 13), 250.0)):
        T0 = np.full(4000, T)
        out = oracle.run([target], T0, seed=23, heavy_fragments=1)
        ev = ledger.from_oracle(out, [target], T0)
        ledger.assert_clean(ledger.check(ev, heavy=True))
        hv = ev.sec_species >= 7
        assert hv.sum() > 0 and (ev.sec_stage[hv] == 1).all()


def test_heavy_and_photons_together():
    T0 = np.full(3000, 200.0)
    out = oracle.run([(40, 20)], T0, seed=29, heavy_fragments=1, photon_evaporation=1)
    ev = ledger.from_oracle(out, [(40, 20)], T0)
    ledger.assert_clean(ledger.check(ev, photons=True, heavy=True))
    assert (ev.sec_species == ledger.PHOTON).any() and (ev.sec_species >= 7).any()


def test_heavy_channels_are_off_by_default():
    T0 = np.full(3000, 200.0)
    base = oracle.run([(24, 12)], T0, seed=31)
    ev = ledger.from_oracle(base, [(24, 12)], T0)
    assert not (ev.sec_species >= 7).any()
    ledger.assert_clean(ledger.check(ev))
    # the default model is the same with the option field present and zero
    again = oracle.run([(24, 12)], T0, seed=31, heavy_fragments=0)
    for a, b in ((base.results, again.results), (base.secondaries, again.secondaries)):
        for name in a.dtype.names:
            assert np.array_equal(a[name], b[name], equal_nan=a[name].dtype.kind == "f"), name
