"""Pins of the oracle's optional photon channel of the evaporation (reading
R19: photons compete with the six particle channels, width from detailed
balance with a photoabsorption cross-section that rises linearly to the
giant-dipole energy and holds the classical dipole sum; off by default,
Sec. 2.4).  Every pin is against something the oracle does not compute
itself: numerical quadrature, closed-form limits, measured giant-dipole
energies, the dipole sum rule, and conservation laws."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy import stats

import evap_ref
import ledger
import oracle


def _quad_J(a, U, x=None):
    f = lambda e: e ** 3 * math.exp(2.0 * math.sqrt(a * max(U - e, 0.0)))
    return integrate.quad(f, 0.0, U if x is None else x, epsabs=0.0, epsrel=1e-12, limit=400)[0]


@pytest.mark.parametrize("a,U", [(2.0, 0.05), (0.5, 3.0), (2.0, 10.0), (5.0, 40.0), (7.0, 150.0), (1.5, 12.0)])
def test_photon_integral_quadrature(a, U):
    # J(a, U) = int_0^U e^3 exp(2 sqrt(a (U - e))) de: both sides of the
    # series / closed-form switch (Y = 2 sqrt(a U) = 10) included
    assert oracle.photon_integral(a, U) == pytest.approx(_quad_J(a, U), rel=1e-9)


def test_photon_integral_and_cdf_without_level_density():
    # a -> 0: the density is e^3, J = U^4 / 4 and the CDF (x / U)^4
    U = 7.0
    assert oracle.photon_integral(1e-13, U) == pytest.approx(U ** 4 / 4, rel=1e-6)
    for x in (0.5, 3.0, 6.9):
        assert oracle.photon_cdf(1e-13, U, x) == pytest.approx((x / U) ** 4, rel=1e-6)


@pytest.mark.parametrize("a,U", [(0.5, 3.0), (5.0, 8.0), (4.0, 60.0)])
def test_photon_cdf_quadrature(a, U):
    for x in np.linspace(0.05, 0.95, 7) * U:
        assert oracle.photon_cdf(a, U, x) == pytest.approx(_quad_J(a, U, x) / _quad_J(a, U), rel=1e-8, abs=1e-12)


@pytest.mark.parametrize("a,U", [(0.5, 3.0), (5.0, 8.0), (4.0, 60.0)])
def test_photon_sampler_inverts_the_cdf(a, U):
    rng = np.random.default_rng(3)
    u = rng.random(4000)
    xs = np.array([oracle.photon_sample(a, U, v) for v in u])
    assert np.all((xs >= 0) & (xs <= U))
    cdf = lambda v: np.array([_quad_J(a, U, t) for t in np.atleast_1d(v)]) / _quad_J(a, U)
    assert stats.kstest(xs, cdf).pvalue > 1e-3


def test_gdr_energy_near_measured():
    # giant-dipole resonance energies of 208Pb, 90Zr, 40Ca (within 5 %) and
    # 16O (whose resonance is fragmented; within 15 %)
    for A, E, tol in ((208, 13.4, 0.05), (90, 16.8, 0.05), (40, 19.8, 0.05), (16, 22.3, 0.15)):
        assert oracle.gdr_energy(A) == pytest.approx(E, rel=tol), A


@pytest.mark.parametrize("A,Z", [(16, 8), (40, 20), (56, 26), (208, 82)])
def test_photoabsorption_ramp_holds_the_dipole_sum(A, Z):
    # int_0^E_G s0 e de = 60 N Z / A mb MeV = 6.0 N Z / A fm^2 MeV
    EG = oracle.gdr_energy(A)
    s0 = oracle.photon_s0(A, Z)
    assert integrate.quad(lambda e: s0 * e, 0.0, EG)[0] == pytest.approx(6.0 * (A - Z) * Z / A, rel=1e-12)


def test_photon_width_against_quadrature():
    # the channel weight of the reading, formula retyped with the integral
    # by quadrature (tests/evap_ref.py); closed at and below 0.1 MeV
    for A, Z, E in ((40, 20, 13.0), (16, 8, 8.0), (56, 26, 30.0)):
        assert oracle.photon_width(A, Z, E) == pytest.approx(evap_ref.photon_weight(A, Z, E), rel=1e-9)
    assert oracle.photon_width(40, 20, 0.1) == 0.0 and oracle.photon_width(40, 20, 0.1001) > 0.0


@pytest.mark.parametrize("A,Z,E", [(40, 20, 13.0), (40, 20, 16.0), (16, 8, 12.0)])
def test_photon_branching_matches_widths(A, Z, E):
    # first-emission frequencies of 10^4 nuclei against the widths
    # (particles and photon) by quadrature
    n = 10000
    first = np.empty(n, dtype=np.int64)
    for i in range(n):
        _, s = oracle.evaporate(A, Z, E, seed=7, event_id=i, photon_evaporation=1)
        first[i] = s["species"][0]
    p = evap_ref.branching(A, Z, E, photons=True)
    obs = np.bincount(first, minlength=7)
    exp = p * n
    keep = exp >= 5
    chi2 = float(np.sum((obs[keep] - exp[keep]) ** 2 / exp[keep])) + (
        float((obs[~keep].sum() - exp[~keep].sum()) ** 2 / exp[~keep].sum()) if exp[~keep].sum() >= 5 else 0.0)
    dof = int(keep.sum()) - 1 + (1 if exp[~keep].sum() >= 5 else 0)
    print(A, Z, E, "photon share", p[6], "observed", obs[6] / n, "chi2 %.1f / %d" % (chi2, dof))
    assert obs[~keep].sum() <= max(5.0, 5 * exp[~keep].sum())
    assert stats.chi2.sf(chi2, max(dof, 1)) > 1e-3


def test_photons_below_the_particle_thresholds():
    # 40Ca at 9 MeV (lowest particle threshold 11.5 MeV), at rest: only
    # photons leave, A and Z stay, the excitation ends at or below 0.1 MeV,
    # and the photons' energies plus the recoil's kinetic energy make up the
    # excitation spent
    M = oracle.mass(40, 20)
    for i in range(200):
        r, s = oracle.evaporate(40, 20, 9.0, seed=9, event_id=i, photon_evaporation=1)
        assert (s["species"] == ledger.PHOTON).all() and len(s) >= 1
        assert r["A_f"] == 40 and r["Z_f"] == 20 and 0.0 <= r["Ex_f"] <= 0.1
        p_f = np.asarray(r["p_f"])
        assert np.allclose(p_f, -(s["u"] * s["T"][:, None]).sum(axis=0), atol=1e-9)
        T_rec = math.sqrt(p_f @ p_f + (M + r["Ex_f"]) ** 2) - (M + r["Ex_f"])
        assert s["T"].sum() + T_rec == pytest.approx(9.0 - r["Ex_f"], abs=1e-9)


def test_first_photon_spectrum():
    # the first photon of 40Ca at rest at E* = 9 MeV: its share e of the
    # excitation (from E_g = e (Mp + Md) / (2 Mp)) follows e^3 rho(E - e),
    # the CDF by quadrature
    A, Z, E = 40, 20, 9.0
    Mp = oracle.mass(A, Z) + E
    eps = []
    for i in range(5000):
        _, s = oracle.evaporate(A, Z, E, seed=11, event_id=i, photon_evaporation=1)
        Eg = s["T"][0]
        eps.append(Mp - math.sqrt(Mp * Mp - 2.0 * Mp * Eg))
    a = A / 8.0
    cdf = lambda v: np.array([_quad_J(a, E, t) for t in np.atleast_1d(v)]) / _quad_J(a, E)
    assert stats.kstest(np.array(eps), cdf).pvalue > 1e-3


def test_photon_ledgers_on_cascades():
    # whole events with the photon channel on: every ledger, every event
    # ends at or below the photon threshold (and photons only in stage 1)
    for target, T in (((16, 8), 200.0), ((40, 20), 70.0), ((56, 26), 250.0)):
        T0 = np.full(4000, T)
        out = oracle.run([target], T0, seed=13, photon_evaporation=1)
        ev = ledger.from_oracle(out, [target], T0)
        s = ledger.check(ev, photons=True)
        ledger.assert_clean(s)
        ph = ev.sec_species == ledger.PHOTON
        assert ph.sum() > 0 and (ev.sec_stage[ph] == 1).all()
        dipole = (ev.A_f - ev.Z_f) * ev.Z_f > 0
        assert (ev.Ex_f[dipole] <= 0.1 + 1e-12).all()


def test_photon_channel_is_off_by_default():
    T0 = np.full(2000, 200.0)
    ev = ledger.from_oracle(oracle.run([(40, 20)], T0, seed=13), [(40, 20)], T0)
    assert not (ev.sec_species == ledger.PHOTON).any()
    ledger.assert_clean(ledger.check(ev))
    assert (ev.Ex_f > 0.1).mean() > 0.5
