"""Pins of the CPU oracle against facts fixed outside it: published
known-answer vectors, closed forms, quadrature of the defining integrals,
special cases with textbook answers, and conservation laws.

Each test names the passage of arXiv:1309.7963 (or the reading of it) that
the pinned function implements.
"""
import dataclasses
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

import evap_ref
import ledger
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
M_P, M_N = 938.272088, 939.565420
HBARC = 197.3269804


# ------------------------------------------------- Philox stream and uniforms
def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((tuple(v[0:4]), tuple(v[4:6]), tuple(v[6:10])))
    return rows


@pytest.mark.parametrize("ctr,key,want", _kat_rows())
def test_philox_known_answers(ctr, key, want):
    # per-event random numbers (Sec. 3.1 draws them per thread); Philox4x32-10
    assert oracle.philox(ctr, key) == want


def test_uniform_mapping_edges():
    assert oracle.uniform(0) == 2.0 ** -24
    assert oracle.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert oracle.uniform(1 << 31) == 0.5 + 2.0 ** -24
    # every value is exactly a float32
    for w in (0, 1, 511, 512, 0x12345678, 0xFFFFFE00, 0xFFFFFFFF):
        u = oracle.uniform(w)
        assert float(np.float32(u)) == u and 0.0 < u < 1.0


def test_stream_layout():
    # word k of event id under seed s is word k%4 of philox((k//4, id lo, id hi, 0), (s lo, s hi))
    seed, eid = 0x0123456789ABCDEF, (7 << 32) + 5
    for k in (0, 1, 2, 3, 4, 9, 1001):
        w = oracle.philox((k // 4, eid & 0xFFFFFFFF, eid >> 32, 0), (seed & 0xFFFFFFFF, seed >> 32))[k % 4]
        assert oracle.stream_uniform(seed, eid, k) == oracle.uniform(w)


# -------------------------------------------------- nucleus shells (Sec. 2.2)
@pytest.mark.parametrize("A,Z", [(12, 6), (16, 8), (40, 20), (56, 26)])
def test_shell_integrals_quadrature(A, Z):
    nu = oracle.nucleus(A, Z)
    c, d = 1.07 * A ** (1 / 3), 0.545
    assert nu.c == pytest.approx(c, rel=1e-14) and nu.R == pytest.approx(c + 2.5, rel=1e-14)
    f = lambda r: r * r / (1.0 + math.exp((r - c) / d))
    for i in range(15):
        ref = integrate.quad(f, nu.r[i], nu.r[i + 1], epsabs=0, epsrel=1e-13)[0]
        assert nu.integral[i] == pytest.approx(ref, rel=1e-10)


@pytest.mark.parametrize("A", [12, 16, 40, 56])
def test_fermi_profile_polylog(A):
    # int_0^inf r^2 / (1 + e^{(r-c)/d}) dr = -2 d^3 Li_3(-e^{c/d})
    mpmath = pytest.importorskip("mpmath")
    c, d = 1.07 * A ** (1 / 3), 0.545
    closed = float(-2 * d ** 3 * mpmath.polylog(3, -mpmath.e ** (c / d)))
    nu = oracle.nucleus(A, A // 2)
    inside = sum(nu.integral)
    tail = integrate.quad(lambda r: r * r / (1.0 + math.exp((r - c) / d)), nu.R, 60.0, epsrel=1e-13)[0]
    assert inside + tail == pytest.approx(closed, rel=1e-9)


@pytest.mark.parametrize("A,Z", [(12, 6), (16, 8), (31, 15), (40, 20), (48, 22), (56, 26)])
def test_shells_hold_the_nucleons(A, Z):
    nu = oracle.nucleus(A, Z)
    vol = [4 / 3 * math.pi * (nu.r[i + 1] ** 3 - nu.r[i] ** 3) for i in range(15)]
    assert sum(nu.rho[1][i] * vol[i] for i in range(15)) == pytest.approx(Z, rel=1e-12)
    assert sum(nu.rho[0][i] * vol[i] for i in range(15)) == pytest.approx(A - Z, rel=1e-12)
    # Fermi gas: the occupied momentum-space volume of every shell holds its nucleons
    for sp, count in ((1, Z), (0, A - Z)):
        states = sum(vol[i] * (nu.pF[sp][i] / HBARC) ** 3 / (3 * math.pi ** 2) for i in range(15))
        assert states == pytest.approx(count, rel=1e-12)
    # densities fall outwards, E_F follows, and E_F is the relativistic kinetic energy
    for sp, m in ((0, M_N), (1, M_P)):
        for i in range(14):
            assert nu.rho[sp][i] > nu.rho[sp][i + 1]
            assert nu.EF[sp][i] > nu.EF[sp][i + 1]
        for i in range(15):
            p = nu.pF[sp][i]
            assert nu.EF[sp][i] == pytest.approx(math.hypot(p, m) - m, rel=1e-12)
            assert nu.EF[sp][i] < p * p / (2 * m)


def test_uniform_density_hook():
    nu = oracle.nucleus(16, 8, uniform_density=1)
    rho = 16 / (4 / 3 * math.pi * nu.R ** 3)
    for i in range(15):
        assert nu.rho[0][i] + nu.rho[1][i] == pytest.approx(rho, rel=1e-12)


def test_binding_energy_systematics():
    # SEMF (reading): B/A near 8 MeV for the therapy nuclei, maximal near iron
    BA = {A: oracle.binding(A, Z) / A for A, Z in [(12, 6), (16, 8), (40, 20), (56, 26), (208, 82)]}
    for A, v in BA.items():
        assert 7.0 < v < 9.0, (A, v)
    assert BA[56] > BA[16] and BA[56] > BA[208]
    # measured values for A <= 4 (deuteron, triton, helion, alpha)
    assert oracle.binding(4, 2) == pytest.approx(28.29566)
    assert oracle.binding(2, 1) == pytest.approx(2.224566)
    assert oracle.mass(1, 1) == pytest.approx(M_P) and oracle.mass(1, 0) == pytest.approx(M_N)


def test_binding_energies_near_measured():
    # the semi-empirical formula of the binding-energy reading against measured
    # total binding energies (atomic mass evaluation, MeV): within 3 % from 12C
    # on and 1 % from 40Ca on, so a slip in any coefficient shows
    measured = {(12, 6): 92.162, (16, 8): 127.619, (40, 20): 342.052, (56, 26): 492.254, (208, 82): 1636.43}
    for (A, Z), b in measured.items():
        rel = abs(oracle.binding(A, Z) / b - 1.0)
        assert rel < (0.01 if A >= 40 else 0.03), (A, Z, rel)


# ------------------------------------------------------- Fermi sphere (Sec. 2.2)
def test_fermi_sampling_distribution():
    rng = np.random.default_rng(11)
    pF = 250.0
    u = rng.random((40000, 3))
    p = np.array([oracle.fermi_sample(pF, *row) for row in u])
    mag = np.linalg.norm(p, axis=1)
    # |p|/pF has CDF x^3 (quadratic distribution of Sec. 2.2), direction isotropic
    assert stats.kstest((mag / pF) ** 3, "uniform").pvalue > 1e-3
    assert stats.kstest((p[:, 2] / mag + 1) / 2, "uniform").pvalue > 1e-3
    assert np.mean(mag ** 2) == pytest.approx(0.6 * pF ** 2, rel=0.02)


# -------------------------------------------------- NN cross-sections (Sec. 2.3)
def test_sigma_anchor_values():
    # stand-in parameterisation at 200 MeV lab kinetic energy
    p = math.sqrt(200.0 ** 2 + 2 * 200.0 * M_P) / 1000
    assert oracle.sigma(1, p) == pytest.approx(23.5, abs=0.05)
    assert oracle.sigma(0, p) == pytest.approx(43.1, abs=0.1)
    # low energies are much larger, np above pp
    assert oracle.sigma(0, 0.3) > oracle.sigma(1, 0.3) > 40


@pytest.mark.parametrize("like", [0, 1])
def test_sigma_continuity(like):
    # the max rule leaves one join, at 0.8 GeV/c, with a jump below 0.06 mb
    assert abs(oracle.sigma(like, 0.8 - 1e-12) - oracle.sigma(like, 0.8)) < 0.06
    ps = np.linspace(0.1374, 1.5, 20001)
    s = np.array([oracle.sigma(like, p) for p in ps])
    d = np.abs(np.diff(s))
    mid = 0.5 * (ps[1:] + ps[:-1])
    # elsewhere no step exceeds twice its neighbours' (no hidden jump)
    k = np.arange(1, d.size - 1)
    ok = d[k] <= 2 * np.maximum(d[k - 1], d[k + 1]) + 1e-6
    assert np.all(ok | (np.abs(mid[k] - 0.8) < 1e-3))
    assert np.all(s > 0)


@pytest.mark.parametrize("like", [0, 1])
def test_sigma_hat_is_the_suffix_maximum(like):
    ps = np.linspace(0.1374, 1.5, 30001)
    s = np.array([oracle.sigma(like, p) for p in ps])
    suffix = np.maximum.accumulate(s[::-1])[::-1]
    for k in range(0, len(ps), 997):
        sh = oracle.sigma_hat(like, ps[k])
        assert sh >= suffix[k] - 1e-12
        assert sh <= suffix[k] + 1e-3
    # below the floor the argument is clamped
    assert oracle.sigma_hat(like, 0.01) == pytest.approx(oracle.sigma_hat(like, 0.1374))


def test_plab_min_is_the_minimum_over_the_sphere():
    rng = np.random.default_rng(5)
    for p, pF in ((600.0, 250.0), (300.0, 200.0), (150.0, 260.0)):
        best = math.inf
        Ex = math.hypot(p, M_P)
        for _ in range(20000):
            q = oracle.fermi_sample(pF, *rng.random(3))
            Et = math.hypot(np.linalg.norm(q), M_N)
            # invariant: p_lab m_y = sqrt((P_x . P_y)^2 - m_x^2 m_y^2)
            dotp = Ex * Et - p * q[2]
            best = min(best, math.sqrt(max(dotp ** 2 - (M_P * M_N) ** 2, 0.0)) / M_N)
        lo = oracle.plab_min(p, M_P, pF, M_N)
        assert lo <= best + 1e-9
        assert best - lo < 0.05 * p + 5.0


# ------------------------------------- angular-distribution slope (Sec. 2.3)
# Reading R9 (recalled Cugnon slopes, (GeV/c)^-2): b_pp = 5.5 p^8 / (7.7 + p^8);
# b_np = 0 below 0.225 GeV/c, 16.53 (p - 0.225) up to 0.6, -1.63 p + 7.16 above.
def test_slope_unlike_breaks_and_branches():
    for p in (0.1374, 0.15, 0.2, 0.2249999):
        assert oracle.slope(0, p) == 0.0
    assert 0.0 < oracle.slope(0, 0.2250001) < 1e-5
    # the two branches meet at 0.6 GeV/c within 0.02 (6.199 against 6.182)
    left, right = oracle.slope(0, 0.6 - 1e-12), oracle.slope(0, 0.6)
    assert left == pytest.approx(16.53 * 0.375, abs=1e-9)
    assert right == pytest.approx(7.16 - 1.63 * 0.6, abs=1e-9)
    assert abs(left - right) < 0.02
    # branch gradients, from differences (a slipped coefficient moves them)
    assert (oracle.slope(0, 0.5) - oracle.slope(0, 0.3)) / 0.2 == pytest.approx(16.53, rel=1e-9)
    assert (oracle.slope(0, 1.2) - oracle.slope(0, 0.8)) / 0.4 == pytest.approx(-1.63, rel=1e-9)
    # outside the table range the argument is clamped like the cross-sections'
    assert oracle.slope(0, 3.0) == oracle.slope(0, 1.5)


def test_slope_like_shape():
    ps = np.linspace(0.1374, 1.5, 500)
    b = np.array([oracle.slope(1, p) for p in ps])
    assert np.all(np.diff(b) > 0) and b[0] < 1e-5
    # half of the asymptote 5.5 where p^8 = 7.7
    assert oracle.slope(1, 7.7 ** 0.125) == pytest.approx(2.75, rel=1e-12)
    assert oracle.slope(1, 1.0) == pytest.approx(5.5 / 8.7, rel=1e-12)


def _pstar2_at_rest(T, mx, my):
    # CM momentum squared of x (kinetic energy T) on y at rest, MeV^2
    s = mx * mx + my * my + 2 * my * (T + mx)
    return (s - (mx + my) ** 2) * (s - (mx - my) ** 2) / (4 * s)


def test_slope_anchors_at_200_MeV():
    # the frozen reading's anchors: k = 2 b p*^2 is ~0.004 for pp (nearly
    # isotropic) and ~1.15 for np (forward-peaked) at 200 MeV lab
    T = 200.0
    for like, (mx, my), k_want, tol in ((1, (M_P, M_P), 0.004, 2e-4), (0, (M_P, M_N), 1.15, 5e-3)):
        plab = math.sqrt(T * T + 2 * T * mx)
        k = 2 * oracle.slope(like, plab / 1000) * _pstar2_at_rest(T, mx, my) / 1e6
        assert k == pytest.approx(k_want, abs=tol), (like, k)


def test_np_angular_mean_through_the_slope():
    # 200 MeV proton on a neutron at rest: the slope at the collision's p_lab
    # fed to the elastic kinematics gives 1 - cos(theta*) with density
    # ~ exp(-k y) on [0, 2], mean 1/k - 2/(e^{2k} - 1)
    T = 200.0
    p = math.sqrt(T * T + 2 * T * M_P)
    plab = oracle.elastic([0, 0, p], M_P, [0, 0, 0], M_N, 0.0, 0.5, 0.5)[4]
    b = oracle.slope(0, plab / 1000)
    ps2 = _pstar2_at_rest(T, M_P, M_N)
    k = 2 * b * ps2 / 1e6
    rng = np.random.default_rng(29)
    y = np.array([M_N * oracle.elastic([0, 0, p], M_P, [0, 0, 0], M_N, b, *rng.random(2))[3] / ps2
                  for _ in range(40000)])
    mean = 1 / k - 2 / math.expm1(2 * k)
    assert abs(y.mean() - mean) < 4 * y.std() / math.sqrt(y.size), (y.mean(), mean)


# ------------------------------------------------ elastic kinematics (Sec. 2.3)
def test_elastic_four_momentum_conservation():
    rng = np.random.default_rng(3)
    for _ in range(300):
        px = rng.normal(size=3) * 400
        pt = rng.normal(size=3) * 150
        mx, my = (M_P, M_N) if rng.random() < 0.5 else (M_P, M_P)
        qx, qt, Tx, Tt, plab = oracle.elastic(px, mx, pt, my, rng.random() * 6, rng.random(), rng.random())
        Ein = math.hypot(np.linalg.norm(px), mx) + math.hypot(np.linalg.norm(pt), my)
        Eout = Tx + Tt + mx + my
        assert Eout == pytest.approx(Ein, rel=1e-12)
        assert np.allclose(qx + qt, px + pt, atol=1e-9)
        assert Tx == pytest.approx(math.hypot(np.linalg.norm(qx), mx) - mx, abs=1e-9)
        # p_lab: momentum of x in the rest frame of y, an invariant
        Ex, Ey = math.hypot(np.linalg.norm(px), mx), math.hypot(np.linalg.norm(pt), my)
        dotp = Ex * Ey - px @ pt
        assert plab == pytest.approx(math.sqrt(dotp ** 2 - (mx * my) ** 2) / my, rel=1e-10)


def test_isotropic_elastic_recoil_is_uniform():
    # equal masses, target at rest, isotropic CM: T of the recoil is uniform on [0, T]
    rng = np.random.default_rng(4)
    T = 150.0
    p = math.sqrt(T * T + 2 * T * M_P)
    Tt = np.array([oracle.elastic([0, 0, p], M_P, [0, 0, 0], M_P, 0.0, *rng.random(2))[3] for _ in range(20000)])
    assert stats.kstest(Tt / T, "uniform").pvalue > 1e-3
    assert Tt.min() >= 0 and Tt.max() <= T


@pytest.mark.parametrize("b", [0.5, 3.0, 8.0])
def test_angular_distribution_truncated_exponential(b):
    # d sigma/dt ~ exp(b t): 1 - cos(theta*) has density ~ exp(-k y) on [0, 2], k = 2 b p*^2
    rng = np.random.default_rng(int(b * 10))
    T = 200.0
    p = math.sqrt(T * T + 2 * T * M_P)
    s = 2 * M_P * M_P + 2 * M_P * (T + M_P)
    pstar2 = s / 4 - M_P * M_P
    k = 2 * b * pstar2 / 1e6
    y = []
    for _ in range(20000):
        _, qt, _, Tt, _ = oracle.elastic([0, 0, p], M_P, [0, 0, 0], M_P, b, *rng.random(2))
        y.append(M_P * Tt / pstar2)   # -t = 2 m T_recoil = 2 p*^2 (1 - cos)
    y = np.array(y)
    cdf = lambda v: (1 - np.exp(-k * v)) / (1 - np.exp(-2 * k))
    assert stats.kstest(y, cdf).pvalue > 1e-3


# ------------------------------------------------------------ flight (Sec. 2.3)
FREE = dict(uniform_density=1, zero_fermi=1, zero_binding=1, no_pauli=1,
            no_evaporation=1, stop_after_first=1)


def test_transparency_closed_form():
    sig = 40.0
    n = 60000
    out = oracle.run([(16, 8)], np.full(n, 150.0), seed=21, const_sigma_mb=sig, **FREE)
    nu = oracle.nucleus(16, 8, uniform_density=1)
    rho = 16 / (4 / 3 * math.pi * nu.R ** 3)
    x = 2 * rho * sig * 0.1 * nu.R
    P = 2 * (1 - (1 + x) * math.exp(-x)) / x ** 2
    retries = int(out.results["n_retry"].sum())
    passes = n + retries
    z = (retries - P * passes) / math.sqrt(passes * P * (1 - P))
    assert abs(z) < 4.0, (retries / passes, P)


def test_first_collision_depth_exponential():
    sig = 30.0
    out = oracle.run([(16, 8)], np.full(30000, 150.0), seed=22, const_sigma_mb=sig, fixed_b=0.0, **FREE)
    nu = oracle.nucleus(16, 8, uniform_density=1)
    lam = 16 / (4 / 3 * math.pi * nu.R ** 3) * sig * 0.1
    depth = out.results["first_z"] + nu.R
    L = 2 * nu.R
    cdf = lambda v: (1 - np.exp(-lam * v)) / (1 - np.exp(-lam * L))
    assert depth.min() >= -1e-9 and depth.max() <= L + 1e-9
    assert stats.kstest(depth, cdf).pvalue > 1e-3


# -------------------------------------------------------- refraction (Sec. 2.3)
def test_refraction_cases():
    n = np.array([0.0, 0.0, 1.0])
    # normal incidence transmits and keeps its direction
    ok, d = oracle.refract([0, 0, 1.0], n, 40.0, 10.0, M_P)
    assert ok and np.allclose(d, [0, 0, 1])
    ok, d = oracle.refract([0, 0, -1.0], n, 10.0, 40.0, M_P)
    assert ok and np.allclose(d, [0, 0, -1])
    rng = np.random.default_rng(9)
    for _ in range(2000):
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        Tf, Tt = rng.uniform(1, 300), rng.uniform(0.5, 300)
        pf = math.sqrt(Tf * Tf + 2 * Tf * M_N)
        pt_ = math.sqrt(Tt * Tt + 2 * Tt * M_N)
        ok, d = oracle.refract(v, n, Tf, Tt, M_N)
        assert np.linalg.norm(d) == pytest.approx(1.0, abs=1e-12)
        tang_in = pf * v[:2]
        if ok:
            # tangential momentum conserved (Snell), normal direction kept
            assert np.allclose(pt_ * d[:2], tang_in, atol=1e-9 * pf)
            assert np.sign(d[2]) == np.sign(v[2])
        else:
            # only when the tangential momentum exceeds the far-side momentum
            assert np.linalg.norm(tang_in) >= pt_ - 1e-9
            assert np.allclose(d[:2], v[:2]) and d[2] == pytest.approx(-v[2])


def test_refraction_critical_angle():
    Tf, Tt = 60.0, 20.0
    pf = math.sqrt(Tf * Tf + 2 * Tf * M_P)
    pt_ = math.sqrt(Tt * Tt + 2 * Tt * M_P)
    sc = pt_ / pf
    for s, want in ((sc * (1 - 1e-9), True), (sc * (1 + 1e-9), False)):
        v = [s, 0.0, math.sqrt(1 - s * s)]
        ok, _ = oracle.refract(v, [0, 0, 1.0], Tf, Tt, M_P)
        assert ok == want


# ---------------------------------------------------------- whole events (Sec. 2)
@pytest.mark.parametrize("target,T", [((16, 8), 200.0), ((40, 20), 200.0), ((12, 6), 70.0), ((56, 26), 250.0)])
def test_event_ledgers(target, T):
    n = 4000
    T0 = np.full(n, T)
    out = oracle.run([target], T0, seed=5)
    ev = ledger.from_oracle(out, [target], T0)
    s = ledger.check(ev, tol_E=1e-7, tol_p=1e-7)
    ledger.assert_clean(s)
    # cutoff (Sec. 2.3): escaping cascade protons carry at least E_C, neutrons >= 0
    nu = oracle.nucleus(*target)
    sec = out.secondaries
    c0 = sec["stage"] == 0
    assert np.all(sec["T"][c0 & (sec["species"] == 1)] >= nu.EC - 1e-9)
    assert np.all(sec["T"][c0 & (sec["species"] == 0)] >= -1e-12)
    assert np.all(out.results["n_coll"] >= 1)
    assert np.all(out.results["flags"] == 0)


def test_mixed_target_ledgers():
    rng = np.random.default_rng(7)
    targets = [(12, 6), (14, 7), (16, 8), (31, 15), (40, 20)]
    n = 5000
    tidx = rng.choice(5, size=n, p=[0.18, 0.03, 0.65, 0.01, 0.13]).astype(np.uint8)
    T0 = rng.uniform(20, 250, n)
    out = oracle.run(targets, T0, seed=9, tidx=tidx)
    ledger.assert_clean(ledger.check(ledger.from_oracle(out, targets, T0, tidx), tol_E=1e-7, tol_p=1e-7))


# ------------------------------------------ Pauli and cutoff (Sec. 2.3, P11)
def test_pauli_and_cutoff_hand_built_collisions():
    # 56Fe has N > Z, so the neutron Fermi energy exceeds the proton one in
    # every shell and a species mix-up changes the decision.  Reading R10:
    # blocked unless BOTH products end strictly above the Fermi energy of
    # their own species in the collision shell.  R11: a product with excess
    # eps = T - E_F below E_B (+ E_C for a proton) is captured.
    nu = oracle.nucleus(56, 26)
    far = 300.0
    for s in (0, 6, 12):
        EF = {0: nu.EF[0][s], 1: nu.EF[1][s]}
        assert EF[0] > EF[1] + 0.1
        for x in (0, 1):
            for y in (0, 1):
                out = lambda Tx, Ty: oracle.collision_outcome(nu, s, x, y, Tx, Ty, 0.0)
                # the moving product below, at and just above its own E_F
                assert out(EF[x] - 1e-6, far)[0] and out(EF[x], far)[0]
                assert not out(np.nextafter(EF[x], np.inf), far)[0]
                # the struck product likewise
                assert out(far, EF[y] - 1e-6)[0] and out(far, EF[y])[0]
                assert not out(far, np.nextafter(EF[y], np.inf))[0]
                # between the two species' Fermi energies: allowed for a
                # proton, blocked for a neutron
                mid = 0.5 * (EF[0] + EF[1])
                assert out(mid, far)[0] == (x == 0)
                assert out(far, mid)[0] == (y == 0)
                # no Pauli test: never blocked
                assert not oracle.collision_outcome(nu, s, x, y, 0.5 * EF[x], 0.5 * EF[y], 0.0, pauli=False)[0]
    # the Fermi energy is the collision shell's: between an inner and an outer
    # shell's E_F the decision flips with the shell
    for sp in (0, 1):
        T = 0.5 * (nu.EF[sp][2] + nu.EF[sp][12])
        assert oracle.collision_outcome(nu, 2, sp, 1 - sp, T, far, 0.0)[0]
        assert not oracle.collision_outcome(nu, 12, sp, 1 - sp, T, far, 0.0)[0]
    # cutoff: captured below E_B (+E_C), tracked from there on; excess energy
    # and hole depth from each product's own species
    s = 4
    EF = {0: nu.EF[0][s], 1: nu.EF[1][s]}
    cut = {0: nu.EB, 1: nu.EB + nu.EC}
    for x in (0, 1):
        y = 1 - x
        for eps, tracked in ((cut[x] - 1e-6, False), (cut[x] + 1e-6, True)):
            b, tx, ty, ex, ey, hole = oracle.collision_outcome(nu, s, x, y, EF[x] + eps, EF[y] + 50.0, 10.0)
            assert not b and tx == tracked and ty
            assert ex == pytest.approx(eps, abs=1e-9) and ey == pytest.approx(50.0, abs=1e-9)
            assert hole == pytest.approx(EF[y] - 10.0, abs=1e-12)
        # the boundary itself, to one ulp of the product's kinetic energy
        T = EF[x] + cut[x]
        while T - EF[x] < cut[x]:
            T = np.nextafter(T, np.inf)
        assert oracle.collision_outcome(nu, s, x, y, T, EF[y] + 50.0, 0.0)[1]
        assert not oracle.collision_outcome(nu, s, x, y, np.nextafter(T, -np.inf), EF[y] + 50.0, 0.0)[1]
        # the struck product's cutoff is its own species'
        b, tx, ty, *_ = oracle.collision_outcome(nu, s, x, y, EF[x] + 50.0, EF[y] + cut[y] - 1e-6, 10.0)
        assert not b and tx and not ty
    # an excess between E_B and E_B + E_C: a proton stays, a neutron leaves
    eps = nu.EB + 0.5 * nu.EC
    assert not oracle.collision_outcome(nu, s, 1, 0, EF[1] + eps, EF[0] + 50, 0.0)[1]
    assert oracle.collision_outcome(nu, s, 0, 1, EF[0] + eps, EF[1] + 50, 0.0)[1]
    # a target above the sea's Fermi energy leaves no hole
    assert oracle.collision_outcome(nu, s, 1, 0, 100.0, 100.0, EF[0] + 1.0)[5] == 0.0


@pytest.mark.parametrize("A,Z,reached", [(4, 2, 0.2), (12, 6, 1e-3)])
def test_sea_occupancy(A, Z, reached):
    # Reading R14: a species can be struck only while one of its nucleons is
    # in the Fermi sea (a strike removes one, a capture returns one), so the
    # occupancy never goes below zero, and at the end of the cascade it equals
    # the residual's N' and Z' (every moving nucleon either escaped or was
    # captured).  On 4He and 12C at 250 MeV a species runs out in a fair share
    # of the events, so the rule is exercised.
    out = oracle.run([(A, Z)], np.full(100000, 250.0), seed=3, n_threads=8, no_evaporation=1)
    r = out.results
    assert r["sea_min"].min() >= 0
    assert np.mean(r["sea_min"] == 0) > reached
    assert np.array_equal(r["sea"][:, 1], r["Z_casc"])
    assert np.array_equal(r["sea"][:, 0], r["A_casc"] - r["Z_casc"])
    assert r["Z_casc"].min() >= 0 and (r["A_casc"] - r["Z_casc"]).min() >= 0


def test_pauli_never_blocks_without_a_fermi_sea():
    out = oracle.run([(16, 8)], np.full(3000, 100.0), seed=4, zero_fermi=1)
    assert out.results["n_pauli"].sum() == 0
    out = oracle.run([(16, 8)], np.full(3000, 100.0), seed=4)
    assert out.results["n_pauli"].sum() > 0


@pytest.mark.parametrize("A,Z", [(16, 8), (40, 20)])
def test_cutoff_bounds_the_escape_energies(A, Z):
    # cutoff (Sec. 2.3): after each collision a product stays in the nucleus unless its
    # excess energy reaches E_B (+ E_C for a proton); the excess is invariant
    # under refraction and an escaping nucleon keeps T = excess - E_B, so
    # cascade neutrons leave with T >= 0 and protons with T >= E_C, and both
    # bounds are reached
    nu = oracle.nucleus(A, Z)
    out = oracle.run([(A, Z)], np.full(100000, 200.0), seed=17, n_threads=8, no_evaporation=1)
    s = out.secondaries
    Tn = s["T"][(s["stage"] == 0) & (s["species"] == 0)]
    Tp = s["T"][(s["stage"] == 0) & (s["species"] == 1)]
    assert Tn.min() >= 0.0 and Tp.min() >= nu.EC - 1e-9
    assert np.sum(Tn < 0.2) > 0 and np.sum(Tp < nu.EC + 0.2) > 0


def test_reaction_cross_section_band():
    # sigma_R = pi R^2 * events / passes; a unit slip (mb vs fm^2) would move it 10x
    out = oracle.run([(16, 8)], np.full(20000, 200.0), seed=8)
    nu = oracle.nucleus(16, 8)
    frac = 20000 / (20000 + out.results["n_retry"].sum())
    sigma_R_mb = math.pi * nu.R ** 2 * frac * 10
    assert 150 < sigma_R_mb < 450


def test_evaporation_cost_grows_with_mass():
    # Sec. 4.2: evaporation work is much larger for 40Ca than for 16O
    o = oracle.run([(16, 8)], np.full(4000, 200.0), seed=3).results
    c = oracle.run([(40, 20)], np.full(4000, 200.0), seed=3).results
    assert c["n_evap"].mean() > 1.5 * o["n_evap"].mean()


def test_determinism_and_thread_independence():
    T0 = np.full(500, 180.0)
    a = oracle.run([(16, 8)], T0, seed=77, n_threads=1)
    b = oracle.run([(16, 8)], T0, seed=77, n_threads=7)
    def same(x, y):
        return all(np.array_equal(x[f], y[f], equal_nan=True) for f in x.dtype.names)

    assert same(a.results, b.results) and same(a.secondaries, b.secondaries)
    # event i depends only on (seed, first_id + i)
    c = oracle.run([(16, 8)], T0[100:200], seed=77, first_id=100)
    assert same(a.results[100:200], c.results)


def test_argument_validation():
    with pytest.raises(ValueError):
        oracle.run([(16, 8)], np.array([19.0]), seed=1)
    with pytest.raises(ValueError):
        oracle.run([(16, 8)], np.array([251.0]), seed=1)
    with pytest.raises(ValueError):
        oracle.run([(16, 16)], np.array([100.0]), seed=1)


# ------------------------------------------------------- evaporation (Sec. 2.4)
@pytest.mark.parametrize("a,U", [(2.0, 0.001), (1.0, 0.3), (2.0, 0.49), (2.0, 0.51), (5.0, 10.0), (7.0, 150.0), (0.125, 3.0)])
def test_width_integral_quadrature(a, U):
    f = lambda x: x * math.exp(2 * math.sqrt(a * max(U - x, 0.0)))
    ref = integrate.quad(f, 0, U, epsabs=0, epsrel=1e-13, limit=200)[0]
    assert oracle.width_integral(a, U) == pytest.approx(ref, rel=1e-9)


@pytest.mark.parametrize("a,U", [(2.0, 0.02), (2.0, 3.0), (6.0, 60.0)])
def test_spectrum_cdf_quadrature(a, U):
    # high-precision quadrature of the defining density x rho(U - x)
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 30
    f = lambda x: x * mp.e ** (2 * mp.sqrt(a * (U - x)))
    tot = mp.quad(f, [0, U])
    for x in np.linspace(0, U, 9):
        ref = float(mp.quad(f, [0, x]) / tot) if x > 0 else 0.0
        assert oracle.spectrum_cdf(a, U, x) == pytest.approx(ref, abs=1e-12)


def test_spectrum_small_a_limit():
    # a -> 0: density ~ x on [0, U], CDF (x/U)^2 (corrections are O(sqrt(a U)))
    for x in (0.1, 0.5, 0.9):
        assert oracle.spectrum_cdf(1e-14, 2.0, 2.0 * x) == pytest.approx(x * x, abs=1e-6)


@pytest.mark.parametrize("a,U", [(2.0, 0.3), (5.0, 25.0)])
def test_spectrum_sampler_histogram(a, U):
    rng = np.random.default_rng(17)
    xs = np.array([oracle.spectrum_sample(a, U, u) for u in rng.random(40000)])
    assert stats.kstest(xs, lambda v: np.array([oracle.spectrum_cdf(a, U, t) for t in np.atleast_1d(v)])).pvalue > 1e-3


def test_emission_thresholds():
    A, Z = 16, 8
    thr = [evap_ref.threshold(A, Z, j) for j in range(6)]
    lowest = min(thr)
    r, s = oracle.evaporate(A, Z, lowest - 1e-6, seed=1)
    assert len(s) == 0 and r["A_f"] == A and r["Ex_f"] == pytest.approx(lowest - 1e-6)
    # window where only one channel is open: only that fragment is emitted first
    order = np.argsort(thr)
    j0, j1 = order[0], order[1]
    E = 0.5 * (thr[j0] + thr[j1])
    for k in range(200):
        r, s = oracle.evaporate(A, Z, E, seed=2, event_id=k)
        assert len(s) >= 1 and s[0]["species"] == j0


def test_evaporation_ledger_at_fixed_excitation():
    for A, Z, E in ((16, 8, 40.0), (40, 20, 120.0), (57, 27, 200.0)):
        P = np.array([30.0, -20.0, 150.0])
        for k in range(50):
            r, s = oracle.evaporate(A, Z, E, P, seed=3, event_id=k)
            m = np.array([oracle.mass(ledger.FRAG_A[j], ledger.FRAG_Z[j]) for j in s["species"]])
            pk = np.sqrt(s["T"] ** 2 + 2 * s["T"] * m)[:, None] * s["u"]
            Ein = math.sqrt(P @ P + (oracle.mass(A, Z) + E) ** 2)
            pf = np.array(r["p_f"])
            Eout = np.sum(s["T"] + m) + math.sqrt(pf @ pf + (oracle.mass(r["A_f"], r["Z_f"]) + r["Ex_f"]) ** 2)
            assert Eout == pytest.approx(Ein, abs=1e-8)
            assert np.allclose(pk.sum(axis=0) + pf, P, atol=1e-8)
            assert r["A_f"] + ledger.FRAG_A[s["species"]].sum() == A


def test_evaporation_batch_checks_catch_mistakes():
    # the per-nucleus checks applied to the GPU's evaporation-only output hold
    # on the oracle's, and each catches a mistake planted in that output
    rng = np.random.default_rng(5)
    n = 2000
    A = rng.integers(5, 58, n)
    Z = np.clip(A // 2 + rng.integers(-2, 3, n), 1, np.minimum(A - 1, 27))
    Ex = rng.uniform(0.0, 200.0, n)
    P = rng.normal(size=(n, 3)) * 200.0
    ev = ledger.evaporate_oracle(A, Z, Ex, P, seed=3)
    ledger.assert_clean(ledger.check_evaporation(ev, P, tol_E=1e-8, tol_p=1e-8))
    k = int(np.argmax(ev.sec_T))
    bad = dataclasses.replace(ev, sec_T=ev.sec_T.copy())
    bad.sec_T[k] += 0.01
    assert ledger.check_evaporation(bad, P)["bad_E2"] == 1
    bad = dataclasses.replace(ev, sec_u=ev.sec_u.copy())
    bad.sec_u[k] *= -1.0
    r = ledger.check_evaporation(bad, P)
    assert r["bad_P"] == 1 and r["bad_E2"] == 0
    keep = np.arange(ev.sec_event.size) != k
    fields = ("sec_event", "sec_species", "sec_stage", "sec_T", "sec_u")
    bad = dataclasses.replace(ev, **{f: getattr(ev, f)[keep] for f in fields})
    r = ledger.check_evaporation(bad, P)
    assert r["bad_A"] == 1 and r["bad_nsec"] == 1 and r["bad_E2"] == 1
    bad = dataclasses.replace(ev, Ex_f=ev.Ex_f + 30.0)
    assert ledger.check_evaporation(bad, P)["bad_threshold"] > 0


def test_channel_branching_matches_widths():
    # first-step channel frequencies follow Gamma_j / sum Gamma (multinomial chi-square)
    A, Z, E = 40, 20, 60.0
    n = 6000
    first = np.array([oracle.evaporate(A, Z, E, seed=4, event_id=k)[1][0]["species"] for k in range(n)])
    w = evap_ref.branching(A, Z, E)
    obs = np.bincount(first, minlength=6)
    use = w * n >= 5
    exp = w[use] * n
    chi2 = np.sum((obs[use] - exp) ** 2 / exp) + 0.0
    assert obs[~use].sum() <= max(5, 3 * w[~use].sum() * n + 3)
    assert stats.chi2.sf(chi2, use.sum() - 1) > 1e-3
