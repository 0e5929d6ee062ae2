"""Per-event conservation checks in float64, shared by the oracle and GPU tests.

Given one batch of events (target, incident energy, residual record and the
emitted secondaries) it checks, event by event:

* integers: A_f + sum a_k = A + 1, Z_f + sum z_k = Z + 1, records = n_sec;
* E1 (cascade, Sec. 2.3): T0 + E_B = sum_stage0 (T_k + E_B) + E*_casc;
* E2 (evaporation, Sec. 2.4): the total energy of the post-cascade nucleus
  equals the evaporated particles' total energies plus the final nucleus';
* P: p0 z = sum_all p_k + p_f;
* E* >= 0, T >= 0, |u| = 1, and E*_f below every emission threshold.

Masses come from the oracle's float64 mass formula (the model's masses).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import oracle

# species 0-5: n, p, d, t, 3He, alpha; 6: photon (massless, no nucleons; the
# optional photon channel); 7-26: the optional heavier fragments, the stable
# isotopes of Li to Mg (6Li 7Li 9Be 10B 11B 12C 13C 14N 15N 16O 17O 18O 19F
# 20Ne 21Ne 22Ne 23Na 24Mg 25Mg 26Mg) with their ground-state 2s + 1
FRAG_A = np.array([1, 1, 2, 3, 3, 4, 0,
                   6, 7, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26])
FRAG_Z = np.array([0, 1, 1, 1, 2, 2, 0,
                   3, 3, 4, 5, 5, 6, 6, 7, 7, 8, 8, 8, 9, 10, 10, 10, 11, 12, 12, 12])
FRAG_G = np.array([2, 2, 3, 2, 2, 1, 2,
                   3, 4, 4, 7, 4, 1, 2, 3, 2, 1, 6, 1, 2, 1, 4, 1, 4, 1, 6, 1])
PHOTON = 6
HEAVY = np.arange(7, 27)
PHOTON_MIN_EXCITATION = 0.1  # MeV: the photon channel is open above this
E2_COULOMB = 1.44
M_PROTON = 938.272088

_AMAX = 260
_MASS = None
_BIND = None


def mass_table():
    global _MASS, _BIND
    if _MASS is None:
        M = np.zeros((_AMAX + 1, _AMAX + 1))
        B = np.zeros((_AMAX + 1, _AMAX + 1))
        for A in range(1, _AMAX + 1):
            for Z in range(0, A + 1):
                M[A, Z] = oracle.mass(A, Z)
                B[A, Z] = oracle.binding(A, Z)
        _MASS, _BIND = M, B
    return _MASS, _BIND


@dataclass
class Events:
    A: np.ndarray
    Z: np.ndarray
    T0: np.ndarray
    A_f: np.ndarray
    Z_f: np.ndarray
    Ex_casc: np.ndarray
    Ex_f: np.ndarray
    p_f: np.ndarray          # (n, 3)
    n_sec: np.ndarray
    flags: np.ndarray
    sec_event: np.ndarray    # (m,) index of the event in this batch
    sec_species: np.ndarray
    sec_stage: np.ndarray
    sec_T: np.ndarray
    sec_u: np.ndarray        # (m, 3)

    @property
    def n(self) -> int:
        return int(self.A.shape[0])


def from_oracle(out, targets, T0, tidx=None) -> Events:
    AZ = np.array(targets, dtype=np.int64).reshape(-1, 2)
    ti = np.zeros(len(T0), dtype=np.int64) if tidx is None else np.asarray(tidx, dtype=np.int64)
    r, s = out.results, out.secondaries
    return Events(
        A=AZ[ti, 0], Z=AZ[ti, 1], T0=np.asarray(T0, dtype=np.float64),
        A_f=r["A_f"].astype(np.int64), Z_f=r["Z_f"].astype(np.int64),
        Ex_casc=r["Ex_casc"].astype(np.float64), Ex_f=r["Ex_f"].astype(np.float64),
        p_f=np.asarray(r["p_f"], dtype=np.float64), n_sec=r["n_sec"].astype(np.int64),
        flags=r["flags"].astype(np.int64),
        sec_event=s["event"].astype(np.int64), sec_species=s["species"].astype(np.int64),
        sec_stage=s["stage"].astype(np.int64), sec_T=s["T"].astype(np.float64),
        sec_u=np.asarray(s["u"], dtype=np.float64),
    )


def evaporate_oracle(A, Z, Ex, P=None, seed: int = 1, first_id: int = 0, with_results: bool = False,
                     photon_evaporation: int = 0):
    """Evaporation alone of nuclei (A[i], Z[i], Ex[i], P[i]) by the oracle, nucleus
    i on the stream of (seed, first_id + i), as an Events batch (T0 = 0); with
    with_results, also the oracle's result records (draw counts included)."""
    n = len(A)
    P = np.zeros((n, 3)) if P is None else np.asarray(P, dtype=np.float64).reshape(n, 3)
    rows, secs = [], []
    for i in range(n):
        r, s = oracle.evaporate(int(A[i]), int(Z[i]), float(Ex[i]), tuple(P[i]), seed=seed, event_id=first_id + i,
                                photon_evaporation=photon_evaporation)
        r = r.copy()
        r["n_sec"] = len(s)
        rows.append(r)
        s = s.copy()
        s["event"] = i
        secs.append(s)
    r = np.array(rows)
    s = np.concatenate(secs) if secs else np.zeros(0, dtype=oracle.SECONDARY_DTYPE)
    ev = Events(
        A=np.asarray(A, dtype=np.int64), Z=np.asarray(Z, dtype=np.int64), T0=np.zeros(n),
        A_f=r["A_f"].astype(np.int64), Z_f=r["Z_f"].astype(np.int64),
        Ex_casc=np.asarray(Ex, dtype=np.float64), Ex_f=r["Ex_f"].astype(np.float64),
        p_f=np.asarray(r["p_f"], dtype=np.float64), n_sec=r["n_sec"].astype(np.int64),
        flags=r["flags"].astype(np.int64),
        sec_event=s["event"].astype(np.int64), sec_species=s["species"].astype(np.int64),
        sec_stage=s["stage"].astype(np.int64), sec_T=s["T"].astype(np.float64),
        sec_u=np.asarray(s["u"], dtype=np.float64),
    )
    return (ev, r) if with_results else ev



def _sum_by_event(idx, w, n):
    return np.bincount(idx, weights=w, minlength=n)


def check(ev: Events, tol_E: float = 1e-3, tol_p: float = 1e-3, tol_u: float = 1e-5, photons: bool = False,
          heavy: bool = False) -> dict:
    """Return violation counts and worst residuals for every per-event check
    (photons: the photon channel was on, so no event may end above its
    threshold either; heavy: the heavier fragments' channels were on, so
    none of them may be left open, and records of them are allowed)."""
    M, B = mass_table()
    n = ev.n
    e = ev.sec_event
    sp = ev.sec_species
    a_k = FRAG_A[sp]
    z_k = FRAG_Z[sp]
    m_k = M[a_k, z_k]
    T = ev.sec_T
    pmag = np.sqrt(T * T + 2.0 * T * m_k)
    pk = ev.sec_u * pmag[:, None]
    st0 = ev.sec_stage == 0
    st1 = ~st0

    out = {}
    # integers
    cnt = np.bincount(e, minlength=n)
    sumA = _sum_by_event(e, a_k.astype(np.float64), n).round().astype(np.int64)
    sumZ = _sum_by_event(e, z_k.astype(np.float64), n).round().astype(np.int64)
    out["bad_A"] = int(np.sum(ev.A_f + sumA != ev.A + 1))
    out["bad_Z"] = int(np.sum(ev.Z_f + sumZ != ev.Z + 1))
    out["bad_nsec"] = int(np.sum(cnt != ev.n_sec))
    # post-cascade state from the stage-0 records
    n0 = np.bincount(e[st0], minlength=n)
    n0p = np.bincount(e[st0 & (sp == 1)], minlength=n)
    A_c = ev.A + 1 - n0
    Z_c = ev.Z + 1 - n0p
    EB = B[ev.A, ev.Z] / ev.A
    p0 = np.sqrt(ev.T0 ** 2 + 2.0 * ev.T0 * M_PROTON)
    sumT0 = _sum_by_event(e[st0], T[st0], n)
    E1 = ev.T0 + EB - sumT0 - n0 * EB - ev.Ex_casc
    out["max_E1"] = float(np.max(np.abs(E1))) if n else 0.0
    out["bad_E1"] = int(np.sum(np.abs(E1) > tol_E))
    pc = np.zeros((n, 3))
    for c in range(3):
        pc[:, c] = -_sum_by_event(e[st0], pk[st0, c], n)
    pc[:, 2] += p0
    ok_c = A_c >= 1
    Mc = np.where(ok_c, M[np.clip(A_c, 0, None), np.clip(Z_c, 0, None)], 0.0)
    E_before = np.sqrt(np.sum(pc ** 2, axis=1) + (Mc + ev.Ex_casc) ** 2)
    E_evap = _sum_by_event(e[st1], T[st1] + m_k[st1], n)
    Mf = M[np.clip(ev.A_f, 0, None), np.clip(ev.Z_f, 0, None)]
    E_after = np.sqrt(np.sum(ev.p_f ** 2, axis=1) + (Mf + ev.Ex_f) ** 2)
    E2 = np.where(ok_c, E_before - E_evap - E_after, 0.0)
    out["max_E2"] = float(np.max(np.abs(E2))) if n else 0.0
    out["bad_E2"] = int(np.sum(np.abs(E2) > tol_E))
    ptot = np.zeros((n, 3))
    for c in range(3):
        ptot[:, c] = _sum_by_event(e, pk[:, c], n)
    ptot += ev.p_f
    ptot[:, 2] -= p0
    P = np.sqrt(np.sum(ptot ** 2, axis=1))
    out["max_P"] = float(np.max(P)) if n else 0.0
    out["bad_P"] = int(np.sum(P > tol_p))
    out["bad_Ex"] = int(np.sum((ev.Ex_casc < 0) | (ev.Ex_f < 0)))
    out["bad_T"] = int(np.sum(T < 0))
    un = np.sqrt(np.sum(ev.sec_u ** 2, axis=1))
    out["bad_u"] = int(np.sum(np.abs(un - 1.0) > tol_u))
    out["bad_threshold"] = _open_channel_left(ev, B, photons, heavy)
    out["n_events"] = n
    out["n_secondaries"] = int(e.shape[0])
    return out


def _open_channel_left(ev: Events, B, photons: bool = False, heavy: bool = False) -> int:
    """Events whose final nucleus still has an open channel: E*_f >= S_j + V_j
    for some valid channel j (beyond 1e-4 MeV of FP32 slack); with the
    channels off, any record of a photon or heavier fragment counts too."""
    bad_thr = np.zeros(ev.n, dtype=bool)
    Af, Zf = ev.A_f, ev.Z_f
    for j in list(range(6)) + (list(HEAVY) if heavy else []):
        Ad = Af - FRAG_A[j]
        Zd = Zf - FRAG_Z[j]
        valid = (Ad >= 1) & (Zd >= 0) & (Zd <= Ad)
        Adc, Zdc = np.clip(Ad, 1, None), np.clip(Zd, 0, None)
        S = B[np.clip(Af, 0, None), np.clip(Zf, 0, None)] - B[Adc, Zdc] - B[FRAG_A[j], FRAG_Z[j]]
        V = np.where(
            FRAG_Z[j] > 0,
            E2_COULOMB * FRAG_Z[j] * Zdc / (1.5 * (np.cbrt(Adc) + np.cbrt(FRAG_A[j]))),
            0.0,
        )
        bad_thr |= valid & (ev.Ex_f - S - V > 1e-4) & (ev.flags & 4 == 0)
    if photons:
        # the photon channel is open above 0.1 MeV wherever there is dipole
        # strength (N Z > 0)
        has_dipole = (Af - Zf) * Zf > 0
        bad_thr |= (ev.Ex_f > PHOTON_MIN_EXCITATION + 1e-4) & has_dipole & (ev.flags & 4 == 0)
    else:
        bad_thr |= np.bincount(ev.sec_event[ev.sec_species == PHOTON], minlength=ev.n) > 0
    if not heavy:
        bad_thr |= np.bincount(ev.sec_event[ev.sec_species >= 7], minlength=ev.n) > 0
    return int(np.sum(bad_thr))


def check_evaporation(ev: Events, P_in, tol_E: float = 1e-3, tol_p: float = 1e-3, tol_u: float = 1e-5,
                      photons: bool = False, heavy: bool = False) -> dict:
    """Per-nucleus checks of an evaporation-only batch (Sec. 2.4): nucleus i,
    (A, Z) with excitation Ex_casc and lab momentum P_in[i], decays into its
    records (all stage 1) and the final nucleus.

    * integers: A_f + sum a_k = A, Z_f + sum z_k = Z, records = n_sec;
    * energy: sqrt(P^2 + (M(A,Z) + E*)^2) = sum (T_k + m_k) + sqrt(p_f^2 + (M_f + E*_f)^2);
    * momentum: P = sum p_k + p_f;
    * E*_f >= 0, T >= 0, |u| = 1, and no channel left open."""
    M, B = mass_table()
    n = ev.n
    e = ev.sec_event
    sp = ev.sec_species
    a_k = FRAG_A[sp]
    z_k = FRAG_Z[sp]
    m_k = M[a_k, z_k]
    T = ev.sec_T
    pk = ev.sec_u * np.sqrt(T * T + 2.0 * T * m_k)[:, None]
    P_in = np.asarray(P_in, dtype=np.float64).reshape(n, 3)
    out = {}
    cnt = np.bincount(e, minlength=n)
    sumA = _sum_by_event(e, a_k.astype(np.float64), n).round().astype(np.int64)
    sumZ = _sum_by_event(e, z_k.astype(np.float64), n).round().astype(np.int64)
    out["bad_A"] = int(np.sum(ev.A_f + sumA != ev.A))
    out["bad_Z"] = int(np.sum(ev.Z_f + sumZ != ev.Z))
    out["bad_nsec"] = int(np.sum(cnt != ev.n_sec))
    out["bad_stage"] = int(np.sum(ev.sec_stage != 1))
    E_before = np.sqrt(np.sum(P_in ** 2, axis=1) + (M[ev.A, ev.Z] + ev.Ex_casc) ** 2)
    E_evap = _sum_by_event(e, T + m_k, n)
    Mf = M[np.clip(ev.A_f, 0, None), np.clip(ev.Z_f, 0, None)]
    E_after = np.sqrt(np.sum(ev.p_f ** 2, axis=1) + (Mf + ev.Ex_f) ** 2)
    E2 = E_before - E_evap - E_after
    out["max_E2"] = float(np.max(np.abs(E2))) if n else 0.0
    out["bad_E2"] = int(np.sum(np.abs(E2) > tol_E))
    ptot = np.stack([_sum_by_event(e, pk[:, c], n) for c in range(3)], axis=1) + ev.p_f - P_in
    P = np.sqrt(np.sum(ptot ** 2, axis=1))
    out["max_P"] = float(np.max(P)) if n else 0.0
    out["bad_P"] = int(np.sum(P > tol_p))
    out["bad_Ex"] = int(np.sum(ev.Ex_f < 0))
    out["bad_T"] = int(np.sum(T < 0))
    un = np.sqrt(np.sum(ev.sec_u ** 2, axis=1))
    out["bad_u"] = int(np.sum(np.abs(un - 1.0) > tol_u))
    out["bad_threshold"] = _open_channel_left(ev, B, photons, heavy)
    out["n_events"] = n
    out["n_secondaries"] = int(e.shape[0])
    return out


def assert_clean(summary: dict):
    bad = {k: v for k, v in summary.items() if k.startswith("bad_") and v}
    assert not bad, "ledger violations: %r (summary %r)" % (bad, summary)
