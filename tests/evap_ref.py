"""Reference quantities of the evaporation step (Sec. 2.4, Weisskopf-Ewing
reading) computed independently of both implementations: emission thresholds
from the float64 mass formula, and first-step branching ratios from the width
formula with its energy integral done by numerical quadrature."""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

import ledger
import oracle


def threshold(A: int, Z: int, j: int) -> float:
    """S_j + V_j of channel j from (A, Z); +inf when the daughter does not exist."""
    a, z = int(ledger.FRAG_A[j]), int(ledger.FRAG_Z[j])
    Ad, Zd = A - a, Z - z
    if Ad < 1 or Zd < 0 or Zd > Ad:
        return math.inf
    Q = oracle.mass(Ad, Zd) + oracle.mass(a, z) - oracle.mass(A, Z)
    V = ledger.E2_COULOMB * z * Zd / (1.5 * (Ad ** (1 / 3) + a ** (1 / 3))) if z else 0.0
    return Q + V


def photon_weight(A: int, Z: int, E: float) -> float:
    """The photon channel's weight in the particle widths' units (reading
    R19): (s0 / pi) int_0^E e^3 exp(2 sqrt(a (E - e))) de, a = A / 8,
    s0 = 12 N Z / (A E_G^2) fm^2/MeV, E_G = 31.2 A^-1/3 + 20.6 A^-1/6 MeV;
    0 at or below 0.1 MeV."""
    if not E > ledger.PHOTON_MIN_EXCITATION:
        return 0.0
    EG = 31.2 * A ** (-1 / 3) + 20.6 * A ** (-1 / 6)
    s0 = 12.0 * (A - Z) * Z / (A * EG * EG)
    a = A / 8.0
    J = integrate.quad(lambda x: x ** 3 * math.exp(2 * math.sqrt(a * max(E - x, 0))), 0, E, epsrel=1e-12)[0]
    return s0 / math.pi * J


def branching(A: int, Z: int, E: float, photons: bool = False, heavy: bool = False) -> np.ndarray:
    """Gamma_j / sum Gamma at excitation E: Gamma_j = g_j m_j R_j^2 I(a_d, U_j),
    I(a, U) = int_0^U x exp(2 sqrt(a (U - x))) dx, a_d = A_d / 8 MeV^-1; with
    photons, the photon channel's weight at index 6; with heavy, the heavier
    fragments' channels 7-26 (the same width form).  Length 6, 7 with
    photons, 27 with heavy."""
    chans = list(range(6)) + (list(ledger.HEAVY) if heavy else [])
    w = np.zeros(27 if heavy else (7 if photons else 6))
    for j in chans:
        a = int(ledger.FRAG_A[j])
        Ad = A - a
        U = E - threshold(A, Z, j)
        if not U > 0:
            continue
        Rj = 1.5 * Ad ** (1 / 3) if j <= 1 else 1.5 * (Ad ** (1 / 3) + a ** (1 / 3))
        aa = Ad / 8.0
        I = integrate.quad(lambda x: x * math.exp(2 * math.sqrt(aa * max(U - x, 0))), 0, U, epsrel=1e-12)[0]
        w[j] = ledger.FRAG_G[j] * oracle.mass(a, int(ledger.FRAG_Z[j])) * Rj * Rj * I
    if photons:
        w[6] = photon_weight(A, Z, E)
    return w / w.sum()
