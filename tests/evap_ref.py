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


def branching(A: int, Z: int, E: float) -> np.ndarray:
    """Gamma_j / sum Gamma at excitation E: Gamma_j = g_j m_j R_j^2 I(a_d, U_j),
    I(a, U) = int_0^U x exp(2 sqrt(a (U - x))) dx, a_d = A_d / 8 MeV^-1."""
    w = []
    for j in range(6):
        a = int(ledger.FRAG_A[j])
        Ad = A - a
        U = E - threshold(A, Z, j)
        if not U > 0:
            w.append(0.0)
            continue
        Rj = 1.5 * Ad ** (1 / 3) if j <= 1 else 1.5 * (Ad ** (1 / 3) + a ** (1 / 3))
        aa = Ad / 8.0
        I = integrate.quad(lambda x: x * math.exp(2 * math.sqrt(aa * max(U - x, 0))), 0, U, epsrel=1e-12)[0]
        w.append(ledger.FRAG_G[j] * oracle.mass(a, int(ledger.FRAG_Z[j])) * Rj * Rj * I)
    w = np.array(w)
    return w / w.sum()
