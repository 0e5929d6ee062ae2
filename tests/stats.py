"""Two-sample statistics for comparing two event samples drawn with independent
seeds: secondary-particle histograms (per-event correlated counts) and
residual-nucleus (A, Z) tables.

Histogram test: every event contributes a vector w_e of counts over the bins.
With N i.i.d. events the per-event mean h = sum_e w_e / N has covariance
C / N, C = E[w w^T] - E[w] E[w]^T, estimated from the sample.  For two samples
the statistic d^T (C1/N1 + C2/N2)^-1 d, d = h1 - h2, is chi-square with as
many degrees of freedom as bins used (bins with too few entries are dropped).
Counts of one event in different bins are correlated, which is why the full
covariance and not a per-bin Poisson variance is used.

Table test: one residual per event, so the (A, Z) table is multinomial; the
usual 2 x K contingency chi-square, with cells of small expected count merged.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps
from scipy import stats


def event_hist(event_idx, values, n_events, bins, lo, hi):
    """Sparse (n_events x bins) matrix of per-event counts."""
    v = np.asarray(values, dtype=np.float64)
    b = np.floor((v - lo) / (hi - lo) * bins).astype(np.int64)
    b = np.clip(b, 0, bins - 1)
    inr = (v >= lo) & (v <= hi)
    e = np.asarray(event_idx, dtype=np.int64)[inr]
    data = np.ones(e.shape[0])
    return sps.csr_matrix((data, (e, b[inr])), shape=(n_events, bins))


def chi2_hist(W1, W2, min_count: int = 20):
    """Two-sample chi-square of per-event count histograms; returns (chi2, dof, p)."""
    N1, N2 = W1.shape[0], W2.shape[0]
    s1 = np.asarray(W1.sum(axis=0)).ravel()
    s2 = np.asarray(W2.sum(axis=0)).ravel()
    use = (s1 + s2) >= min_count
    if not use.any():
        return 0.0, 0, 1.0
    W1u, W2u = W1[:, use], W2[:, use]
    h1, h2 = s1[use] / N1, s2[use] / N2
    C1 = np.asarray((W1u.T @ W1u).todense()) / N1 - np.outer(h1, h1)
    C2 = np.asarray((W2u.T @ W2u).todense()) / N2 - np.outer(h2, h2)
    S = C1 / N1 + C2 / N2
    d = h1 - h2
    # pseudo-inverse guards against exactly degenerate bins
    x = np.linalg.lstsq(S, d, rcond=1e-12)[0]
    chi2 = float(d @ x)
    dof = int(np.linalg.matrix_rank(S, tol=1e-12 * np.abs(S).max()))
    return chi2, dof, float(stats.chi2.sf(chi2, dof))


def chi2_table(keys1, keys2, min_expected: float = 5.0):
    """Two-sample chi-square of categorical outcomes (e.g. A*1000+Z)."""
    k1 = np.asarray(keys1)
    k2 = np.asarray(keys2)
    cats = np.union1d(k1, k2)
    c1 = np.array([np.sum(k1 == c) for c in cats], dtype=np.float64) if cats.size < 50 else None
    if c1 is None:
        idx1 = np.searchsorted(cats, k1)
        idx2 = np.searchsorted(cats, k2)
        c1 = np.bincount(idx1, minlength=cats.size).astype(np.float64)
        c2 = np.bincount(idx2, minlength=cats.size).astype(np.float64)
    else:
        c2 = np.array([np.sum(k2 == c) for c in cats], dtype=np.float64)
    return chi2_counts(c1, c2, min_expected)


def chi2_counts(c1, c2, min_expected: float = 5.0):
    """Two-sample chi-square of two count vectors over the same categories;
    cells with an expected count below min_expected are merged into one."""
    c1 = np.asarray(c1, dtype=np.float64)
    c2 = np.asarray(c2, dtype=np.float64)
    N1, N2 = c1.sum(), c2.sum()
    tot = c1 + c2
    e1 = tot * N1 / (N1 + N2)
    e2 = tot * N2 / (N1 + N2)
    small = (e1 < min_expected) | (e2 < min_expected)
    rows1 = list(c1[~small])
    rows2 = list(c2[~small])
    if small.any():
        rows1.append(c1[small].sum())
        rows2.append(c2[small].sum())
    table = np.array([rows1, rows2])
    table = table[:, table.sum(axis=0) > 0]
    if table.shape[1] < 2:
        return 0.0, 0, 1.0
    chi2, p, dof, _ = stats.chi2_contingency(table, correction=False)
    return float(chi2), int(dof), float(p)


def compare_samples(ev1, ev2, T_max: float, bins: int = 100):
    """All parity statistics between two Events samples: n and p kinetic-energy
    and cos(theta) histograms (both stages) and the final (A, Z) table."""
    res = {}
    for sp, name in ((0, "n"), (1, "p")):
        m1 = ev1.sec_species == sp
        m2 = ev2.sec_species == sp
        W1 = event_hist(ev1.sec_event[m1], ev1.sec_T[m1], ev1.n, bins, 0.0, T_max)
        W2 = event_hist(ev2.sec_event[m2], ev2.sec_T[m2], ev2.n, bins, 0.0, T_max)
        res[name + "_T"] = chi2_hist(W1, W2)
        W1 = event_hist(ev1.sec_event[m1], ev1.sec_u[m1, 2], ev1.n, bins, -1.0, 1.0)
        W2 = event_hist(ev2.sec_event[m2], ev2.sec_u[m2, 2], ev2.n, bins, -1.0, 1.0)
        res[name + "_cos"] = chi2_hist(W1, W2)
    k1 = ev1.A_f * 1000 + ev1.Z_f
    k2 = ev2.A_f * 1000 + ev2.Z_f
    res["AZ"] = chi2_table(k1, k2)
    return res
