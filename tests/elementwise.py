"""Element-wise comparison of GPU and oracle events generated from the same
random streams (replay).

Both sides draw event i's numbers from the same Philox stream in the same
order, so an event whose discrete history is the same on both sides (the
same residual A and Z, the same number of collisions and transparent passes,
the same secondaries in the same emission order, species and stage) took the
same branches everywhere; its continuous outputs then differ only by FP32
rounding of the same arithmetic.  For those events every continuous output is
compared value by value: Ex_casc, Ex_f, the residual's momentum, and each
secondary's T and direction, records matched by emission order.

Records of one event keep their emission order in the output arrays on both
sides (the GPU writer reserves slots in emission order), so a stable sort by
event gives each event's records in order.
"""
from __future__ import annotations

import numpy as np


def _in_order(ev):
    order = np.argsort(ev.sec_event, kind="stable")
    bounds = np.searchsorted(ev.sec_event[order], np.arange(ev.n + 1))
    return order, bounds


def same_history(g, o, g_counts=None, o_counts=None):
    """Mask of events whose discrete history agrees.  g_counts / o_counts:
    optional (n, k) integer arrays (e.g. collisions and transparent passes)
    that must agree too."""
    n = g.n
    assert o.n == n
    og, bg = _in_order(g)
    oo, bo = _in_order(o)
    ng = np.diff(bg)
    no = np.diff(bo)
    m = (g.A_f == o.A_f) & (g.Z_f == o.Z_f) & (ng == no)
    if g_counts is not None:
        m &= np.all(np.asarray(g_counts) == np.asarray(o_counts), axis=1)
    code_g = (g.sec_stage[og] * 32 + g.sec_species[og]).astype(np.int64)
    code_o = (o.sec_stage[oo] * 32 + o.sec_species[oo]).astype(np.int64)
    for i in np.flatnonzero(m):
        if not np.array_equal(code_g[bg[i]:bg[i + 1]], code_o[bo[i]:bo[i + 1]]):
            m[i] = False
    return m


def deviations(g, o, mask):
    """Absolute differences of the continuous outputs over the events of
    `mask` and their records, in emission order: dict of arrays."""
    og, bg = _in_order(g)
    oo, bo = _in_order(o)
    ev = np.flatnonzero(mask)
    cnt = (bg[ev + 1] - bg[ev]).astype(np.int64)
    # record positions of the matched events, in event then emission order
    rel = np.arange(int(cnt.sum())) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    rg = og[np.repeat(bg[ev], cnt) + rel]
    ro = oo[np.repeat(bo[ev], cnt) + rel]
    return dict(
        Ex_casc=np.abs(g.Ex_casc[ev] - o.Ex_casc[ev]),
        Ex_f=np.abs(g.Ex_f[ev] - o.Ex_f[ev]),
        p_f=np.abs(g.p_f[ev] - o.p_f[ev]).max(axis=1),
        sec_T=np.abs(g.sec_T[rg] - o.sec_T[ro]),
        sec_T_rel=np.abs(g.sec_T[rg] - o.sec_T[ro]) / np.maximum(o.sec_T[ro], 1.0),
        sec_u=np.abs(g.sec_u[rg] - o.sec_u[ro]).max(axis=1),
        records=np.array([cnt.sum()]),
    )


def summary(dev):
    """(max, 99.9th percentile) of every deviation array, for printing."""
    out = {}
    for k, v in dev.items():
        if k == "records" or v.size == 0:
            continue
        out[k] = (float(v.max()), float(np.quantile(v, 0.999)))
    return out


def event_deviation(g, o, mask):
    """Per event, the largest normalised difference of its continuous
    outputs (NaN outside `mask`): |dEx_casc| / max(Ex_casc, 1 MeV),
    |dEx_f| / max(Ex_f, 1 MeV), max_k |dp_f,k| / max(|p_f|, 10 MeV/c), and
    over its records |dT| / max(T, 1 MeV) and max_k |du_k|."""
    n = g.n
    D = np.full(n, np.nan)
    ev = np.flatnonzero(mask)
    if ev.size == 0:
        return D
    og, bg = _in_order(g)
    oo, bo = _in_order(o)
    cnt = (bg[ev + 1] - bg[ev]).astype(np.int64)
    rel = np.arange(int(cnt.sum())) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    rg = og[np.repeat(bg[ev], cnt) + rel]
    ro = oo[np.repeat(bo[ev], cnt) + rel]
    d = np.maximum(np.abs(g.Ex_casc[ev] - o.Ex_casc[ev]) / np.maximum(o.Ex_casc[ev], 1.0),
                   np.abs(g.Ex_f[ev] - o.Ex_f[ev]) / np.maximum(o.Ex_f[ev], 1.0))
    d = np.maximum(d, np.abs(g.p_f[ev] - o.p_f[ev]).max(axis=1) / np.maximum(np.linalg.norm(o.p_f[ev], axis=1), 10.0))
    rec = np.maximum(np.abs(g.sec_T[rg] - o.sec_T[ro]) / np.maximum(o.sec_T[ro], 1.0),
                     np.abs(g.sec_u[rg] - o.sec_u[ro]).max(axis=1))
    per = np.zeros(ev.size)
    np.maximum.at(per, np.repeat(np.arange(ev.size), cnt), rec)
    D[ev] = np.maximum(d, per)
    return D


# First-order bound of the element-wise comparison.  An output of an event
# depends on at most about 2^14 dependent FP32 operations (the oracle counts
# ~300 uniforms, ~100 flight segments and ~50 collisions per 16O event at
# 200 MeV, each step a few tens of operations), so rounding moves it by at
# most N_U = 2^14 x 2^-24 (about 1e-3) times the event's amplification.  The
# amplification kappa of each event is measured on the oracle itself: the
# same event with its input moved by one FP32 ulp (relative size delta) moves
# its outputs by D_pert, kappa = D_pert / delta.  An event whose discrete
# history changes under that one-ulp move sits on a discontinuity of the
# model (kappa infinite); such events must stay rare.
N_U = 2.0 ** 14 * 2.0 ** -24
# Events over their bound: none allowed (MAX_OVER_BOUND is a fraction of the
# matched events), and none beyond D_CAP in any case.
MAX_OVER_BOUND = 0.0
D_CAP = 0.1


def one_ulp_up(x, top=np.inf):
    """x (FP32 values) moved by one FP32 ulp, up unless that passes `top`
    (then down), as float64, and the relative size of the move."""
    x32 = np.asarray(x, dtype=np.float32)
    up = np.nextafter(x32, np.float32(np.inf))
    down = np.nextafter(x32, np.float32(-np.inf))
    moved = np.where(up.astype(np.float64) <= top, up, down).astype(np.float64)
    x64 = x32.astype(np.float64)
    return moved, np.abs(moved - x64) / np.maximum(np.abs(x64), np.finfo(np.float64).tiny)
MIN_MATCHED = 0.9
MAX_DISCONTINUOUS = 0.01


def assert_replay_close(g, o, g_res, o_res, label, g_hist=None, o_pert=None, delta=None):
    """Replay gate.  The events whose discrete history agrees (A_f, Z_f, the
    secondaries' species and stages in emission order, collision and
    transparent-pass counts, and, given g_hist, the GPU's history words
    against the oracle's draw and flight-segment counts and shell
    fingerprint) are at least
    MIN_MATCHED of the batch.  Given o_pert = (events, results) of the oracle
    on the same events with the input moved by one FP32 ulp and delta the
    per-event relative size of that move, the matched events satisfy
    D_gpu <= N_U max(1, kappa) but for at most MAX_OVER_BOUND of them, which
    stay within D_CAP; the events with infinite kappa are at most
    MAX_DISCONTINUOUS of the batch.  Prints the quantiles of D_gpu and the
    events over their bound."""
    def counts(res, hist=None, oracle_side=False):
        cols = [res["n_coll"], res["n_retry"]]
        if hist is not None:
            cols += [hist[:, 0], hist[:, 1], hist[:, 2]]
        elif oracle_side:
            cols += [res["n_draw"], res["n_seg"], res["tent_shells"]]
        return np.stack([np.asarray(c, np.int64) for c in cols], 1)

    with_hist = g_hist is not None
    m = same_history(g, o, counts(g_res, g_hist), counts(o_res, oracle_side=with_hist))
    D = event_deviation(g, o, m)
    Dm = D[m]
    msg = "%s: same history %.4f of %d events; D_gpu median %.1e, 99%% %.1e, 99.9%% %.1e, max %.1e" % (
        label, m.mean(), g.n, np.median(Dm), np.quantile(Dm, 0.99), np.quantile(Dm, 0.999), Dm.max())
    assert m.mean() > MIN_MATCHED, (label, m.mean())
    if o_pert is None:
        print(msg)
        return
    op, op_res = o_pert
    mp = same_history(o, op, counts(o_res, oracle_side=True), counts(op_res, oracle_side=True))
    Dp = event_deviation(o, op, mp)
    kappa = np.where(mp, Dp / np.asarray(delta, np.float64), np.inf)
    bound = N_U * np.maximum(1.0, kappa)
    over = m & (D > bound)
    beyond = m & (D > N_U)
    print(msg + "; above N_U: %d events (kappa of those: min %.1e); discontinuous under one ulp: %.4f; "
          "worst D_gpu / bound %.2e; over the bound: %d events %s" % (
              beyond.sum(), kappa[beyond].min() if beyond.any() else np.nan, np.mean(~mp),
              np.nanmax(np.where(m, D / bound, np.nan)), over.sum(),
              [(int(e), "%.1e" % D[e], "%.1f" % kappa[e]) for e in np.flatnonzero(over)[:8]]))
    assert over.sum() <= MAX_OVER_BOUND * m.sum(), (label, np.flatnonzero(over)[:10], D[over][:10])
    assert not (over & (D > D_CAP)).any(), (label, np.flatnonzero(over & (D > D_CAP)))
    assert np.mean(~mp) <= MAX_DISCONTINUOUS, (label, np.mean(~mp))
