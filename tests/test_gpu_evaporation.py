"""Evaporation alone on the GPU (inc_evaporate_dev; Sec. 2.4, Weisskopf-Ewing
reading) against the pins of the evaporation step and against the oracle.

* every nucleus passes the float64 checks: exact integers, energy within
  1e-3 MeV, momentum within 1e-3 MeV/c, no channel left open;
* thresholds: below the lowest threshold nothing is emitted and the nucleus
  is returned untouched; where one channel is open only that fragment comes
  first;
* branching: first-emission frequencies at fixed (A, Z, E*) follow
  Gamma_j / sum Gamma from the width formula by quadrature;
* spectrum: where exactly one neutron can be emitted, x = U - E*_f follows the
  closed-form distribution x exp(2 sqrt(a (U - x))) (equiprobable bins from the
  oracle's independent bisection sampler);
* replay: with the same stream the oracle reaches the same integer outcome,
  fragments in emission order, for almost every nucleus;
* distributions vs the oracle with independent seeds (two-sample chi-square);
* invalid nuclei are flagged, the rest of the batch is unaffected.
"""
import numpy as np
import pytest
from scipy.stats import chi2 as chi2_dist

import evap_ref
import elementwise
import ledger
import oracle
import stats

pytestmark = pytest.mark.gpu

TARGETS = [(16, 8), (40, 20), (56, 26)]  # tables cover A <= 57, Z <= 27
FLAG_RANGE = 0x8000


@pytest.fixture(scope="module")
def ctx():
    import paper_1309_7963_amd as inc

    c = inc.Context(TARGETS)
    yield c
    c.close()


@pytest.fixture(scope="module", params=[0, 1], ids=["ieee", "fast_math"])
def any_ctx(request):
    """A context of the default build, then one of the fast-math build (the
    statistical pins must hold for both, Sec. 4.2)."""
    import paper_1309_7963_amd as inc

    c = inc.Context(TARGETS, fast_math=request.param)
    yield c
    c.close()


def _inputs(A, Z, Ex, P):
    """The float32/int16 inputs as the device sees them, back in float64."""
    n = len(Ex)
    A = np.asarray(A, dtype=np.int16)
    Z = np.asarray(Z, dtype=np.int16)
    Ex = np.asarray(Ex, dtype=np.float32)
    P = None if P is None else np.asarray(P, dtype=np.float32).reshape(n, 3)
    return A, Z, Ex, P


def _run(ctx, A, Z, Ex, P=None, seed=1, first_id=0, capacity=None, raw=False, history=None):
    """history: a dict that receives the per-nucleus history words (n x 2)."""
    import torch
    import paper_1309_7963_amd as inc

    A, Z, Ex, P = _inputs(A, Z, Ex, P)
    n = len(Ex)
    out = None
    if history is not None:
        out = inc.DeviceOutput.allocate(n, capacity or 8 * n + 4096, "cuda", history=True)
    out = ctx.evaporate(torch.as_tensor(A, device="cuda"), torch.as_tensor(Z, device="cuda"),
                        torch.as_tensor(Ex, device="cuda"), seed=seed,
                        P=None if P is None else torch.as_tensor(P, device="cuda"), first_event_id=first_id,
                        capacity=capacity, out=out)
    torch.cuda.synchronize()
    assert out.n_sec() <= out.capacity, (out.n_sec(), out.capacity)
    h = out.to_numpy()
    h["n_flagged"] = out.n_flagged()
    if history is not None:
        history["history"] = h["history"]
    if raw:
        return h
    r = h["res"]
    return ledger.Events(
        A=A.astype(np.int64), Z=Z.astype(np.int64), T0=np.zeros(n),
        A_f=r["A_f"].astype(np.int64), Z_f=r["Z_f"].astype(np.int64),
        Ex_casc=r["Ex_casc"].astype(np.float64), Ex_f=r["Ex_f"].astype(np.float64),
        p_f=r["p_f"].astype(np.float64), n_sec=r["n_sec"].astype(np.int64), flags=r["flags"].astype(np.int64),
        sec_event=h["sec_event"].astype(np.int64), sec_species=h["sec_species"].astype(np.int64),
        sec_stage=h["sec_stage"].astype(np.int64), sec_T=h["sec_T"].astype(np.float64),
        sec_u=h["sec_u"].astype(np.float64),
    )


def _mixture(n, seed, E_max=200.0, p_max=600.0):
    """Nuclei of the tables' range near stability, E* ~ U(0, E_max), isotropic
    momenta with |p| ~ U(0, p_max) MeV/c."""
    rng = np.random.default_rng(seed)
    A = rng.integers(5, 58, n)
    Z = np.clip(A // 2 + rng.integers(-2, 3, n), 1, np.minimum(A - 1, 27))
    Ex = rng.uniform(0.0, E_max, n)
    d = rng.normal(size=(n, 3))
    P = d / np.linalg.norm(d, axis=1)[:, None] * rng.uniform(0.0, p_max, n)[:, None]
    return A, Z, Ex, P


def _first_species(ev):
    """Species of each nucleus's first emission (records keep emission order
    within a nucleus); -1 where nothing was emitted."""
    order = np.argsort(ev.sec_event, kind="stable")
    e = ev.sec_event[order]
    first = np.full(ev.n, -1, dtype=np.int64)
    starts = np.flatnonzero(np.r_[True, e[1:] != e[:-1]]) if e.size else np.zeros(0, dtype=np.int64)
    first[e[starts]] = ev.sec_species[order][starts]
    return first


def _keys_in_order(ev):
    """Per-nucleus integer outcome: (A_f, Z_f, species in emission order)."""
    order = np.argsort(ev.sec_event, kind="stable")
    e = ev.sec_event[order]
    sp = ev.sec_species[order]
    bounds = np.searchsorted(e, np.arange(ev.n + 1))
    return [(int(ev.A_f[i]), int(ev.Z_f[i]), tuple(sp[bounds[i]:bounds[i + 1]].tolist())) for i in range(ev.n)]


@pytest.mark.parametrize("fast_math", [0, 1])
def test_evaporation_ledgers_every_nucleus(fast_math):
    import paper_1309_7963_amd as inc

    A, Z, Ex, P = _mixture(300_000, seed=21)
    c = inc.Context(TARGETS, fast_math=fast_math)
    try:
        ev = _run(c, A, Z, Ex, P, seed=5)
    finally:
        c.close()
    _, _, Ex32, P32 = _inputs(A, Z, Ex, P)
    s = ledger.check_evaporation(ev, P32.astype(np.float64))
    print("evaporation ledgers (fast_math=%d)" % fast_math, s)
    ledger.assert_clean(s)
    assert np.array_equal(ev.Ex_casc, Ex32.astype(np.float64))
    assert not ev.flags.any()
    assert s["n_secondaries"] == int(ev.n_sec.sum()) > ev.n


def _post_cascade(targets, T0, tidx, seed):
    """(A', Z', E*, p) of each event after the cascade (a cascade-only launch),
    as device tensors, with the full events of the same stream."""
    import torch

    import paper_1309_7963_amd as inc

    T0_d = torch.as_tensor(np.asarray(T0, dtype=np.float32), device="cuda")
    ti_d = torch.as_tensor(np.asarray(tidx, dtype=np.uint8), device="cuda")
    c = inc.Context(targets, no_evaporation=1)
    try:
        out = c.simulate(T0_d, seed=seed, target_idx=ti_d)
        torch.cuda.synchronize()
    finally:
        c.close()
    n = len(T0)
    r16 = out.res.view(torch.int16).view(n, 16)
    r32 = out.res.view(torch.float32).view(n, 8)
    return r16[:, 0].contiguous(), r16[:, 1].contiguous(), r32[:, 3].contiguous(), r32[:, 4:7].contiguous()


def test_evaporation_of_post_cascade_nuclei():
    # the nuclei the 200 MeV p+16O / p+40Ca cascades leave, evaporated alone:
    # every nucleus within the event ledgers' flat 1e-3 MeV and MeV/c gates,
    # and the fragments and final nuclei distributed as when the same
    # cascades are evaporated inside the event kernels (two-sample chi-square)
    import torch

    import paper_1309_7963_amd as inc

    targets = [(16, 8), (40, 20)]
    n = 200_000
    tidx = np.repeat([0, 1], n // 2).astype(np.uint8)
    T0 = np.full(n, 200.0, dtype=np.float32)
    A, Z, Ex, P = _post_cascade(targets, T0, tidx, seed=31)
    keep = (A > 0).cpu().numpy()
    c = inc.Context(targets)
    try:
        out = c.evaporate(A, Z, Ex, seed=32, P=P)
        torch.cuda.synchronize()
        h = out.to_numpy()
        full = c.simulate(torch.as_tensor(T0, device="cuda"), seed=31,
                          target_idx=torch.as_tensor(tidx, device="cuda"))
        torch.cuda.synchronize()
        f = full.to_numpy()
    finally:
        c.close()
    r = h["res"]
    idx = np.flatnonzero(keep)
    sel = np.isin(h["sec_event"], idx)
    remap = np.full(n, -1, dtype=np.int64)
    remap[idx] = np.arange(idx.size)
    ev = ledger.Events(
        A=A.cpu().numpy()[idx].astype(np.int64), Z=Z.cpu().numpy()[idx].astype(np.int64), T0=np.zeros(idx.size),
        A_f=r["A_f"][idx].astype(np.int64), Z_f=r["Z_f"][idx].astype(np.int64),
        Ex_casc=r["Ex_casc"][idx].astype(np.float64), Ex_f=r["Ex_f"][idx].astype(np.float64),
        p_f=r["p_f"][idx].astype(np.float64), n_sec=r["n_sec"][idx].astype(np.int64),
        flags=r["flags"][idx].astype(np.int64),
        sec_event=remap[h["sec_event"][sel].astype(np.int64)], sec_species=h["sec_species"][sel].astype(np.int64),
        sec_stage=h["sec_stage"][sel].astype(np.int64), sec_T=h["sec_T"][sel].astype(np.float64),
        sec_u=h["sec_u"][sel].astype(np.float64),
    )
    s = ledger.check_evaporation(ev, P.cpu().numpy()[idx].astype(np.float64))
    print("post-cascade evaporation ledgers", s)
    ledger.assert_clean(s)
    assert (r["flags"][~keep] == FLAG_RANGE).all()
    # the same cascades evaporated inside the event kernels (their stage-1 records)
    st1 = f["sec_stage"] == 1
    fe = np.full(n, -1, dtype=np.int64)
    fe[idx] = np.arange(idx.size)
    fsel = st1 & (fe[f["sec_event"]] >= 0)
    ref = ledger.Events(
        A=ev.A, Z=ev.Z, T0=ev.T0, A_f=f["res"]["A_f"][idx].astype(np.int64),
        Z_f=f["res"]["Z_f"][idx].astype(np.int64), Ex_casc=ev.Ex_casc, Ex_f=f["res"]["Ex_f"][idx].astype(np.float64),
        p_f=f["res"]["p_f"][idx].astype(np.float64), n_sec=ev.n_sec, flags=ev.flags,
        sec_event=fe[f["sec_event"][fsel]], sec_species=f["sec_species"][fsel].astype(np.int64),
        sec_stage=f["sec_stage"][fsel].astype(np.int64), sec_T=f["sec_T"][fsel].astype(np.float64),
        sec_u=f["sec_u"][fsel].astype(np.float64),
    )
    assert np.array_equal(f["res"]["Ex_casc"][idx], r["Ex_casc"][idx])
    res = stats.compare_samples(ev, ref, 60.0)
    print("evaporation alone vs inside the events", {k: (round(v[0], 1), v[1], round(v[2], 4)) for k, v in res.items()})
    assert not stats.gate(res), stats.gate(res)


def test_evaporation_thresholds(ctx):
    A, Z = 16, 8
    thr = np.array([evap_ref.threshold(A, Z, j) for j in range(6)])
    n = 10000
    rng = np.random.default_rng(3)
    P = rng.normal(size=(n, 3)) * 100.0
    E = np.full(n, min(thr) - 1e-3)
    ev = _run(ctx, np.full(n, A), np.full(n, Z), E, P, seed=2)
    _, _, E32, P32 = _inputs(np.full(n, A), np.full(n, Z), E, P)
    assert ev.sec_event.size == 0 and not ev.n_sec.any()
    assert (ev.A_f == A).all() and (ev.Z_f == Z).all()
    assert np.array_equal(ev.Ex_f, E32.astype(np.float64)) and np.array_equal(ev.p_f, P32.astype(np.float64))
    # window where exactly one channel is open
    j0, j1 = np.argsort(thr)[:2]
    E = np.full(n, 0.5 * (thr[j0] + thr[j1]))
    ev = _run(ctx, np.full(n, A), np.full(n, Z), E, P, seed=2)
    first = _first_species(ev)
    assert (first == j0).all(), np.bincount(first + 1)


def test_evaporation_branching_matches_widths(any_ctx):
    A, Z, E = 40, 20, 60.0
    n = 1_000_000
    ev = _run(any_ctx, np.full(n, A), np.full(n, Z), np.full(n, E), seed=4)
    first = _first_species(ev)
    assert (first >= 0).all()
    w = evap_ref.branching(A, Z, E)
    obs = np.bincount(first, minlength=6)
    use = w * n >= 5
    exp = w[use] * n
    chi2 = float(np.sum((obs[use] - exp) ** 2 / exp))
    p = float(chi2_dist.sf(chi2, int(use.sum()) - 1))
    print("first-emission branching", dict(zip("n p d t h a".split(), np.round(obs / n, 5))),
          "expected", np.round(w, 5), "chi2 %.1f p %.3f" % (chi2, p))
    assert obs[~use].sum() <= max(5, 3 * w[~use].sum() * n + 3)
    assert p > 0.01


def test_evaporation_single_neutron_spectrum(any_ctx):
    # 41Ar at E* = 14 MeV: only the neutron channel is open (threshold 6.08 MeV,
    # the next one above 16.6 MeV) and the daughter 40Ar stays below all of
    # its thresholds, so each nucleus emits exactly one neutron and keeps
    # E*_f = U - x
    A, Z, E = 41, 18, 14.0
    thr = [evap_ref.threshold(A, Z, j) for j in range(6)]
    assert np.argmin(thr) == 0 and sorted(thr)[1] > E
    assert thr[0] + min(evap_ref.threshold(A - 1, Z, j) for j in range(6)) > E
    n = 1_000_000
    ev = _run(any_ctx, np.full(n, A), np.full(n, Z), np.full(n, E), seed=6)
    assert (ev.n_sec == 1).all() and (ev.sec_species == 0).all()
    U = E - thr[0]
    a = (A - 1) / 8.0
    x = U - ev.Ex_f
    k = 50
    edges = np.array([0.0] + [oracle.spectrum_sample(a, U, q / k) for q in range(1, k)] + [U])
    obs = np.bincount(np.clip(np.searchsorted(edges, x, side="right") - 1, 0, k - 1), minlength=k)
    chi2 = float(np.sum((obs - n / k) ** 2 / (n / k)))
    p = float(chi2_dist.sf(chi2, k - 1))
    print("single-neutron spectrum: U %.4f MeV, chi2 %.1f / %d, p %.3f" % (U, chi2, k - 1, p))
    assert x.min() > -1e-4 and x.max() < U + 1e-4
    assert p > 0.01


def test_evaporation_replay_matches_oracle(ctx):
    n = 20000
    A, Z, Ex, P = _mixture(n, seed=23)
    hist = {}
    g = _run(ctx, A, Z, Ex, P, seed=9, first_id=1000, history=hist)
    A16, Z16, Ex32, P32 = _inputs(A, Z, Ex, P)
    o, rows = ledger.evaporate_oracle(A16, Z16, Ex32.astype(np.float64), P32.astype(np.float64), seed=9,
                                      first_id=1000, with_results=True)
    same = np.array([a == b for a, b in zip(_keys_in_order(g), _keys_in_order(o))])
    print("evaporation replay agreement", same.mean())
    assert same.mean() > 0.97
    # fragment by fragment on the nuclei whose emissions and draws agree, each
    # within the FP32 bound times its own amplification (the oracle with the
    # excitation energies moved up by one FP32 ulp)
    zeros = np.zeros(n, np.int64)
    Exp, delta = elementwise.one_ulp_up(Ex32)
    op, rows_p = ledger.evaporate_oracle(A16, Z16, Exp, P32.astype(np.float64), seed=9, first_id=1000,
                                         with_results=True)
    elementwise.assert_replay_close(g, o, dict(n_coll=zeros, n_retry=zeros), rows, "evaporation replay",
                                    g_hist=hist["history"], o_pert=(op, rows_p), delta=delta)


def test_evaporation_distributions_match_oracle(any_ctx):
    # same input mixture, GPU seed 1 (10^6 nuclei) vs oracle seed 2 (10^5)
    A, Z, Ex, P = _mixture(1_000_000, seed=25, E_max=150.0)
    g = _run(any_ctx, A, Z, Ex, P, seed=1)
    m = 100_000
    A16, Z16, Ex32, P32 = _inputs(A[:m], Z[:m], Ex[:m], P[:m])
    o = ledger.evaporate_oracle(A16, Z16, Ex32.astype(np.float64), P32.astype(np.float64), seed=2)
    res = stats.compare_samples(g, o, 60.0)
    print("evaporation GPU vs oracle", {k: (round(v[0], 1), v[1], round(v[2], 4)) for k, v in res.items()})
    assert not stats.gate(res), stats.gate(res)


def test_evaporation_invalid_nuclei_flagged(ctx):
    import paper_1309_7963_amd as inc

    good_A, good_Z, good_E, good_P = _mixture(64, seed=27)
    bad = [(0, 0, 10.0), (58, 20, 10.0), (20, 21, 10.0), (57, 28, 10.0), (40, 20, -1.0), (40, 20, 600.0),
           (40, 20, float("nan")), (40, 20, 20.0)]
    A = np.concatenate([good_A, [b[0] for b in bad]])
    Z = np.concatenate([good_Z, [b[1] for b in bad]])
    E = np.concatenate([good_E, [b[2] for b in bad]])
    P = np.concatenate([good_P, np.zeros((len(bad), 3))])
    P[-1, 1] = np.inf  # non-finite momentum
    h = _run(ctx, A, Z, E, P, seed=8, raw=True)
    r = h["res"]
    nb = len(bad)
    assert (r["flags"][-nb:] == FLAG_RANGE).all() and (r["A_f"][-nb:] == 0).all() and (r["n_sec"][-nb:] == 0).all()
    assert h["n_flagged"] == nb
    assert not np.isin(h["sec_event"], np.arange(len(A) - nb, len(A))).any()
    # the valid nuclei come out as they do without the invalid ones (records
    # compared nucleus by nucleus, in emission order)
    alone = _run(ctx, good_A, good_Z, good_E, good_P, seed=8, raw=True)
    assert alone["res"].tobytes() == r[:-nb].tobytes()
    oa = np.argsort(alone["sec_event"], kind="stable")
    ob = np.argsort(h["sec_event"], kind="stable")
    for f in ("sec_event", "sec_species", "sec_stage", "sec_T", "sec_u"):
        assert np.array_equal(alone[f][oa], h[f][ob]), f
    import torch

    empty = torch.zeros(0, dtype=torch.int16, device="cuda")
    with pytest.raises(inc.IncError):
        ctx.evaporate(empty, empty, torch.zeros(0, dtype=torch.float32, device="cuda"), seed=1)


@pytest.mark.parametrize("n", [1, 63, 65, 257])
def test_evaporation_ragged_batches_are_prefixes(ctx, n):
    # nucleus i's result depends only on its stream (seed, first_event_id + i):
    # a short batch equals the head of a longer one, whatever the chunking
    A, Z, Ex, P = _mixture(1000, seed=29)
    full = _run(ctx, A, Z, Ex, P, seed=12, first_id=77, raw=True)
    part = _run(ctx, A[:n], Z[:n], Ex[:n], P[:n], seed=12, first_id=77, raw=True)
    assert part["res"].tobytes() == full["res"][:n].tobytes()
    keep = full["sec_event"] < n
    oa = np.argsort(part["sec_event"], kind="stable")
    ob = np.argsort(full["sec_event"][keep], kind="stable")
    for f in ("sec_event", "sec_species", "sec_stage", "sec_T", "sec_u"):
        assert np.array_equal(part[f][oa], full[f][keep][ob]), f
