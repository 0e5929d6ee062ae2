"""The optional photon channel of the evaporation (photon_evaporation = 1;
the oracle's reading R19) on the GPU, through the C ABI, against the
oracle: ledgers with photons on every event, first-emission branching and
the first photon's spectrum against the widths by quadrature, same-stream
replay value by value, and two-sample statistics at 10^6 events.  With the
option off (the default) no photon is ever emitted."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.stats import chi2 as chi2_dist

import elementwise
import evap_ref
import ledger
import oracle
import stats
from gpu_util import events_from_gpu, run_gpu

pytestmark = pytest.mark.gpu

O16, CA40, FE56 = (16, 8), (40, 20), (56, 26)


def _evaporate(ctx, A, Z, E, seed, first_id=0):
    import torch
    import paper_1309_7963_amd as inc

    n = len(E)
    out = inc.DeviceOutput.allocate(n, 24 * n + 4096, "cuda", history=True)
    ctx.evaporate(torch.as_tensor(np.asarray(A, np.int16), device="cuda"),
                  torch.as_tensor(np.asarray(Z, np.int16), device="cuda"),
                  torch.as_tensor(np.asarray(E, np.float32), device="cuda"), seed=seed, first_event_id=first_id,
                  out=out)
    torch.cuda.synchronize()
    assert out.n_sec() <= out.capacity
    return out.to_numpy()


@pytest.mark.parametrize("mode", ["plain", "persistent", "staged"])
@pytest.mark.parametrize("target,T", [(O16, 200.0), (CA40, 70.0), (FE56, 250.0)])
def test_photon_ledgers_every_event(mode, target, T):
    n = 20000
    T0 = np.full(n, T, dtype=np.float32)
    h = run_gpu([target], T0, seed=1, mode=mode, photon_evaporation=1)
    ev = events_from_gpu(h, [target], T0)
    s = ledger.check(ev, photons=True)
    ledger.assert_clean(s)
    ph = ev.sec_species == ledger.PHOTON
    print("photons", target, T, mode, "per event %.2f" % (ph.sum() / n), "max |E2| %.1e" % s["max_E2"])
    assert ph.sum() > n and (ev.sec_stage[ph] == 1).all()


def test_photon_option_off_emits_no_photon():
    T0 = np.full(20000, 200.0, dtype=np.float32)
    h = run_gpu([CA40], T0, seed=1, mode="staged")
    assert not (h["sec_species"] == ledger.PHOTON).any()


@pytest.mark.parametrize("A,Z,E", [(40, 20, 13.0), (40, 20, 16.0), (16, 8, 12.0)])
def test_photon_branching_matches_widths(A, Z, E):
    # first emissions of 10^6 nuclei against Gamma_j / sum Gamma (particles and
    # photon) from the width formulas with their integrals by quadrature
    import paper_1309_7963_amd as inc

    ctx = inc.Context([(A - 1, Z - 1)], photon_evaporation=1)
    n = 1_000_000
    h = _evaporate(ctx, np.full(n, A), np.full(n, Z), np.full(n, E), seed=4)
    ctx.close()
    order = np.argsort(h["sec_event"], kind="stable")
    ev = h["sec_event"][order]
    first = h["sec_species"][order][np.searchsorted(ev, np.arange(n))]
    p = evap_ref.branching(A, Z, E, photons=True)
    obs = np.bincount(first, minlength=7)
    keep = p * n >= 5
    chi2 = float(np.sum((obs[keep] - p[keep] * n) ** 2 / (p[keep] * n)))
    pv = float(chi2_dist.sf(chi2, keep.sum() - 1))
    print(A, Z, E, "photon share %.5f observed %.5f, chi2 %.1f / %d, p %.3f" % (p[6], obs[6] / n, chi2,
                                                                                keep.sum() - 1, pv))
    assert obs[~keep].sum() <= 10 and pv > 0.01


def test_first_photon_spectrum():
    # 40Ca at rest at E* = 9 MeV (below every particle threshold): the first
    # photon's share e of the excitation, from its energy, in 50 equiprobable
    # bins of the spectrum e^3 rho(E - e) (edges by quadrature)
    import paper_1309_7963_amd as inc

    A, Z, E = 40, 20, 9.0
    ctx = inc.Context([(39, 19)], photon_evaporation=1)
    n = 1_000_000
    h = _evaporate(ctx, np.full(n, A), np.full(n, Z), np.full(n, E), seed=6)
    ctx.close()
    order = np.argsort(h["sec_event"], kind="stable")
    ev = h["sec_event"][order]
    Eg = h["sec_T"][order][np.searchsorted(ev, np.arange(n))].astype(np.float64)
    Mp = oracle.mass(A, Z) + E
    eps = Mp - np.sqrt(Mp * Mp - 2.0 * Mp * Eg)
    a = A / 8.0
    f = lambda e: e ** 3 * math.exp(2.0 * math.sqrt(a * max(E - e, 0.0)))
    total = integrate.quad(f, 0.0, E, epsrel=1e-12)[0]
    k = 50
    edges = [0.0]
    for q in range(1, k):
        lo, hi = edges[-1], E
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            if integrate.quad(f, 0.0, mid, epsrel=1e-12)[0] / total < q / k:
                lo = mid
            else:
                hi = mid
        edges.append(0.5 * (lo + hi))
    edges.append(E)
    obs = np.bincount(np.clip(np.searchsorted(edges, eps, side="right") - 1, 0, k - 1), minlength=k)
    chi2 = float(np.sum((obs - n / k) ** 2 / (n / k)))
    p = float(chi2_dist.sf(chi2, k - 1))
    print("first photon spectrum: chi2 %.1f / %d, p %.3f" % (chi2, k - 1, p))
    assert eps.min() >= 0.0 and eps.max() <= E + 1e-4 and p > 0.01


def test_photon_replay_elementwise():
    # same seed on both sides, the photon channel on: whole events (16O and
    # 40Ca at 200 MeV) and the evaporation alone, value by value on the
    # events whose discrete history agrees
    for target in (O16, CA40):
        n = 10000
        T0 = np.full(n, 200.0, dtype=np.float32)
        h = run_gpu([target], T0, seed=1, mode="staged", history=True, photon_evaporation=1)
        g = events_from_gpu(h, [target], T0)
        out = oracle.run([target], T0.astype(np.float64), seed=1, n_threads=16, photon_evaporation=1)
        o = ledger.from_oracle(out, [target], T0)
        Tp, delta = elementwise.one_ulp_up(T0, top=250.0)
        outp = oracle.run([target], Tp, seed=1, n_threads=16, photon_evaporation=1)
        elementwise.assert_replay_close(g, o, h["res"], out.results, "photon replay %s" % (target,),
                                        g_hist=h["history"],
                                        o_pert=(ledger.from_oracle(outp, [target], Tp), outp.results), delta=delta)


@pytest.mark.parametrize("target", [O16, CA40])
def test_photon_chi2_paper_scale(target):
    n = 1_000_000
    T0 = np.full(n, 200.0, dtype=np.float32)
    g = events_from_gpu(run_gpu([target], T0, seed=1, mode="staged", photon_evaporation=1), [target], T0)
    out = oracle.run([target], T0.astype(np.float64), seed=2, n_threads=16, photon_evaporation=1)
    o = ledger.from_oracle(out, [target], T0)
    res = stats.compare_samples(g, o, 200.0)
    print("photons on, 200 MeV", target, {k: (round(v[0], 1), v[1], round(v[2], 4)) for k, v in res.items()})
    assert res["gamma_T"][1] > 0
    assert not stats.gate(res), stats.gate(res)
