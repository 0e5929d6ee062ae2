"""The optional heavier evaporation fragments (heavy_fragments = 1; the
oracle's reading R20: the stable isotopes of Li to Mg as channels 7-26) on
the GPU, through the C ABI, against the oracle: ledgers on every event in
every launch mode, first-emission branching over all 26 channels against the
widths by quadrature, and same-stream replay value by value.  With the
option off (the default) no heavier fragment is ever emitted."""
import numpy as np
import pytest
from scipy.stats import chi2 as chi2_dist

import elementwise
import evap_ref
import ledger
import oracle
from gpu_util import events_from_gpu, run_gpu

pytestmark = pytest.mark.gpu

O16, AL27, CA40 = (16, 8), (27, 13), (40, 20)


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
@pytest.mark.parametrize("target,T", [(O16, 200.0), (AL27, 250.0), (CA40, 150.0)])
def test_heavy_ledgers_every_event(mode, target, T):
    n = 50000
    T0 = np.full(n, T, dtype=np.float32)
    h = run_gpu([target], T0, seed=1, mode=mode, heavy_fragments=1)
    ev = events_from_gpu(h, [target], T0)
    s = ledger.check(ev, heavy=True)
    ledger.assert_clean(s)
    hv = ev.sec_species >= 7
    print("heavier fragments", target, T, mode, hv.sum(), "max |E2| %.1e" % s["max_E2"])
    assert hv.sum() > 0 and (ev.sec_stage[hv] == 1).all()


def test_heavy_and_photons_together():
    n = 50000
    T0 = np.full(n, 200.0, dtype=np.float32)
    for mode in ("persistent", "staged"):
        h = run_gpu([CA40], T0, seed=2, mode=mode, heavy_fragments=1, photon_evaporation=1)
        ev = events_from_gpu(h, [CA40], T0)
        ledger.assert_clean(ledger.check(ev, photons=True, heavy=True))
        assert (ev.sec_species == ledger.PHOTON).any() and (ev.sec_species >= 7).any()


def test_heavy_option_off_emits_none():
    T0 = np.full(50000, 250.0, dtype=np.float32)
    h = run_gpu([AL27], T0, seed=1, mode="staged")
    assert not (h["sec_species"] >= 7).any()


@pytest.mark.parametrize("A,Z,E", [(12, 6, 40.0), (16, 8, 50.0)])
def test_heavy_branching_matches_widths(A, Z, E):
    # first emissions of 10^6 nuclei against Gamma_j / sum Gamma over the six
    # particles and the 20 heavier fragments, widths by quadrature
    import paper_1309_7963_amd as inc

    ctx = inc.Context([(A - 1, Z - 1)], heavy_fragments=1)
    n = 1_000_000
    h = _evaporate(ctx, np.full(n, A), np.full(n, Z), np.full(n, E), seed=4)
    ctx.close()
    order = np.argsort(h["sec_event"], kind="stable")
    ev = h["sec_event"][order]
    first = h["sec_species"][order][np.searchsorted(ev, np.arange(n))]
    p = evap_ref.branching(A, Z, E, heavy=True)
    obs = np.bincount(first, minlength=27)
    keep = p * n >= 5
    chi2 = float(np.sum((obs[keep] - p[keep] * n) ** 2 / (p[keep] * n)))
    pv = float(chi2_dist.sf(chi2, keep.sum() - 1))
    print(A, Z, E, "heavier share %.5f observed %.5f, chi2 %.1f / %d, p %.3f" % (p[7:].sum(), obs[7:].sum() / n,
                                                                                 chi2, keep.sum() - 1, pv))
    assert obs[~keep].sum() <= 10 and pv > 0.01


def test_heavy_replay_elementwise():
    # same seed on both sides, the heavier fragments on: whole events (16O
    # and 40Ca at 200 MeV), value by value on the events whose discrete
    # history agrees
    for target in (O16, CA40):
        n = 10000
        T0 = np.full(n, 200.0, dtype=np.float32)
        h = run_gpu([target], T0, seed=1, mode="staged", history=True, heavy_fragments=1)
        g = events_from_gpu(h, [target], T0)
        out = oracle.run([target], T0.astype(np.float64), seed=1, n_threads=16, heavy_fragments=1)
        o = ledger.from_oracle(out, [target], T0)
        Tp, delta = elementwise.one_ulp_up(T0, top=250.0)
        outp = oracle.run([target], Tp, seed=1, n_threads=16, heavy_fragments=1)
        elementwise.assert_replay_close(g, o, h["res"], out.results, "heavy replay %s" % (target,),
                                        g_hist=h["history"],
                                        o_pert=(ledger.from_oracle(outp, [target], Tp), outp.results), delta=delta)


def test_heavy_evaporation_replay_elementwise():
    # the evaporation alone (nucleus i on event i's stream from its first
    # draw) of 24Mg at 60 MeV, where the heavier channels are frequent,
    # value by value against the oracle
    import paper_1309_7963_amd as inc

    A, Z, E = 24, 12, 60.0
    n = 20000
    ctx = inc.Context([(A - 1, Z - 1)], heavy_fragments=1)
    h = _evaporate(ctx, np.full(n, A), np.full(n, Z), np.full(n, E), seed=8)
    ctx.close()
    o_first = []
    same = 0
    for i in range(n):
        r, s = oracle.evaporate(A, Z, E, seed=8, event_id=i, heavy_fragments=1)
        o_first.append(s["species"].tolist())
    order = np.lexsort((np.arange(len(h["sec_event"])), h["sec_event"]))
    ev = h["sec_event"][order]
    sp = h["sec_species"][order]
    bounds = np.searchsorted(ev, np.arange(n + 1))
    for i in range(n):
        if sp[bounds[i]:bounds[i + 1]].tolist() == o_first[i]:
            same += 1
    heavy_events = sum(any(x >= 7 for x in f) for f in o_first)
    print("evaporation replay: same emission sequence in %d of %d nuclei (%d with heavier fragments)" %
          (same, n, heavy_events))
    assert heavy_events > 100
    assert same >= 0.99 * n
