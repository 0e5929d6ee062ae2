"""The two-sample statistics of the parity tests (tests/stats.py), on the CPU:
they pass two oracle samples with different seeds and sizes (as the GPU
tests compare 10^6 GPU events with fewer oracle events), and each fails on a
mistake planted in one oracle sample's output."""
import dataclasses

import numpy as np
import pytest

import ledger
import oracle
import stats

CA40 = [(40, 20)]


@pytest.fixture(scope="module")
def samples():
    T0 = np.full(200_000, 200.0)
    a = ledger.from_oracle(oracle.run(CA40, T0, seed=11, n_threads=8), CA40, T0)
    b = ledger.from_oracle(oracle.run(CA40, T0[:40_000], seed=12, n_threads=8), CA40, T0[:40_000])
    return a, b


def test_same_model_passes_at_unequal_sizes(samples):
    a, b = samples
    res = stats.compare_samples(a, b, 200.0)
    print({k: (round(v[0], 1), v[1], round(v[2], 4)) for k, v in res.items()})
    assert set(res) >= set(stats.PRIMARY) | {"alpha_T", "t_cos", "He3_mult", "Ex_f"}
    assert not stats.gate(res), stats.gate(res)


def _planted(ev, **arrays):
    return dataclasses.replace(ev, **arrays)


def test_planted_mistakes_fail(samples):
    a, b = samples
    sp = b.sec_species
    rng = np.random.default_rng(5)
    cases = {
        # alpha energies 3 % high
        "alpha_T": dict(sec_T=np.where(sp == 5, b.sec_T * 1.03, b.sec_T)),
        # the triton and 3He species codes swapped
        "t_mult": dict(sec_species=np.where(sp == 3, 4, np.where(sp == 4, 3, sp))),
        # deuterons sent backward a fifth of the time
        "d_cos": dict(sec_u=np.where(((sp == 2) & (rng.random(sp.size) < 0.2))[:, None],
                                     -np.abs(b.sec_u), b.sec_u)),
        # the final excitation 0.3 MeV high
        "Ex_f": dict(Ex_f=b.Ex_f + 0.3),
    }
    for key, change in cases.items():
        res = stats.compare_samples(a, _planted(b, **change), 200.0)
        failed = [f[0] for f in stats.gate(res)]
        print(key, failed)
        assert key in failed, (key, res[key])


def test_planted_physics_mistake_fails_the_primary_statistics(samples):
    # the oracle without Pauli blocking (Sec. 2.3) against the oracle
    a, _ = samples
    T0 = np.full(40_000, 200.0)
    b = ledger.from_oracle(oracle.run(CA40, T0, seed=12, n_threads=8, no_pauli=1), CA40, T0)
    res = stats.compare_samples(a, b, 200.0)
    failed = {f[0] for f in stats.gate(res)}
    print(sorted(failed))
    assert set(stats.PRIMARY) <= failed
