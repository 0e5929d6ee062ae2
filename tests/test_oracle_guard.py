"""Guard on the oracle's whole output while its code is reorganised.

Not a pin (a pin ties the oracle to something outside it; see
test_oracle_pins.py): this records a SHA-256 of every field the oracle
produces for two fixed workloads, so that a change meant to move code without
touching the arithmetic (a helper extracted, a duplicate removed) shows at
once if it changed any event.  A change that does alter the arithmetic must
update the digests here and name, in its commit, the passage of the paper or
the reading that justifies it.

Workloads: 10^4 events of 200 MeV p + 16O (seed 1), and 10^4 events of the
tissue mixture (12C/14N/16O/31P/40Ca with weights .18/.03/.65/.01/.13, T0
uniform in 20-250 MeV from numpy's generator seeded 1; physics seed 1).
"""
import hashlib

import numpy as np

import oracle

RESULT_FIELDS = ("A_casc", "Z_casc", "A_f", "Z_f", "Ex_casc", "Ex_f", "p_casc", "p_f", "n_sec", "flags",
                 "n_retry", "n_coll", "n_tent", "n_pauli", "n_seg", "n_evap", "n_draw", "first_z")
SECONDARY_FIELDS = ("event", "species", "stage", "T", "u")

DIGEST_O16 = "8e74f73b7154c6a714106c3346046ca70db9eeb8b6e670aafe583fb49d2e63f1"
DIGEST_TISSUE = "8edea9111c861c8883b948ec1bc34c959110218f61a6aceb026f1296f82de4db"


def digest(out) -> str:
    h = hashlib.sha256()
    for f in RESULT_FIELDS:
        h.update(np.ascontiguousarray(out.results[f]).tobytes())
    for f in SECONDARY_FIELDS:
        h.update(np.ascontiguousarray(out.secondaries[f]).tobytes())
    return h.hexdigest()


def test_oxygen_output_unchanged():
    out = oracle.run([(16, 8)], np.full(10000, 200.0), seed=1)
    assert digest(out) == DIGEST_O16


def test_tissue_mixture_output_unchanged():
    rng = np.random.default_rng(1)
    targets = [(12, 6), (14, 7), (16, 8), (31, 15), (40, 20)]
    tidx = rng.choice(5, size=10000, p=[0.18, 0.03, 0.65, 0.01, 0.13]).astype(np.uint8)
    T0 = rng.uniform(20, 250, 10000)
    out = oracle.run(targets, T0, seed=1, tidx=tidx)
    assert digest(out) == DIGEST_TISSUE


def test_digest_sees_a_one_ulp_change():
    out = oracle.run([(16, 8)], np.full(200, 200.0), seed=1)
    d0 = digest(out)
    out.secondaries["T"][7] = np.nextafter(out.secondaries["T"][7], np.inf)
    assert digest(out) != d0
