"""CPU oracle for the intranuclear cascade + evaporation method of
arXiv:1309.7963 (Sec. 2), in double precision.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no code
with the GPU library (``paper_1309_7963_amd``) and never imports it.

The C++ source ``inc_oracle.cpp`` is compiled with g++ into ``liboracle.so``
next to it (``build()``); importing this module compiles it when the library is
missing or older than its source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "inc_oracle.cpp")
_HDR = os.path.join(_HERE, "inc_oracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")

NSHELL = 15
SPECIES = ("n", "p", "d", "t", "He3", "alpha")
# (a, z) of the six evaporated fragments, Sec. 2.4
FRAGMENT_AZ = ((1, 0), (1, 1), (2, 1), (3, 1), (3, 2), (4, 2))


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(_HDR)
    ):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB)
    return _LIB


class Nucleus(C.Structure):
    _fields_ = [
        ("A", C.c_int), ("Z", C.c_int),
        ("c", C.c_double), ("delta", C.c_double), ("R", C.c_double),
        ("r", C.c_double * (NSHELL + 1)),
        ("integral", C.c_double * NSHELL),
        ("rho", (C.c_double * NSHELL) * 2),
        ("pF", (C.c_double * NSHELL) * 2),
        ("EF", (C.c_double * NSHELL) * 2),
        ("EB", C.c_double), ("EC", C.c_double),
    ]


class Options(C.Structure):
    _fields_ = [
        ("uniform_density", C.c_int),
        ("zero_fermi", C.c_int),
        ("zero_binding", C.c_int),
        ("no_pauli", C.c_int),
        ("no_evaporation", C.c_int),
        ("stop_after_first", C.c_int),
        ("const_sigma_mb", C.c_double),
        ("fixed_b", C.c_double),
        ("max_stack", C.c_int),
        ("max_segments", C.c_int),
        ("photon_evaporation", C.c_int),
        ("heavy_fragments", C.c_int),
    ]


class Result(C.Structure):
    _fields_ = [
        ("A_casc", C.c_int), ("Z_casc", C.c_int),
        ("A_f", C.c_int), ("Z_f", C.c_int),
        ("Ex_casc", C.c_double), ("Ex_f", C.c_double),
        ("p_casc", C.c_double * 3), ("p_f", C.c_double * 3),
        ("n_sec", C.c_int), ("flags", C.c_int),
        ("n_retry", C.c_int), ("n_coll", C.c_int), ("n_tent", C.c_int),
        ("n_pauli", C.c_int), ("n_seg", C.c_int), ("n_evap", C.c_int),
        ("n_draw", C.c_int),
        ("first_z", C.c_double),
        ("sea", C.c_int * 2), ("sea_min", C.c_int), ("tent_shells", C.c_uint32),
        ("n_tau", C.c_int), ("n_majorant", C.c_int),
    ]


class Secondary(C.Structure):
    _fields_ = [
        ("event", C.c_uint32), ("species", C.c_int), ("stage", C.c_int),
        ("T", C.c_double), ("u", C.c_double * 3),
    ]


RESULT_DTYPE = np.dtype(
    [
        ("A_casc", "i4"), ("Z_casc", "i4"), ("A_f", "i4"), ("Z_f", "i4"),
        ("Ex_casc", "f8"), ("Ex_f", "f8"), ("p_casc", "f8", 3), ("p_f", "f8", 3),
        ("n_sec", "i4"), ("flags", "i4"), ("n_retry", "i4"), ("n_coll", "i4"),
        ("n_tent", "i4"), ("n_pauli", "i4"), ("n_seg", "i4"), ("n_evap", "i4"),
        ("n_draw", "i4"), ("first_z", "f8"), ("sea", "i4", 2), ("sea_min", "i4"), ("tent_shells", "u4"),
        ("n_tau", "i4"), ("n_majorant", "i4"),
    ],
    align=True,
)
SECONDARY_DTYPE = np.dtype(
    [("event", "u4"), ("species", "i4"), ("stage", "i4"), ("T", "f8"), ("u", "f8", 3)],
    align=True,
)
assert RESULT_DTYPE.itemsize == C.sizeof(Result)
assert SECONDARY_DTYPE.itemsize == C.sizeof(Secondary)

_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB)
        d, i, u32, u64 = C.c_double, C.c_int, C.c_uint32, C.c_uint64
        L.orc_philox4x32_10.argtypes = [C.POINTER(u32), C.POINTER(u32), C.POINTER(u32)]
        L.orc_uniform.argtypes = [u32]
        L.orc_uniform.restype = d
        L.orc_stream_uniform.argtypes = [u64, u64, u64]
        L.orc_stream_uniform.restype = d
        L.orc_binding.argtypes = [i, i]
        L.orc_binding.restype = d
        L.orc_mass.argtypes = [i, i]
        L.orc_mass.restype = d
        L.orc_nucleus_setup.argtypes = [i, i, C.POINTER(Options), C.POINTER(Nucleus)]
        L.orc_nucleus_setup.restype = i
        for name in ("orc_sigma", "orc_sigma_hat", "orc_slope"):
            getattr(L, name).argtypes = [i, d]
            getattr(L, name).restype = d
        L.orc_plab_min.argtypes = [d, d, d, d]
        L.orc_plab_min.restype = d
        P3 = d * 3
        L.orc_elastic.argtypes = [P3, d, P3, d, d, d, d, P3, P3, C.POINTER(d), C.POINTER(d)]
        L.orc_elastic.restype = d
        L.orc_refract.argtypes = [P3, P3, d, d, d]
        L.orc_refract.restype = i
        L.orc_collision_outcome.argtypes = [C.POINTER(Nucleus), i, i, i, d, d, d, i, d * 3]
        L.orc_collision_outcome.restype = i
        L.orc_width_integral.argtypes = [d, d]
        L.orc_width_integral.restype = d
        L.orc_spectrum_cdf.argtypes = [d, d, d]
        L.orc_spectrum_cdf.restype = d
        L.orc_spectrum_sample.argtypes = [d, d, d]
        L.orc_spectrum_sample.restype = d
        L.orc_fermi_sample.argtypes = [d, d, d, d, d * 3]
        for name in ("orc_photon_integral", "orc_photon_cdf", "orc_photon_sample"):
            getattr(L, name).argtypes = [d, d] + ([d] if name != "orc_photon_integral" else [])
            getattr(L, name).restype = d
        L.orc_gdr_energy.argtypes = [i]
        L.orc_gdr_energy.restype = d
        L.orc_photon_s0.argtypes = [i, i]
        L.orc_photon_s0.restype = d
        L.orc_photon_width.argtypes = [i, i, d]
        L.orc_photon_width.restype = d
        L.orc_fragment.argtypes = [i, C.POINTER(i), C.POINTER(i), C.POINTER(i)]
        L.orc_fragment.restype = i
        L.orc_evaporate.argtypes = [i, i, d, d * 3, u64, u64, C.POINTER(Options), C.c_void_p, C.c_void_p, i]
        L.orc_evaporate.restype = i
        L.orc_run.argtypes = [
            C.POINTER(C.c_int), i, C.POINTER(Options), C.c_size_t,
            C.c_void_p, C.c_void_p, u64, u64, C.c_void_p, C.c_void_p, C.c_size_t, i,
        ]
        L.orc_run.restype = C.c_int64
        _lib = L
    return _lib


# ---------------------------------------------------------------- wrappers
def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return tuple(o)


def uniform(w: int) -> float:
    return lib().orc_uniform(w)


def stream_uniform(seed: int, event_id: int, k: int) -> float:
    return lib().orc_stream_uniform(seed, event_id, k)


def binding(A: int, Z: int) -> float:
    return lib().orc_binding(A, Z)


def mass(A: int, Z: int) -> float:
    return lib().orc_mass(A, Z)


def options(**kw) -> Options:
    o = Options()
    o.fixed_b = -1.0
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def nucleus(A: int, Z: int, **hooks) -> Nucleus:
    n = Nucleus()
    if lib().orc_nucleus_setup(A, Z, C.byref(options(**hooks)), C.byref(n)) != 0:
        raise ValueError("invalid nucleus (%d, %d)" % (A, Z))
    return n


def sigma(like: int, p_GeV: float) -> float:
    return lib().orc_sigma(like, p_GeV)


def sigma_hat(like: int, p_GeV: float) -> float:
    return lib().orc_sigma_hat(like, p_GeV)


def slope(like: int, p_GeV: float) -> float:
    return lib().orc_slope(like, p_GeV)


def plab_min(p, mx, pF, my) -> float:
    return lib().orc_plab_min(p, mx, pF, my)


def elastic(px, mx, pt, my, b, u_theta, u_phi):
    P3 = C.c_double * 3
    qx, qt = P3(), P3()
    Tx, Tt = C.c_double(), C.c_double()
    plab = lib().orc_elastic(P3(*px), mx, P3(*pt), my, b, u_theta, u_phi, qx, qt, C.byref(Tx), C.byref(Tt))
    return np.array(qx[:]), np.array(qt[:]), Tx.value, Tt.value, plab


def refract(d, n, T_from, T_to, m):
    P3 = C.c_double * 3
    dd = P3(*d)
    r = lib().orc_refract(dd, P3(*n), T_from, T_to, m)
    return bool(r), np.array(dd[:])


def collision_outcome(nu, shell, sp_x, sp_y, Tx, Ty, Tt, pauli=True):
    """Pauli and cutoff decision after a collision (Sec. 2.3); returns
    (blocked, track_x, track_y, eps_x, eps_y, hole)."""
    out = (C.c_double * 3)()
    r = lib().orc_collision_outcome(C.byref(nu), shell, sp_x, sp_y, Tx, Ty, Tt, int(pauli), out)
    if r < 0:
        raise ValueError("bad arguments")
    return bool(r & 1), bool(r & 2), bool(r & 4), out[0], out[1], out[2]


def width_integral(a, U) -> float:
    return lib().orc_width_integral(a, U)


def spectrum_cdf(a, U, x) -> float:
    return lib().orc_spectrum_cdf(a, U, x)


def spectrum_sample(a, U, u) -> float:
    return lib().orc_spectrum_sample(a, U, u)


def fermi_sample(pF, u1, u2, u3):
    p = (C.c_double * 3)()
    lib().orc_fermi_sample(pF, u1, u2, u3, p)
    return np.array(p[:])


def evaporate(A, Z, Ex, P=(0.0, 0.0, 0.0), seed=1, event_id=0, photon_evaporation=0, heavy_fragments=0):
    """Evaporate one excited nucleus; returns (result record, secondaries)."""
    res = np.zeros(1, dtype=RESULT_DTYPE)
    opt = options(photon_evaporation=photon_evaporation, heavy_fragments=heavy_fragments)
    cap = A + 1
    while True:
        sec = np.zeros(cap, dtype=SECONDARY_DTYPE)
        n = lib().orc_evaporate(A, Z, Ex, (C.c_double * 3)(*P), seed, event_id, C.byref(opt), res.ctypes.data,
                                sec.ctypes.data, cap)
        if n < 0:
            raise ValueError("invalid nucleus")
        if n <= cap:
            return res[0], sec[:n].copy()
        cap = n  # photons do not use up nucleons: run again with room for all


def fragment(j: int):
    """(a, z, g) of emitted species j (0-5 particles, 7-26 heavier fragments,
    reading R20); None for the photon (6) or out of range."""
    a, z, g = C.c_int(), C.c_int(), C.c_int()
    if not lib().orc_fragment(j, C.byref(a), C.byref(z), C.byref(g)):
        return None
    return a.value, z.value, g.value


def gdr_energy(A: int) -> float:
    return lib().orc_gdr_energy(A)


def photon_s0(A: int, Z: int) -> float:
    return lib().orc_photon_s0(A, Z)


def photon_integral(a, U) -> float:
    return lib().orc_photon_integral(a, U)


def photon_cdf(a, U, x) -> float:
    return lib().orc_photon_cdf(a, U, x)


def photon_sample(a, U, u) -> float:
    return lib().orc_photon_sample(a, U, u)


def photon_width(A: int, Z: int, E: float) -> float:
    return lib().orc_photon_width(A, Z, E)


@dataclass
class RunOutput:
    results: np.ndarray        # RESULT_DTYPE, one per event
    secondaries: np.ndarray    # SECONDARY_DTYPE, sorted by event
    n_sec_total: int


def run(targets, T0, seed, tidx=None, first_id=0, n_threads=None, sec_per_event=None, **hooks) -> RunOutput:
    """Simulate len(T0) non-elastic events.  targets: list of (A, Z)."""
    T0 = np.ascontiguousarray(T0, dtype=np.float64)
    n = T0.shape[0]
    AZ = np.ascontiguousarray(np.array(targets, dtype=np.int32).reshape(-1, 2))
    if tidx is not None:
        tidx = np.ascontiguousarray(tidx, dtype=np.uint8)
        assert tidx.shape[0] == n
    if n_threads is None:
        n_threads = max(1, min(os.cpu_count() or 1, 16))
    if sec_per_event is None:
        sec_per_event = int(AZ[:, 0].max()) + 1
    res = np.zeros(n, dtype=RESULT_DTYPE)
    cap = max(1, n * sec_per_event)
    opt = options(**hooks)
    while True:
        sec = np.zeros(cap, dtype=SECONDARY_DTYPE)
        total = lib().orc_run(
            AZ.ctypes.data_as(C.POINTER(C.c_int)), AZ.shape[0], C.byref(opt), n,
            tidx.ctypes.data if tidx is not None else None, T0.ctypes.data,
            seed, first_id, res.ctypes.data, sec.ctypes.data, cap, n_threads,
        )
        if total < 0:
            raise ValueError("oracle rejected the arguments")
        if total <= cap:
            return RunOutput(res, sec[:total].copy(), int(total))
        cap = int(total)  # (photons add records beyond A + 1 per event) run again
