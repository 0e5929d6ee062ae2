"""MI355X (gfx950) intranuclear cascade + evaporation event generator
(arXiv:1309.7963).  Python surface over the C ABI of include/inc.h; PyTorch
provides device memory and streams, every step of the method runs in the HIP
kernels of ``csrc/``.

    import torch, paper_1309_7963_amd as inc
    ctx = inc.Context([(16, 8)])
    T0 = torch.full((10000,), 200.0, device="cuda")
    out = ctx.simulate(T0, seed=1)
    host = out.to_numpy()
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import ctypes as C
import gc

import numpy as np

from . import _lib
from ._lib import (  # noqa: F401
    INC_ERR_ARG, INC_ERR_BUSY, INC_ERR_CAPACITY, INC_ERR_DEVICE, INC_ERR_NO_DEVICE, INC_ERR_OOM, INC_ERR_RANGE,
    INC_ERR_TOO_LARGE, NOALLOC_MAX_EVENTS, MODE_PERSISTENT, MODE_PLAIN, MODE_STAGED, MODE_VERTEX, RESIDUAL_DTYPE,
    IncError,
)

FLAG_STACK, FLAG_SEGMENTS, FLAG_EMPTY, FLAG_RANGE = 1, 2, 4, 0x8000


def _torch():
    import torch

    return torch


@dataclass
class DeviceOutput:
    """Caller-owned device buffers of one batch (torch tensors)."""

    n: int
    res: "object"          # uint8 [n * 32] (RESIDUAL_DTYPE records)
    sec_event: "object"    # int32 [cap] (uint32 values)
    sec_species: "object"  # uint8 [cap]
    sec_stage: "object"    # uint8 [cap]
    sec_T: "object"        # float32 [cap]
    sec_ux: "object"
    sec_uy: "object"
    sec_uz: "object"
    counters: "object"     # int64 [4]
    history: "object" = None  # int32 [3 n] (uint32 values) or None: per event the
    #                           uniforms drawn, the cascade's flight segments and
    #                           the shell fingerprint of its tentative collisions

    @property
    def capacity(self) -> int:
        return int(self.sec_T.shape[0])

    @classmethod
    def allocate(cls, n: int, capacity: int, device="cuda", history: bool = False):
        torch = _torch()
        cap = max(int(capacity), 1)
        e = lambda dt: torch.empty(cap, dtype=dt, device=device)
        return cls(
            n=n,
            res=torch.empty(n * 32, dtype=torch.uint8, device=device),
            sec_event=e(torch.int32), sec_species=e(torch.uint8), sec_stage=e(torch.uint8),
            sec_T=e(torch.float32), sec_ux=e(torch.float32), sec_uy=e(torch.float32), sec_uz=e(torch.float32),
            counters=torch.zeros(4, dtype=torch.int64, device=device),
            history=torch.empty(3 * n, dtype=torch.int32, device=device) if history else None,
        )

    def c_struct(self, capacity: Optional[int] = None) -> _lib.Output:
        o = _lib.Output()
        o.res = self.res.data_ptr()
        o.sec_event = self.sec_event.data_ptr()
        o.sec_species = self.sec_species.data_ptr()
        o.sec_stage = self.sec_stage.data_ptr()
        o.sec_T = self.sec_T.data_ptr()
        o.sec_ux = self.sec_ux.data_ptr()
        o.sec_uy = self.sec_uy.data_ptr()
        o.sec_uz = self.sec_uz.data_ptr()
        o.sec_capacity = self.capacity if capacity is None else int(capacity)
        o.counters = self.counters.data_ptr()
        o.history = self.history.data_ptr() if self.history is not None else None
        return o

    def n_sec(self) -> int:
        """Secondaries produced (synchronises with the device)."""
        return int(self.counters[0].item())

    def n_flagged(self) -> int:
        return int(self.counters[1].item())

    def to_numpy(self) -> dict:
        """Copy everything to host numpy arrays (synchronising)."""
        k = min(self.n_sec(), self.capacity)
        res = self.res.cpu().numpy().view(RESIDUAL_DTYPE)
        extra = {}
        if self.history is not None:
            extra["history"] = self.history.cpu().numpy().view(np.uint32).reshape(self.n, 3)
        return dict(
            **extra,
            res=res,
            n_sec_total=self.n_sec(),
            sec_event=self.sec_event[:k].cpu().numpy().view(np.uint32),
            sec_species=self.sec_species[:k].cpu().numpy(),
            sec_stage=self.sec_stage[:k].cpu().numpy(),
            sec_T=self.sec_T[:k].cpu().numpy(),
            sec_u=np.stack(
                [self.sec_ux[:k].cpu().numpy(), self.sec_uy[:k].cpu().numpy(), self.sec_uz[:k].cpu().numpy()], axis=1
            ),
        )


class Context:
    """Resident nucleus, cross-section and binding tables for a set of target
    nuclei on the current device (inc_ctx_create)."""

    def __init__(self, targets: Sequence[Sequence[int]], **options):
        L = _lib.load()
        self.targets = [(int(a), int(z)) for a, z in targets]
        arr = (_lib.Nucleus * len(self.targets))(*[_lib.Nucleus(a, z) for a, z in self.targets])
        opt = _lib.Options()
        known = {f[0] for f in _lib.Options._fields_} | {"fixed_b"}
        for k, v in options.items():
            if k not in known:
                raise TypeError("unknown Context option %r" % k)
            if k == "fixed_b" and v is not None:
                opt.fixed_b_on = 1
                opt.fixed_b = float(v)
            elif v is not None:
                setattr(opt, k, v)
        self.options = dict(options)
        h = C.c_void_p()
        _lib.check(L.inc_ctx_create(arr, len(self.targets), C.byref(opt), C.byref(h)), "inc_ctx_create")
        self._h = h
        self.max_A = max(a for a, _ in self.targets)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.load().inc_ctx_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tables(self) -> np.ndarray:
        """Shell tables per target: (n_targets, 108) floats (see inc.h)."""
        out = np.zeros((len(self.targets), 108), dtype=np.float32)
        _lib.check(_lib.load().inc_ctx_tables(self._h, out.ctypes.data), "inc_ctx_tables")
        return out

    def xs_table(self) -> dict:
        """The context's NN elastic table (inc_ctx_xs_table): node momenta
        p_lab (GeV/c, float64 from the float32 grid ends) and per column
        (unlike, like) sigma (mb), its suffix maximum and the slope b."""
        L = _lib.load()
        n, lo, hi = C.c_int(), C.c_float(), C.c_float()
        _lib.check(L.inc_ctx_xs_table(self._h, None, C.byref(n), C.byref(lo), C.byref(hi)), "inc_ctx_xs_table")
        buf = np.zeros(6 * n.value, dtype=np.float32)
        _lib.check(L.inc_ctx_xs_table(self._h, buf.ctypes.data, C.byref(n), C.byref(lo), C.byref(hi)),
                   "inc_ctx_xs_table")
        t = buf.reshape(3, 2, n.value)
        k = np.arange(n.value, dtype=np.float64)
        p = float(lo.value) * np.exp(np.log(float(hi.value) / float(lo.value)) * k / (n.value - 1))
        return dict(p=p, p_lo=float(lo.value), p_hi=float(hi.value), sigma=t[0], sigma_max=t[1], slope=t[2])

    def default_capacity(self, n: int) -> int:
        """Secondary records to allocate for n events: above the mean
        multiplicity of every real target up to 250 MeV (about 4.6 for 16O,
        5.8 for 40Ca, 15 for A = 250), at most A + 1 per event.  A call that
        needs more reports the required total (counters[0]); allocate that and
        run again."""
        per_event = min(self.max_A + 1, 6 + self.max_A // 10)
        if self.options.get("photon_evaporation"):
            per_event += 12  # photons leave A and Z: a few per event on top
        return int(n * per_event) + 4096

    def simulate(self, T0, seed: int, target_idx=None, first_event_id: int = 0, mode: str = "staged",
                 out: Optional[DeviceOutput] = None, capacity: Optional[int] = None, stream=None) -> DeviceOutput:
        """Generate len(T0) non-elastic events asynchronously on `stream`
        (default: torch's current stream).  T0: float32 cuda tensor (MeV);
        target_idx: uint8 cuda tensor or None."""
        return self._simulate("inc_simulate_dev", T0, seed, target_idx, first_event_id, mode, out, capacity, stream)

    def simulate_noalloc(self, T0, seed: int, out: DeviceOutput, target_idx=None, first_event_id: int = 0,
                         mode: str = "staged", capacity: Optional[int] = None, stream=None) -> DeviceOutput:
        """inc_simulate_dev_noalloc: as simulate(), into the caller's `out`,
        with the library's static workspace (no device allocation; at most
        NOALLOC_MAX_EVENTS events; calls on one device must not overlap)."""
        if out is None:
            raise TypeError("simulate_noalloc needs caller-allocated output buffers")
        return self._simulate("inc_simulate_dev_noalloc", T0, seed, target_idx, first_event_id, mode, out, capacity,
                              stream)

    def _simulate(self, entry, T0, seed, target_idx, first_event_id, mode, out, capacity, stream):
        torch = _torch()
        if not (torch.is_tensor(T0) and T0.is_cuda and T0.dtype == torch.float32 and T0.is_contiguous()):
            raise TypeError("T0 must be a contiguous float32 CUDA tensor")
        n = int(T0.shape[0])
        if target_idx is not None:
            if not (target_idx.is_cuda and target_idx.dtype == torch.uint8 and target_idx.shape[0] == n
                    and target_idx.is_contiguous()):
                raise TypeError("target_idx must be a contiguous uint8 CUDA tensor of len(T0)")
        if out is None:
            out = DeviceOutput.allocate(n, self.default_capacity(n) if capacity is None else capacity, T0.device)
        elif out.n < n:
            raise ValueError("output buffers hold %d events, batch has %d" % (out.n, n))
        b = _lib.Batch()
        b.n = n
        b.target_idx = target_idx.data_ptr() if target_idx is not None else None
        b.T0 = T0.data_ptr()
        b.seed = int(seed)
        b.first_event_id = int(first_event_id)
        o = out.c_struct(capacity)
        s = stream if stream is not None else torch.cuda.current_stream()
        m = MODES[mode]
        _lib.check(getattr(_lib.load(), entry)(self._h, C.byref(b), C.byref(o), C.c_void_p(s.cuda_stream), m), entry)
        return out

    def evaporate(self, A, Z, Ex, seed: int, P=None, first_event_id: int = 0, out: Optional[DeviceOutput] = None,
                  capacity: Optional[int] = None, stream=None) -> DeviceOutput:
        """Evaporate given excited nuclei asynchronously (inc_evaporate_dev).
        A, Z: int16 or uint16 CUDA tensors; Ex: float32 CUDA tensor (MeV);
        P: float32 CUDA tensor of shape (n, 3) (MeV/c) or None (at rest).
        The default capacity allows min(A + 1, 4 + A / 4) fragments per
        nucleus for the context's heaviest target; out.n_sec() above
        out.capacity means records were dropped: allocate that many and run
        again."""
        torch = _torch()
        n = int(Ex.shape[0]) if torch.is_tensor(Ex) else -1
        for name, t, dts in (("A", A, (torch.int16, torch.uint16)), ("Z", Z, (torch.int16, torch.uint16)),
                             ("Ex", Ex, (torch.float32,))):
            if not (torch.is_tensor(t) and t.is_cuda and t.dtype in dts and t.is_contiguous() and t.dim() == 1
                    and int(t.shape[0]) == n):
                raise TypeError("%s must be a contiguous 1-D CUDA tensor of %s and len(Ex)" % (name, dts))
        if P is not None and not (torch.is_tensor(P) and P.is_cuda and P.dtype == torch.float32 and P.is_contiguous()
                                  and tuple(P.shape) == (n, 3)):
            raise TypeError("P must be a contiguous float32 CUDA tensor of shape (len(Ex), 3)")
        if out is None:
            per = min(self.max_A + 1, 4 + self.max_A // 4) + (12 if self.options.get("photon_evaporation") else 0)
            cap = per * n + 4096 if capacity is None else capacity
            out = DeviceOutput.allocate(n, cap, Ex.device)
        elif out.n < n:
            raise ValueError("output buffers hold %d nuclei, batch has %d" % (out.n, n))
        x = _lib.Excited()
        x.n = n
        x.A = A.data_ptr()
        x.Z = Z.data_ptr()
        x.Ex = Ex.data_ptr()
        x.P = P.data_ptr() if P is not None else None
        x.seed = int(seed)
        x.first_event_id = int(first_event_id)
        o = out.c_struct(capacity)
        s = stream if stream is not None else torch.cuda.current_stream()
        _lib.check(_lib.load().inc_evaporate_dev(self._h, C.byref(x), C.byref(o), C.c_void_p(s.cuda_stream)),
                   "inc_evaporate_dev")
        return out


    def tally_shape(self):
        """(n_targets, amax, zmax) of the residual-nuclide table (inc_ctx_tally_shape)."""
        t, a, z = C.c_int(), C.c_int(), C.c_int()
        _lib.check(_lib.load().inc_ctx_tally_shape(self._h, C.byref(t), C.byref(a), C.byref(z)), "inc_ctx_tally_shape")
        return t.value, a.value, z.value

    def tally(self, T0, out: DeviceOutput, target_idx=None, n_ebins: int = 1, table=None, stream=None):
        """Residual-nuclide counts of a generated batch (inc_tally_residuals):
        an int64 CUDA tensor (n_targets, n_ebins, zmax + 1, amax + 1) indexed
        [target, energy bin over 20-250 MeV, Z_f, A_f]; `table` accumulates."""
        torch = _torch()
        nt, amax, zmax = self.tally_shape()
        shape = (nt, int(n_ebins), zmax + 1, amax + 1)
        if table is None:
            table = torch.zeros(shape, dtype=torch.int64, device=T0.device)
        elif tuple(table.shape) != shape or table.dtype != torch.int64 or not table.is_contiguous():
            raise ValueError("table must be a contiguous int64 tensor of shape %s" % (shape,))
        b = _lib.Batch()
        b.n = int(T0.shape[0])
        b.target_idx = target_idx.data_ptr() if target_idx is not None else None
        b.T0 = T0.data_ptr()
        s = stream if stream is not None else torch.cuda.current_stream()
        _lib.check(_lib.load().inc_tally_residuals(self._h, C.byref(b), C.c_void_p(out.res.data_ptr()), int(n_ebins),
                                                   C.c_void_p(table.data_ptr()), C.c_void_p(s.cuda_stream)),
                   "inc_tally_residuals")
        return table


MODES = {"plain": MODE_PLAIN, "persistent": MODE_PERSISTENT, "staged": MODE_STAGED, "vertex": MODE_VERTEX}


# Positron emitters reachable from tissue nuclei (C, N, O, P, Ca) by
# nucleon and light-fragment removal: (A, Z) -> (name, half-life in s).
POSITRON_EMITTERS = {
    (10, 6): ("10C", 19.29), (11, 6): ("11C", 1221.8), (13, 7): ("13N", 597.9), (14, 8): ("14O", 70.62),
    (15, 8): ("15O", 122.24), (29, 15): ("29P", 4.142), (30, 15): ("30P", 149.9), (34, 17): ("34Cl", 1.527),
    (37, 19): ("37K", 1.226), (38, 19): ("38K", 458.2), (39, 20): ("39Ca", 0.8603),
}


def positron_yields(table, targets) -> dict:
    """Counts of each positron emitter per target and energy bin from a
    residual-nuclide table (numpy or torch, shape (n_targets, n_ebins, zmax+1,
    amax+1)): {(A_t, Z_t): {name: counts per energy bin}}."""
    t = table.cpu().numpy() if hasattr(table, "cpu") else np.asarray(table)
    out = {}
    for i, (a_t, z_t) in enumerate(targets):
        row = {}
        for (a, z), (name, _) in POSITRON_EMITTERS.items():
            if z < t.shape[2] and a < t.shape[3]:
                c = t[i, :, z, a]
                if c.sum() > 0:
                    row[name] = c.copy()
        out[(a_t, z_t)] = row
    return out


def simulate_host(A: int, Z: int, energies: np.ndarray, seed: int, capacity: Optional[int] = None) -> dict:
    """The synchronous host-array call inc_simulate(target_A, target_Z,
    energies, n_events, seed, out...).  Raises IncError on failure."""
    L = _lib.load()
    e = np.ascontiguousarray(energies, dtype=np.float32)
    n = e.shape[0]
    cap = n * min(A + 1, 6 + A // 10) + 4096 if capacity is None else int(capacity)
    res = np.zeros(n, dtype=RESIDUAL_DTYPE)
    ev = np.zeros(max(cap, 1), dtype=np.uint32)
    sp = np.zeros(max(cap, 1), dtype=np.uint8)
    st = np.zeros(max(cap, 1), dtype=np.uint8)
    T = np.zeros(max(cap, 1), dtype=np.float32)
    ux, uy, uz = (np.zeros(max(cap, 1), dtype=np.float32) for _ in range(3))
    nsec = C.c_size_t(0)
    rc = L.inc_simulate(A, Z, e.ctypes.data, n, seed, res.ctypes.data, ev.ctypes.data, sp.ctypes.data,
                        st.ctypes.data, T.ctypes.data, ux.ctypes.data, uy.ctypes.data, uz.ctypes.data, cap,
                        C.byref(nsec))
    k = min(nsec.value, cap)
    out = dict(res=res, n_sec_total=nsec.value, sec_event=ev[:k], sec_species=sp[:k], sec_stage=st[:k],
               sec_T=T[:k], sec_u=np.stack([ux[:k], uy[:k], uz[:k]], axis=1))
    if rc != _lib.INC_OK and rc != _lib.INC_ERR_CAPACITY:
        _lib.check(rc, "inc_simulate")
    out["rc"] = rc
    return out


class Server:
    """Continuous-batching serving loop over a Context (inc_server_*).

    submit() admits a host-side event batch when a slot and HBM budget are
    free (else returns None: retry later); poll()/wait() follow it; fetch()
    returns its results as host arrays and releases its memory."""

    def __init__(self, ctx: Context, hbm_budget: int = 2 << 30, max_slots: int = 4):
        self.ctx = ctx
        h = C.c_void_p()
        _lib.check(_lib.load().inc_server_create(ctx._h, int(hbm_budget), int(max_slots), C.byref(h)),
                   "inc_server_create")
        self._h = h
        self._keep = {}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.load().inc_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _request(T0, tidx, seed, first_event_id, capacity):
        T0 = np.ascontiguousarray(T0, dtype=np.float32)
        ti = None if tidx is None else np.ascontiguousarray(tidx, dtype=np.uint8)
        r = _lib.Request()
        r.n = T0.shape[0]
        r.T0 = T0.ctypes.data
        r.target_idx = ti.ctypes.data if ti is not None else None
        r.seed = int(seed)
        r.first_event_id = int(first_event_id)
        r.sec_capacity = int(capacity or 0)
        return r, (T0, ti)

    def submit(self, T0, seed: int, target_idx=None, first_event_id: int = 0, capacity: int = 0):
        r, keep = self._request(T0, target_idx, seed, first_event_id, capacity)
        t = C.c_uint64()
        rc = _lib.load().inc_server_submit(self._h, C.byref(r), C.byref(t))
        if rc == _lib.INC_ERR_BUSY:
            return None
        _lib.check(rc, "inc_server_submit")
        self._keep[t.value] = (int(r.n), int(capacity or self.ctx.default_capacity(r.n)))
        return t.value

    def poll(self, ticket: int) -> bool:
        rc = _lib.load().inc_server_poll(self._h, ticket)
        if rc < 0:
            _lib.check(rc, "inc_server_poll")
        return rc == 1

    def wait(self, ticket: int):
        rc = _lib.load().inc_server_wait(self._h, ticket)
        if rc < 0:
            _lib.check(rc, "inc_server_wait")

    def fetch(self, ticket: int) -> dict:
        n, cap = self._keep.pop(ticket)
        res = np.zeros(n, dtype=RESIDUAL_DTYPE)
        ev = np.zeros(cap, np.uint32)
        sp = np.zeros(cap, np.uint8)
        st = np.zeros(cap, np.uint8)
        T, ux, uy, uz = (np.zeros(cap, np.float32) for _ in range(4))
        nsec = C.c_ulonglong()
        lat = C.c_double()
        o = _lib.HostOutput(res.ctypes.data, ev.ctypes.data, sp.ctypes.data, st.ctypes.data, T.ctypes.data,
                            ux.ctypes.data, uy.ctypes.data, uz.ctypes.data, cap, C.pointer(nsec), C.pointer(lat))
        rc = _lib.load().inc_server_fetch(self._h, ticket, C.byref(o))
        if rc not in (_lib.INC_OK, _lib.INC_ERR_CAPACITY):
            _lib.check(rc, "inc_server_fetch")
        k = min(nsec.value, cap)
        return dict(rc=rc, res=res, n_sec_total=nsec.value, latency_s=lat.value, sec_event=ev[:k],
                    sec_species=sp[:k], sec_stage=st[:k], sec_T=T[:k], sec_u=np.stack([ux[:k], uy[:k], uz[:k]], 1))

    def stats(self) -> dict:
        """Counters and the native latency statistics (p50, p99, events/s)
        over the requests completed since creation or stats_reset()."""
        s = _lib.ServerStats()
        _lib.check(_lib.load().inc_server_stats_get(self._h, C.byref(s)), "inc_server_stats_get")
        return {f: getattr(s, f) for f, _ in s._fields_}

    def stats_reset(self):
        _lib.check(_lib.load().inc_server_stats_reset(self._h), "inc_server_stats_reset")

    def hold(self, on: bool = True):
        """Queue admitted requests without launching them (on), or release
        the queue (off): a burst submitted while held goes out in as few
        launches as possible."""
        _lib.check(_lib.load().inc_server_hold(self._h, int(bool(on))), "inc_server_hold")

    def replay(self, arrivals_s, requests):
        """Native request loop.  requests: list of dicts with T0, target_idx,
        seed, first_event_id.  Returns (latency per request in s, span s)."""
        arr = np.ascontiguousarray(arrivals_s, dtype=np.float64)
        reqs = (_lib.Request * len(requests))()
        keep = []
        for i, q in enumerate(requests):
            r, k = self._request(q["T0"], q.get("target_idx"), q["seed"], q.get("first_event_id", 0),
                                 q.get("capacity", 0))
            reqs[i] = r
            keep.append(k)
        lat = np.zeros(len(requests), dtype=np.float64)
        span = C.c_double()
        _lib.check(_lib.load().inc_server_replay(self._h, len(requests), arr.ctypes.data, C.addressof(reqs),
                                                 lat.ctypes.data, C.byref(span)), "inc_server_replay")
        return lat, span.value


class Ring:
    """Streaming output through a bounded ring of `slots` records
    (inc_ring_*): the secondaries of a batch are drained to host arrays while
    the kernel runs.  placement "host": the ring in coherent host memory
    (inc_ring_create); "device": in device memory, drained chunk by chunk
    (`chunk` slots) by asynchronous copies (inc_ring_create_device)."""

    def __init__(self, ctx: Context, slots: int = 1 << 20, placement: str = "device", chunk: int = 1 << 16):
        self.ctx = ctx
        h = C.c_void_p()
        if placement == "host":
            _lib.check(_lib.load().inc_ring_create(ctx._h, int(slots), C.byref(h)), "inc_ring_create")
        elif placement == "device":
            _lib.check(_lib.load().inc_ring_create_device(ctx._h, int(slots), int(chunk), C.byref(h)),
                       "inc_ring_create_device")
        else:
            raise ValueError("placement must be 'host' or 'device'")
        self._h = h
        self.slots = int(slots)
        self.placement = placement

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib.load().inc_ring_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def host_buffers(capacity: int, n_events: int = 0) -> dict:
        """Host arrays for `capacity` secondaries (written once, so that a
        later drain into them takes no first-touch page faults) and, with
        n_events, pinned host memory for that many residuals (their copy then
        overlaps the drain); pass them to simulate(out=...) to reuse them
        across batches."""
        out = dict(ev=np.zeros(capacity, np.uint32), sp=np.zeros(capacity, np.uint8),
                   st=np.zeros(capacity, np.uint8), T=np.zeros(capacity, np.float32),
                   ux=np.zeros(capacity, np.float32), uy=np.zeros(capacity, np.float32),
                   uz=np.zeros(capacity, np.float32))
        for a in out.values():
            a.fill(0)
        if n_events:
            torch = _torch()
            pinned = torch.zeros(int(n_events) * RESIDUAL_DTYPE.itemsize, dtype=torch.uint8, pin_memory=True)
            out["res_pinned"] = pinned  # keeps the allocation alive
            out["res"] = pinned.numpy().view(RESIDUAL_DTYPE)
        return out

    def simulate(self, T0, seed: int, target_idx=None, first_event_id: int = 0, mode: str = "staged",
                 capacity: Optional[int] = None, stream=None, out: Optional[dict] = None) -> dict:
        """T0 / target_idx: CUDA tensors as in Context.simulate.  Returns host
        arrays of the secondaries and residuals (views of `out` when given,
        see host_buffers) and the ring statistics."""
        torch = _torch()
        n = int(T0.shape[0])
        if out is not None:
            cap = int(out["T"].shape[0])
        else:
            cap = int(capacity) if capacity is not None else self.ctx.default_capacity(n)
            out = dict(ev=np.zeros(cap, np.uint32), sp=np.zeros(cap, np.uint8), st=np.zeros(cap, np.uint8),
                       T=np.zeros(cap, np.float32), ux=np.zeros(cap, np.float32), uy=np.zeros(cap, np.float32),
                       uz=np.zeros(cap, np.float32))
        res_d = torch.empty(n * 32, dtype=torch.uint8, device=T0.device)
        ev, sp, st, T, ux, uy, uz = (out[k] for k in ("ev", "sp", "st", "T", "ux", "uy", "uz"))
        res_h = out.get("res")
        if res_h is None or res_h.shape[0] < n:
            res_h = np.empty(n, RESIDUAL_DTYPE)
        nsec = C.c_ulonglong()
        o = _lib.HostOutput(res_h.ctypes.data, ev.ctypes.data, sp.ctypes.data, st.ctypes.data, T.ctypes.data,
                            ux.ctypes.data, uy.ctypes.data, uz.ctypes.data, cap, C.pointer(nsec), None)
        b = _lib.Batch()
        b.n = n
        b.target_idx = target_idx.data_ptr() if target_idx is not None else None
        b.T0 = T0.data_ptr()
        b.seed = int(seed)
        b.first_event_id = int(first_event_id)
        stats = _lib.RingStats()
        s = stream if stream is not None else torch.cuda.current_stream()
        m = MODES[mode]
        rc = _lib.load().inc_ring_simulate(self._h, C.byref(b), C.c_void_p(res_d.data_ptr()), C.byref(o),
                                           C.c_void_p(s.cuda_stream), m, C.byref(stats))
        if rc not in (_lib.INC_OK, _lib.INC_ERR_CAPACITY):
            _lib.check(rc, "inc_ring_simulate")
        k = min(nsec.value, cap)
        return dict(rc=rc, res=res_h[:n], n_sec_total=nsec.value,
                    sec_event=ev[:k], sec_species=sp[:k], sec_stage=st[:k], sec_T=T[:k],
                    sec_ux=ux[:k], sec_uy=uy[:k], sec_uz=uz[:k],
                    stats={f: getattr(stats, f) for f, _ in stats._fields_})


    def stream(self, T0, seed: int, consumer, target_idx=None, first_event_id: int = 0, mode: str = "staged",
               res=None, stream=None) -> dict:
        """Generate len(T0) events and hand their secondaries to
        consumer(chunk) run by run as they leave the ring
        (inc_ring_simulate_to).  chunk: dict with "first" (index of the run's
        first record in the batch's output sequence) and numpy views "event",
        "species", "stage", "T", "ux", "uy", "uz" into the ring, valid only
        during the call (copy what you keep).  res: host RESIDUAL_DTYPE array
        of len(T0) (pinned memory lets its copy overlap the drain) or None.
        The kernel may be waiting for the consumer: it must not synchronise
        with the device or release device objects (Python's cyclic garbage
        collector is paused for the call).  Returns the record count and the
        ring statistics; an exception the consumer raised is re-raised after
        the drain."""
        torch = _torch()
        n = int(T0.shape[0])
        if res is not None and (res.dtype != RESIDUAL_DTYPE or res.shape[0] < n):
            raise TypeError("res must be a RESIDUAL_DTYPE array of at least len(T0) records")
        errors = []

        def on_chunk(cp, _user):
            if errors:
                return
            c = cp.contents
            m = int(c.n)
            view = lambda ptr: np.ctypeslib.as_array(ptr, shape=(m,))
            kind = view(c.kind)
            try:
                consumer(dict(first=int(c.first), event=view(c.event), species=(kind & 0xFF).astype(np.uint8),
                              stage=((kind >> 8) & 0xFF).astype(np.uint8), T=view(c.T), ux=view(c.ux),
                              uy=view(c.uy), uz=view(c.uz)))
            except BaseException as e:  # noqa: BLE001  (reported after the drain)
                errors.append(e)

        cb = _lib.RING_CONSUMER(on_chunk)
        res_d = torch.empty(n * 32, dtype=torch.uint8, device=T0.device)
        b = _lib.Batch()
        b.n = n
        b.target_idx = target_idx.data_ptr() if target_idx is not None else None
        b.T0 = T0.data_ptr()
        b.seed = int(seed)
        b.first_event_id = int(first_event_id)
        stats = _lib.RingStats()
        nsec = C.c_ulonglong()
        s = stream if stream is not None else torch.cuda.current_stream()
        # The consumer runs while the kernel may wait for it to drain: a
        # garbage-collection pass inside it could finalize an unrelated
        # object whose release waits on the device (a Context's hipFree), and
        # then neither side moves until the producer's bounded wait fails.
        gc_was_enabled = gc.isenabled()
        gc.disable()
        try:
            rc = _lib.load().inc_ring_simulate_to(self._h, C.byref(b), C.c_void_p(res_d.data_ptr()),
                                                  None if res is None else C.c_void_p(res.ctypes.data), cb, None,
                                                  C.byref(nsec), C.c_void_p(s.cuda_stream), MODES[mode],
                                                  C.byref(stats))
        finally:
            if gc_was_enabled:
                gc.enable()
        _lib.check(rc, "inc_ring_simulate_to")
        if errors:
            raise errors[0]
        return dict(n_sec_total=nsec.value, stats={f: getattr(stats, f) for f, _ in stats._fields_})


def contract_version() -> int:
    return _lib.load().inc_contract_version()
