"""Python binding of the C ABI with the same names and steps.

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch provides device memory (tensors passed by pointer) and the
stream the plan enqueues on.
"""
from __future__ import annotations

import ctypes as ct
import math
import weakref
from typing import Optional, Sequence, Tuple

import numpy as np

from . import _lib
from ._lib import check, lib

try:  # torch is the device-memory provider; imported lazily by callers that need it
    import torch
except Exception:  # pragma: no cover
    torch = None


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _i64ptr(a: np.ndarray):
    return a.ctypes.data_as(ct.POINTER(ct.c_int64))


def plan_desc(N: int, L: float = 2 * math.pi, prec: str = "f32", n_slots: int = 1,
              n_modes: int = 200, n_alpha: int = 50, u_min: float = 1e-3, u_max: float = 15.0,
              u_p: float = 1.0, sigma_p: float = 0.5, A_p: float = 10.0,
              alpha_chunk: int = 0, scratch_terms: int = 0, batch: int = 0,
              autotune: int = 0) -> _lib.PlanDesc:
    d = _lib.PlanDesc()
    d.N, d.L, d.prec, d.n_slots = N, L, _prec_code(prec), n_slots
    d.n_modes, d.n_alpha = n_modes, n_alpha
    d.u_min, d.u_max, d.u_p, d.sigma_p, d.A_p = u_min, u_max, u_p, sigma_p, A_p
    d.alpha_chunk = alpha_chunk
    d.scratch_terms = scratch_terms
    d.batch = batch
    d.autotune = autotune
    return d


def _prec_code(prec) -> int:
    if prec in ("f32", "fp32", "float32", _lib.SIGW_F32):
        return _lib.SIGW_F32
    if prec in ("f64", "fp64", "float64", _lib.SIGW_F64):
        return _lib.SIGW_F64
    raise ValueError(f"unknown precision {prec!r}")


def sigw_plan_footprint(desc: _lib.PlanDesc) -> int:
    out = ct.c_size_t(0)
    check(lib().sigw_plan_footprint(ct.byref(desc), ct.byref(out)), None, "sigw_plan_footprint")
    return int(out.value)


def sigw_kernel_table(desc: _lib.PlanDesc, m: int):
    """Host-only kernel table: (sigma[n_alpha], phi[n_modes, n_alpha], edges[n_modes+1])."""
    sigma = np.zeros(desc.n_alpha)
    phi = np.zeros((desc.n_modes, desc.n_alpha))
    edges = np.zeros(desc.n_modes + 1)
    check(lib().sigw_kernel_table(ct.byref(desc), m, _dptr(sigma), _dptr(phi), _dptr(edges)),
          None, "sigw_kernel_table")
    return sigma, phi, edges


def sigw_stream_probe(kind: int, nbytes: int = 1 << 30, reps: int = 5) -> float:
    """GB/s of the streaming probe kind (0 read, 1 write, 2 copy, 3 2-read:3-write)
    over arrays of nbytes each, in a buffer that torch allocates."""
    arrays = (1, 1, 2, 5)[kind]
    buf = torch.empty(arrays * nbytes + (32 << 10), dtype=torch.uint8, device="cuda")
    buf.zero_()
    out = ct.c_double(0.0)
    s = torch.cuda.current_stream()
    check(lib().sigw_stream_probe(int(kind), ct.c_void_p(buf.data_ptr()), nbytes, int(reps),
                                  ct.c_void_p(s.cuda_stream), ct.byref(out)), None, "sigw_stream_probe")
    del buf
    return out.value


def sigw_kernel_table_w(desc: _lib.PlanDesc, w: float, m: int):
    """Host-only table for a constant equation of state w:
    (sigma[n_alpha], phi[n_modes, n_alpha], edges[n_modes+1])."""
    sigma = np.zeros(desc.n_alpha)
    phi = np.zeros((desc.n_modes, desc.n_alpha))
    edges = np.zeros(desc.n_modes + 1)
    check(lib().sigw_kernel_table_w(ct.byref(desc), float(w), m, _dptr(sigma), _dptr(phi), _dptr(edges)),
          None, "sigw_kernel_table_w")
    return sigma, phi, edges


def sigw_spectrum_noalloc(desc: _lib.PlanDesc, phi_hat, targets, k_lo, k_hi, stream=None):
    """Allocation-free spectrum of one realisation given as a device half
    spectrum (torch tensor of the path's complex dtype): (omega, nmodes).
    No plan; all device state lives in the library's static per-GPU buffer."""
    t = np.ascontiguousarray(targets, dtype=np.float64)
    lo = np.ascontiguousarray(k_lo, dtype=np.float64)
    hi = np.ascontiguousarray(k_hi, dtype=np.float64)
    om = np.zeros(len(t))
    nb = np.zeros(len(t), dtype=np.int64)
    s = stream if stream is not None else torch.cuda.current_stream()
    st = lib().sigw_spectrum_noalloc(ct.byref(desc), ct.c_void_p(phi_hat.data_ptr()), len(t), _dptr(t), _dptr(lo),
                                     _dptr(hi), _dptr(om), _i64ptr(nb), ct.c_void_p(s.cuda_stream))
    check(st, None, "sigw_spectrum_noalloc")
    return om, nb


def lognormal_struct(spec) -> _lib.Lognormal:
    s = _lib.Lognormal()
    s.A, s.sigma, s.k_star = float(spec.A), float(spec.sigma), float(spec.k_star)
    return s


def ngmap_struct(m) -> _lib.NGMap:
    s = _lib.NGMap()
    s.kind = _lib.MAP_KINDS[m.kind] if isinstance(m.kind, str) else int(m.kind)
    s.F_NL, s.G_NL = float(getattr(m, "F_NL", 0.0)), float(getattr(m, "G_NL", 0.0))
    s.beta, s.clip = float(getattr(m, "beta", 0.0)), float(getattr(m, "clip", 1e-6))
    s.alpha_NL, s.beta_NL = float(getattr(m, "alpha_NL", 0.0)), float(getattr(m, "beta_NL", 0.0))
    s.k_NL = float(getattr(m, "k_NL", 0.0))
    return s


class Plan:
    """Owns one sigw_plan_t.  Device tensors are torch tensors on cuda:0."""

    def __init__(self, N: int, L: float = 2 * math.pi, prec: str = "f32", n_slots: int = 1,
                 stream=None, **decomp):
        if torch is None or not torch.cuda.is_available():
            raise RuntimeError("a GPU is required: the HIP library has no CPU path")
        self.desc = plan_desc(N, L, prec, n_slots, **decomp)
        self.N, self.L, self.n_slots = N, L, n_slots
        self.prec = _prec_code(prec)
        self.rdtype = torch.float32 if self.prec == _lib.SIGW_F32 else torch.float64
        self.cdtype = torch.complex64 if self.prec == _lib.SIGW_F32 else torch.complex128
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ct.c_void_p()
        st = lib().sigw_plan_create(ct.byref(self.desc), ct.c_void_p(self.stream.cuda_stream),
                                    ct.byref(h))
        check(st, None, f"sigw_plan_create(N={N}, prec={prec})")
        self.h = h
        self._graphs = weakref.WeakSet()     # live graphs: destroyed before the plan

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            for g in list(getattr(self, "_graphs", ())):
                g.close()
            lib().sigw_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def half_shape(self):
        return (self.N // 2 + 1, self.N, self.N)

    def _chk(self, st, what):
        check(st, self.h, what)

    # -- fields -----------------------------------------------------------
    def white_noise(self, seed: int):
        out = torch.empty((self.N,) * 3, dtype=self.rdtype, device="cuda")
        self._chk(lib().sigw_white_noise(self.h, ct.c_uint64(seed), ct.c_void_p(out.data_ptr())),
                  "sigw_white_noise")
        return out

    def generate_field(self, slot: int, seed: int, spectrum, ngmap):
        ls, ms = lognormal_struct(spectrum), ngmap_struct(ngmap)
        self._chk(lib().sigw_generate_field(self.h, slot, ct.c_uint64(seed), ct.byref(ls),
                                            ct.byref(ms)), "sigw_generate_field")

    def set_zeta(self, slot: int, zeta):
        z = zeta.to(device="cuda", dtype=self.rdtype).contiguous()
        self._chk(lib().sigw_set_zeta(self.h, slot, ct.c_void_p(z.data_ptr())), "sigw_set_zeta")
        self.synchronize()

    def set_phi_hat(self, slot: int, phi_hat):
        t = phi_hat.to(device="cuda", dtype=self.cdtype).contiguous()
        assert tuple(t.shape) == self.half_shape
        self._chk(lib().sigw_set_phi_hat(self.h, slot, ct.c_void_p(t.data_ptr())), "sigw_set_phi_hat")
        self.synchronize()

    def get_phi_hat(self, slot: int):
        out = torch.empty(self.half_shape, dtype=self.cdtype, device="cuda")
        self._chk(lib().sigw_get_phi_hat(self.h, slot, ct.c_void_p(out.data_ptr())), "sigw_get_phi_hat")
        self.synchronize()
        return out

    # -- the per-target path --------------------------------------------------
    def source_convolutions(self, slot: int, k_target: float):
        out = torch.empty((2, 6) + self.half_shape, dtype=self.cdtype, device="cuda")
        self._chk(lib().sigw_source_convolutions(self.h, slot, float(k_target),
                                                 ct.c_void_p(out.data_ptr())),
                  "sigw_source_convolutions")
        self.synchronize()
        return out

    def spectrum(self, slot: int, targets, k_lo, k_hi) -> Tuple[np.ndarray, np.ndarray]:
        om, nb = self.spectrum_batch([slot], targets, k_lo, k_hi)
        return om[0], nb[0]

    def spectrum_batch(self, slots: Sequence[int], targets, k_lo, k_hi):
        t = np.ascontiguousarray(targets, dtype=np.float64)
        lo = np.ascontiguousarray(k_lo, dtype=np.float64)
        hi = np.ascontiguousarray(k_hi, dtype=np.float64)
        sl = np.ascontiguousarray(slots, dtype=np.int32)
        om = np.zeros((len(sl), len(t)))
        nb = np.zeros((len(sl), len(t)), dtype=np.int64)
        st = lib().sigw_spectrum_batch(self.h, len(sl), sl.ctypes.data_as(ct.POINTER(ct.c_int32)),
                                       len(t), _dptr(t), _dptr(lo), _dptr(hi), _dptr(om), _i64ptr(nb))
        self._chk(st, "sigw_spectrum_batch")
        return om, nb

    def spectrum_jackknife(self, slot: int, targets, k_lo, k_hi, M: int = 4):
        """(omega, nmodes, omega_err, replicas[n_k, M^3]) with jackknife errors."""
        t = np.ascontiguousarray(targets, dtype=np.float64)
        lo = np.ascontiguousarray(k_lo, dtype=np.float64)
        hi = np.ascontiguousarray(k_hi, dtype=np.float64)
        n = len(t)
        om, err = np.zeros(n), np.zeros(n)
        nb = np.zeros(n, dtype=np.int64)
        rep = np.zeros((n, M ** 3))
        st = lib().sigw_spectrum_jackknife(self.h, slot, n, _dptr(t), _dptr(lo), _dptr(hi), int(M), _dptr(om),
                                           _i64ptr(nb), _dptr(err), _dptr(rep))
        self._chk(st, "sigw_spectrum_jackknife")
        return om, nb, err, rep

    def spectrum_adaptive(self, slot: int, seed: int, spectrum, ngmap, targets, eps: float = 0.1):
        """Per-target box protocol: (omega, nmodes, box side L) per target."""
        t = np.ascontiguousarray(targets, dtype=np.float64)
        n = len(t)
        om, box = np.zeros(n), np.zeros(n)
        nb = np.zeros(n, dtype=np.int64)
        ls, ms = lognormal_struct(spectrum), ngmap_struct(ngmap)
        st = lib().sigw_spectrum_adaptive(self.h, slot, ct.c_uint64(seed), ct.byref(ls), ct.byref(ms), n, _dptr(t),
                                          float(eps), _dptr(om), _i64ptr(nb), _dptr(box))
        self._chk(st, "sigw_spectrum_adaptive")
        return om, nb, box

    def spectrum_enqueue(self, slot: int, targets, k_lo, k_hi):
        self._pend = (np.ascontiguousarray(targets, dtype=np.float64),
                      np.ascontiguousarray(k_lo, dtype=np.float64),
                      np.ascontiguousarray(k_hi, dtype=np.float64))
        t, lo, hi = self._pend
        self._chk(lib().sigw_spectrum_enqueue(self.h, slot, len(t), _dptr(t), _dptr(lo), _dptr(hi)),
                  "sigw_spectrum_enqueue")

    def spectrum_poll(self) -> Optional[Tuple[np.ndarray, np.ndarray]]:
        n = len(self._pend[0])
        om = np.zeros(n)
        nb = np.zeros(n, dtype=np.int64)
        st = lib().sigw_spectrum_poll(self.h, _dptr(om), _i64ptr(nb))
        if st == _lib.SIGW_E_PENDING:
            return None
        self._chk(st, "sigw_spectrum_poll")
        return om, nb

    def graph(self, slots: Sequence[int], targets, k_lo, k_hi) -> "SpectrumGraph":
        return SpectrumGraph(self, slots, targets, k_lo, k_hi)

    # -- kernel tables --------------------------------------------------------
    def set_kernel_table(self, m: int, sigma, phi, edges=None):
        """Use the caller's separable table for kernel m (0 = I_s, 1 = I_c):
        sigma[n_alpha], phi[n_modes, n_alpha], and optionally a new u grid
        edges[n_modes + 1] shared by both kernels."""
        s = np.ascontiguousarray(sigma, dtype=np.float64)
        f = np.ascontiguousarray(phi, dtype=np.float64)
        e = None if edges is None else np.ascontiguousarray(edges, dtype=np.float64)
        d = self.desc
        if s.shape != (d.n_alpha,) or f.shape != (d.n_modes, d.n_alpha) or (
                e is not None and e.shape != (d.n_modes + 1,)):
            raise ValueError("table shapes must be sigma[n_alpha], phi[n_modes, n_alpha], edges[n_modes + 1]")
        self._chk(lib().sigw_plan_set_kernel_table(self.h, int(m), _dptr(s), _dptr(f),
                                                   None if e is None else _dptr(e)),
                  "sigw_plan_set_kernel_table")

    def set_equation_of_state(self, w: float):
        """Install the kernel tables of a constant equation of state w (both
        kernels, on this plan's grid)."""
        for m in (0, 1):
            self.set_kernel_table(m, *sigw_kernel_table_w(self.desc, w, m))

    # -- x-pass schedule ------------------------------------------------------
    def autotune(self, force: bool = False) -> str:
        self._chk(lib().sigw_autotune(self.h, _lib.SIGW_TUNE_FORCE if force else 0), "sigw_autotune")
        return self.schedule()[2]

    def schedule(self):
        """(index, count, text) of the active x-pass schedule."""
        idx, cnt = ct.c_int32(0), ct.c_int32(0)
        buf = ct.create_string_buffer(512)
        self._chk(lib().sigw_plan_schedule(self.h, ct.byref(idx), ct.byref(cnt), buf, len(buf)),
                  "sigw_plan_schedule")
        return idx.value, cnt.value, buf.value.decode()

    def set_schedule(self, index: int):
        self._chk(lib().sigw_plan_set_schedule(self.h, int(index)), "sigw_plan_set_schedule")

    # -- timing --------------------------------------------------------------
    def set_timing(self, on: bool):
        self._chk(lib().sigw_set_timing(self.h, 1 if on else 0), "sigw_set_timing")

    def kernel_time(self, name: str):
        ms = ct.c_double(0.0)
        n = ct.c_int64(0)
        self._chk(lib().sigw_kernel_time(self.h, name.encode(), ct.byref(ms), ct.byref(n)),
                  "sigw_kernel_time")
        return ms.value, n.value

    def synchronize(self):
        self._chk(lib().sigw_synchronize(self.h), "sigw_synchronize")


class SpectrumGraph:
    """A captured batched spectrum (sigw_graph_t): replay it after refilling
    the same slots with new fields."""

    def __init__(self, plan: Plan, slots, targets, k_lo, k_hi):
        self.plan = plan
        self.t = np.ascontiguousarray(targets, dtype=np.float64)
        self.lo = np.ascontiguousarray(k_lo, dtype=np.float64)
        self.hi = np.ascontiguousarray(k_hi, dtype=np.float64)
        self.sl = np.ascontiguousarray(slots, dtype=np.int32)
        h = ct.c_void_p()
        st = lib().sigw_graph_create(plan.h, len(self.sl), self.sl.ctypes.data_as(ct.POINTER(ct.c_int32)),
                                     len(self.t), _dptr(self.t), _dptr(self.lo), _dptr(self.hi),
                                     ct.byref(h))
        check(st, plan.h, "sigw_graph_create")
        self.h = h
        plan._graphs.add(self)

    def launch(self):
        check(lib().sigw_graph_launch(self.h), self.plan.h, "sigw_graph_launch")

    def results(self):
        om = np.zeros((len(self.sl), len(self.t)))
        nb = np.zeros((len(self.sl), len(self.t)), dtype=np.int64)
        check(lib().sigw_graph_results(self.h, _dptr(om), _i64ptr(nb)), self.plan.h, "sigw_graph_results")
        return om, nb

    def close(self):
        if getattr(self, "h", None):
            lib().sigw_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
