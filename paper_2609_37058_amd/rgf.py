"""Python binding of librgf (ctypes): argument marshalling only.

Every step of the transmission path runs in the HIP library; this module
only turns torch tensors (device memory) and streams into the C-ABI
structs of ``include/rgf.h``.  It raises if the library is missing: there
is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librgf.so")

RGF_FP64, RGF_MIXED = 0, 1
RGF_LEFT, RGF_RIGHT = 0, 1
RGF_OK, RGF_EINVAL, RGF_ENOMEM, RGF_EDEVICE, RGF_EAGAIN, RGF_ETOOBIG, RGF_ENOTICKET = 0, -1, -2, -3, -4, -5, -6
INFO_SR_LEFT, INFO_SR_RIGHT, INFO_SINGULAR, INFO_NONFINITE = 1, 2, 4, 8
PRECISION = {"fp64": RGF_FP64, "mixed": RGF_MIXED, RGF_FP64: RGF_FP64, RGF_MIXED: RGF_MIXED}


class RgfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"librgf error {code}: {msg}")
        self.code = code


class rgf_lead(C.Structure):
    _fields_ = [("M", C.c_int32), ("H00", C.c_void_p), ("H01", C.c_void_p), ("S00", C.c_void_p),
                ("S01", C.c_void_p)]


class rgf_device(C.Structure):
    _fields_ = [("N", C.c_int32), ("M", C.c_int32), ("Hd", C.c_void_p), ("Hu", C.c_void_p),
                ("Sd", C.c_void_p), ("Su", C.c_void_p), ("left", rgf_lead), ("right", rgf_lead)]


class rgf_server_opts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("lead_cache_bytes", C.c_uint64), ("max_slots", C.c_int32)]


class rgf_server_stats(C.Structure):
    _fields_ = [("finished", C.c_uint64), ("cache_hits", C.c_uint64), ("cache_misses", C.c_uint64),
                ("peak_inflight_bytes", C.c_uint64), ("cache_bytes", C.c_uint64), ("admitted_ahead", C.c_uint64)]


_lib = None

#: every symbol include/rgf.h declares, with (restype, argtypes)
SIGNATURES = {
    "rgf_transmission": (C.c_int, [C.POINTER(rgf_device), C.c_void_p, C.c_int64, C.c_double, C.c_int,
                                   C.c_void_p, C.c_void_p, C.c_void_p]),
    "lead_self_energy": (C.c_int, [C.POINTER(rgf_lead), C.c_int, C.c_void_p, C.c_int64, C.c_double, C.c_int,
                                   C.c_void_p, C.c_void_p, C.c_void_p]),
    "transport_open": (C.c_int, [C.POINTER(rgf_server_opts), C.POINTER(C.c_void_p)]),
    "transport_submit": (C.c_int, [C.c_void_p, C.POINTER(rgf_device), C.c_uint64, C.c_uint64, C.c_void_p,
                                   C.c_int64, C.c_double, C.c_int, C.POINTER(C.c_uint64)]),
    "transport_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "transport_close": (C.c_int, [C.c_void_p]),
    "transport_stats": (C.c_int, [C.c_void_p, C.POINTER(rgf_server_stats)]),
    "rgf_last_error": (C.c_char_p, []),
    "rgf_version": (C.c_char_p, []),
    "rgf_release_workspaces": (C.c_int, []),
    "rgf_profile": (C.c_int, [C.c_int]),
    "rgf_check_device": (C.c_int, [C.POINTER(rgf_device), C.c_double, C.POINTER(C.c_double), C.c_void_p]),
    "rgf_set_checks": (C.c_int, [C.c_int]),
    "rgf_get_checks": (C.c_int, []),
    "rgf_profile_read": (C.c_int, [C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "rgf_profile_classes": (C.c_int, [C.c_int, C.c_uint32]),
    "rgf_transmission_noalloc": (C.c_int, [C.POINTER(rgf_device), C.c_void_p, C.c_int64, C.c_double, C.c_int,
                                           C.c_void_p, C.c_void_p, C.c_void_p]),
    "rgf_set_sr_maxit": (C.c_int, [C.c_int32]),
    "rgf_get_sr_maxit": (C.c_int, []),
    "rgf_profile_read_class": (C.c_int, [C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                         C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "rgf_get_tile": (C.c_int, [C.c_int, C.POINTER(C.c_int32)]),
    "rgf_set_mixed_parts": (C.c_int, [C.c_int]),
    "rgf_get_mixed_parts": (C.c_int, []),
    "rgf_set_tile": (C.c_int, [C.c_int, C.c_int32]),
    "rgf_transmission_bias": (C.c_int, [C.POINTER(rgf_device), C.c_void_p, C.c_int64, C.c_double, C.c_double,
                                        C.c_double, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rgf_landauer_current": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_double, C.c_double,
                                       C.c_void_p, C.c_void_p]),
    "rgf_kpm_moments": (C.c_int, [C.POINTER(rgf_device), C.c_double, C.c_double, C.c_int32, C.c_void_p,
                                  C.c_int32, C.c_void_p, C.c_void_p]),
    "rgf_kpm_fermi": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_void_p,
                                C.c_void_p]),
    "rgf_kpm_dos": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_void_p, C.c_int64, C.c_void_p,
                              C.c_void_p]),
    "rgf_ldos": (C.c_int, [C.POINTER(rgf_device), C.c_void_p, C.c_int64, C.c_double, C.c_void_p, C.c_void_p,
                           C.c_void_p, C.c_void_p, C.c_void_p]),
    "rgf_transmission_kmesh": (C.c_int, [C.POINTER(rgf_device), C.c_int32, C.POINTER(C.c_int32),
                                         C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int32, C.c_void_p,
                                         C.c_int64, C.c_double, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p]),
    "rgf_set_graphs": (C.c_int, [C.c_int]),
    "rgf_get_graphs": (C.c_int, []),
    "rgf_get_tuning": (C.c_int, [C.c_int32, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "rgf_set_tuning": (C.c_int, [C.c_int32, C.c_int, C.c_int32, C.c_int32]),
    "rgf_autotune": (C.c_int, [C.c_int32, C.c_int, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                               C.POINTER(C.c_double)]),
    "rgf_transmission_batch": (C.c_int, [C.POINTER(rgf_device), C.c_int32, C.POINTER(C.c_void_p),
                                         C.POINTER(C.c_int64), C.c_double, C.c_int, C.POINTER(C.c_void_p),
                                         C.POINTER(C.c_void_p), C.c_void_p]),
}


def load(path: str = LIB_PATH):
    """Load librgf.so (built in-tree by ``paper_2609_37058_amd.build``); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2609_37058_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != RGF_OK:
        raise RgfError(rc, load().rgf_last_error().decode())


def _ptr(t: Optional[torch.Tensor], dtype: Optional[torch.dtype] = None, what: str = "tensor") -> Optional[int]:
    """Device address of a contiguous CUDA tensor, checked against the dtype the C call reads or
    writes through it (a float32 energy grid read as float64 would be an out-of-bounds access)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"librgf takes device tensors ({what} is on {t.device})")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {t.dtype}")
    return t.data_ptr()


_F64, _I32, _C128 = torch.float64, torch.int32, torch.complex128


def _energies(E: torch.Tensor) -> torch.Tensor:
    if not isinstance(E, torch.Tensor) or E.dtype != _F64:
        raise ValueError(f"energies must be a float64 device tensor, got {getattr(E, 'dtype', type(E))}")
    return E.contiguous()


def _stream(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


@dataclass
class LeadTensors:
    """One lead principal layer on the device (complex128 M x M each)."""
    H00: torch.Tensor
    H01: torch.Tensor
    S00: torch.Tensor
    S01: torch.Tensor

    @property
    def M(self) -> int:
        return self.H00.shape[-1]

    def cstruct(self) -> rgf_lead:
        for name in ("H00", "H01", "S00", "S01"):
            t = getattr(self, name)
            if t.shape != (self.M, self.M):
                raise ValueError(f"lead {name} must be {self.M} x {self.M}, got {tuple(t.shape)}")
        return rgf_lead(self.M, _ptr(self.H00, _C128, "H00"), _ptr(self.H01, _C128, "H01"),
                        _ptr(self.S00, _C128, "S00"), _ptr(self.S01, _C128, "S01"))


@dataclass
class DeviceTensors:
    """A block-tridiagonal device on the GPU: Hd, Sd [N, M, M]; Hu, Su [N-1, M, M] (complex128)."""
    Hd: torch.Tensor
    Hu: torch.Tensor
    Sd: torch.Tensor
    Su: torch.Tensor
    left: LeadTensors
    right: LeadTensors

    @property
    def N(self) -> int:
        return self.Hd.shape[0]

    @property
    def M(self) -> int:
        return self.Hd.shape[-1]

    def cstruct(self) -> rgf_device:
        N, M = self.N, self.M
        for name, n in (("Hd", N), ("Sd", N), ("Hu", N - 1), ("Su", N - 1)):
            t = getattr(self, name)
            if tuple(t.shape) != (n, M, M) and not (n == 0 and t.numel() == 0):
                raise ValueError(f"{name} must be [{n}, {M}, {M}], got {tuple(t.shape)}")
        hu = _ptr(self.Hu, _C128, "Hu") if self.Hu.numel() else None
        su = _ptr(self.Su, _C128, "Su") if self.Su.numel() else None
        return rgf_device(N, M, _ptr(self.Hd, _C128, "Hd"), hu, _ptr(self.Sd, _C128, "Sd"), su,
                          self.left.cstruct(), self.right.cstruct())


def transmission(dev: DeviceTensors, E: torch.Tensor, eta: float, precision="fp64", stream=None,
                 out: Optional[torch.Tensor] = None, info: Optional[torch.Tensor] = None
                 ) -> Tuple[torch.Tensor, torch.Tensor]:
    """T(E) for every energy in E (float64 device tensor); returns (T, info) device tensors.

    Stream-ordered like the C call: synchronise the stream before reading T.
    """
    lib = load()
    E = _energies(E)
    nE = E.numel()
    if out is None:
        out = torch.empty(nE, dtype=torch.float64, device=E.device)
    if info is None:
        info = torch.empty(nE, dtype=torch.int32, device=E.device)
    if out.numel() < nE or info.numel() < nE:
        raise ValueError("out and info need one element per energy")
    d = dev.cstruct()
    _check(lib.rgf_transmission(C.byref(d), _ptr(E, _F64, "E"), nE, float(eta), PRECISION[precision],
                                _ptr(out, _F64, "out"), _ptr(info, _I32, "info"), _stream(stream)))
    return out, info


#: bytes of the device scratch array behind transmission_noalloc (RGF_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 128 << 20


def transmission_noalloc(dev: DeviceTensors, E: torch.Tensor, eta: float, out: torch.Tensor,
                         info: torch.Tensor, precision="fp64", stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """T(E) into the caller's out (float64) and info (int32) through rgf_transmission_noalloc: the
    library's workspace is its static device scratch array, so the call allocates nothing."""
    lib = load()
    E = _energies(E)
    nE = E.numel()
    if out.numel() < nE or info.numel() < nE:
        raise ValueError("out and info need one element per energy")
    d = dev.cstruct()
    _check(lib.rgf_transmission_noalloc(C.byref(d), _ptr(E, _F64, "E"), nE, float(eta), PRECISION[precision],
                                        _ptr(out, _F64, "out"), _ptr(info, _I32, "info"), _stream(stream)))
    return out, info


def set_sr_maxit(maxit: int):
    """Cap the decimation at `maxit` steps (1..100) for later calls; 0 restores the default 100."""
    _check(load().rgf_set_sr_maxit(int(maxit)))


def get_sr_maxit() -> int:
    return int(load().rgf_get_sr_maxit())


def transmission_bias(dev: DeviceTensors, E: torch.Tensor, eta: float, u_left: float, u_right: float,
                      precision="fp64", stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """T(E, V_b) with the zero-bias device and electrodes rigidly shifted by u_left / u_right (eV)."""
    lib = load()
    E = _energies(E)
    nE = E.numel()
    out = torch.empty(nE, dtype=torch.float64, device=E.device)
    info = torch.empty(nE, dtype=torch.int32, device=E.device)
    d = dev.cstruct()
    _check(lib.rgf_transmission_bias(C.byref(d), _ptr(E), nE, float(eta), float(u_left), float(u_right),
                                     PRECISION[precision], _ptr(out), _ptr(info), _stream(stream)))
    return out, info


def ldos(dev: DeviceTensors, E: torch.Tensor, eta: float, parts=("dos", "left", "right"), stream=None):
    """Orbital-resolved LDOS: (dos, ados_left, ados_right, info), each [nE, N, M] (None when not in parts)."""
    lib = load()
    E = _energies(E)
    nE = E.numel()
    N, M = dev.N, dev.M
    unknown = set(parts) - {"dos", "left", "right"}
    if unknown or not parts:
        raise ValueError(f"parts must be a non-empty subset of dos/left/right, got {parts}")
    mk = lambda name: torch.empty((nE, N, M), dtype=torch.float64, device=E.device) if name in parts else None
    dos, adl, adr = mk("dos"), mk("left"), mk("right")
    info = torch.empty(nE, dtype=torch.int32, device=E.device)
    d = dev.cstruct()
    _check(lib.rgf_ldos(C.byref(d), _ptr(E), nE, float(eta), _ptr(dos), _ptr(adl), _ptr(adr), _ptr(info),
                        _stream(stream)))
    return dos, adl, adr, info


def kpm_moments(dev: DeviceTensors, e_min: float, e_max: float, n_mom: int, vectors: torch.Tensor,
                stream=None) -> torch.Tensor:
    """Chebyshev moments [n_mom] of S^-1 (H - b S) / a of the device blocks; vectors: [N*M, R] complex128."""
    lib = load()
    vectors = vectors.contiguous()
    if vectors.dtype != torch.complex128 or vectors.dim() != 2 or vectors.shape[0] != dev.N * dev.M:
        raise ValueError("vectors must be complex128 of shape [N*M, R]")
    mu = torch.empty(int(n_mom), dtype=torch.float64, device=vectors.device)
    d = dev.cstruct()
    _check(lib.rgf_kpm_moments(C.byref(d), float(e_min), float(e_max), int(n_mom), _ptr(vectors),
                               int(vectors.shape[1]), _ptr(mu), _stream(stream)))
    return mu


def kpm_fermi(mu: torch.Tensor, e_min: float, e_max: float, n_states: float, stream=None) -> torch.Tensor:
    """The Fermi level (a one-element device tensor) at which the Jackson-smoothed state count is n_states."""
    lib = load()
    mu = mu.contiguous()
    _ptr(mu, _F64, "mu")
    ef = torch.empty(1, dtype=torch.float64, device=mu.device)
    _check(lib.rgf_kpm_fermi(_ptr(mu), mu.numel(), float(e_min), float(e_max), float(n_states), _ptr(ef),
                             _stream(stream)))
    return ef


def kpm_dos(mu: torch.Tensor, e_min: float, e_max: float, E: torch.Tensor, stream=None) -> torch.Tensor:
    """Jackson-smoothed density of states per unit energy at the energies E."""
    lib = load()
    mu, E = mu.contiguous(), _energies(E)
    _ptr(mu, _F64, "mu")
    out = torch.empty(E.numel(), dtype=torch.float64, device=E.device)
    _check(lib.rgf_kpm_dos(_ptr(mu), mu.numel(), float(e_min), float(e_max), _ptr(E), E.numel(), _ptr(out),
                           _stream(stream)))
    return out


def landauer_current(E: torch.Tensor, T: torch.Tensor, mu_left: float, mu_right: float, kT: float,
                     stream=None) -> torch.Tensor:
    """I (amperes, a one-element device tensor) = G0 * trapezoid of (f_L - f_R) T over the ascending E."""
    lib = load()
    E = _energies(E)
    T = T.contiguous()
    _ptr(T, _F64, "T")
    if E.numel() != T.numel():
        raise ValueError("E and T differ in length")
    I = torch.empty(1, dtype=torch.float64, device=E.device)
    _check(lib.rgf_landauer_current(_ptr(E), _ptr(T), E.numel(), float(mu_left), float(mu_right), float(kT),
                                    _ptr(I), _stream(stream)))
    return I


def current(dev: DeviceTensors, E: torch.Tensor, eta: float, e_fermi: float, v_bias: float, kT: float,
            precision="fp64", stream=None):
    """Symmetric bias: (T(E, V_b), info, I) with mu_L,R = E_F +- V_b/2 and electrodes shifted by +-V_b/2."""
    T, info = transmission_bias(dev, E, eta, v_bias / 2.0, -v_bias / 2.0, precision, stream)
    I = landauer_current(E, T, e_fermi + v_bias / 2.0, e_fermi - v_bias / 2.0, kT, stream)
    return T, info, I


def transmission_kmesh(images, R, kpts, weights, E: torch.Tensor, eta: float, precision="fp64", stream=None):
    """k-averaged T(E) over a transverse mesh from real-space images.

    images: list of DeviceTensors (one per lattice image R[r]); R: [nR, 2] ints;
    kpts: [nk, 2] fractional; weights: [nk].  Returns (T [nE], Tk [nk, nE], info [nk, nE]).
    """
    import numpy as np
    lib = load()
    R = np.ascontiguousarray(R, dtype=np.int32).reshape(-1, 2)
    kpts = np.ascontiguousarray(kpts, dtype=np.float64).reshape(-1, 2)
    weights = np.ascontiguousarray(weights, dtype=np.float64)
    nR, nk = len(R), len(kpts)
    if len(images) != nR or len(weights) != nk:
        raise ValueError("one image per lattice vector and one weight per k-point")
    E = _energies(E)
    nE = E.numel()
    T = torch.empty(nE, dtype=torch.float64, device=E.device)
    Tk = torch.empty((nk, nE), dtype=torch.float64, device=E.device)
    info = torch.empty((nk, nE), dtype=torch.int32, device=E.device)
    cimg = (rgf_device * nR)(*[im.cstruct() for im in images])
    _check(lib.rgf_transmission_kmesh(cimg, nR, R.ctypes.data_as(C.POINTER(C.c_int32)),
                                      kpts.ctypes.data_as(C.POINTER(C.c_double)),
                                      weights.ctypes.data_as(C.POINTER(C.c_double)), nk, _ptr(E), nE, float(eta),
                                      PRECISION[precision], _ptr(T), _ptr(Tk), _ptr(info), _stream(stream)))
    return T, Tk, info


def transmission_batch(devs, Es, eta: float, precision="fp64", stream=None):
    """T(E) of several devices of uneven (N, M) and energy counts in one call.

    devs: list of DeviceTensors; Es: list of float64 device tensors.  Returns a list
    of (T, info) device tensors.  Stream-ordered like the C call.
    """
    lib = load()
    n = len(devs)
    if len(Es) != n:
        raise ValueError("one energy tensor per device")
    Es = [_energies(E) for E in Es]
    outs = [torch.empty(E.numel(), dtype=torch.float64, device=E.device) for E in Es]
    infos = [torch.empty(E.numel(), dtype=torch.int32, device=E.device) for E in Es]
    cdevs = (rgf_device * max(n, 1))(*[d.cstruct() for d in devs])
    P = C.c_void_p * max(n, 1)
    e_ptrs = P(*[_ptr(E) for E in Es])
    t_ptrs = P(*[_ptr(t) for t in outs])
    i_ptrs = P(*[_ptr(i) for i in infos])
    counts = (C.c_int64 * max(n, 1))(*[E.numel() for E in Es])
    _check(lib.rgf_transmission_batch(cdevs, n, e_ptrs, counts, float(eta), PRECISION[precision], t_ptrs,
                                      i_ptrs, _stream(stream)))
    return list(zip(outs, infos))


def lead_self_energy(lead: LeadTensors, side: int, E: torch.Tensor, eta: float, precision="fp64",
                     stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Sigma[nE, M, M] of one lead (side RGF_LEFT: L g_L U, RGF_RIGHT: U g_R L) and info."""
    lib = load()
    E = _energies(E)
    nE = E.numel()
    sigma = torch.empty((nE, lead.M, lead.M), dtype=torch.complex128, device=E.device)
    info = torch.empty(nE, dtype=torch.int32, device=E.device)
    ls = lead.cstruct()
    _check(lib.lead_self_energy(C.byref(ls), int(side), _ptr(E), nE, float(eta), PRECISION[precision],
                                _ptr(sigma), _ptr(info), _stream(stream)))
    return sigma, info


def release_workspaces():
    _check(load().rgf_release_workspaces())


def check_device(dev: DeviceTensors, tol: float = 1e-10, stream=None) -> float:
    """Hermiticity and overlap-diagonal check of the device and electrode blocks (raises RgfError
    naming the first failing block); returns the largest relative deviation."""
    w = C.c_double()
    d = dev.cstruct()
    _check(load().rgf_check_device(C.byref(d), float(tol), C.byref(w), _stream(stream)))
    return w.value


def set_checks(enable: bool):
    """Run check_device at the start of every transmission, LDOS and KPM call (synchronizes)."""
    _check(load().rgf_set_checks(1 if enable else 0))


def get_checks() -> bool:
    return bool(load().rgf_get_checks())


def profile(enable: bool, every: int = 1):
    """Record HIP events around every `every`-th launch of the dominant block product."""
    _check(load().rgf_profile(int(every) if enable else 0))


def profile_read() -> Tuple[int, float, float]:
    """(launches, total kernel ms, total algorithmic flops) of the sweep's main block products."""
    n = C.c_int64()
    ms = C.c_double()
    fl = C.c_double()
    _check(load().rgf_profile_read(C.byref(n), C.byref(ms), C.byref(fl)))
    return n.value, ms.value, fl.value


#: kernel classes of rgf_profile_classes (include/rgf.h, RGF_PROF_*)
PROFILE_CLASSES = ("sweep", "lu_update", "solve", "row64", "panel", "lead", "other", "fused")


def profile_classes(enable: bool, every: int = 1, classes=PROFILE_CLASSES):
    """Time every `every`-th launch of each named kernel class; count the flops of all launches."""
    mask = 0
    for c in classes:
        mask |= 1 << PROFILE_CLASSES.index(c)
    _check(load().rgf_profile_classes(int(every) if enable else 0, mask if enable else 0))


def profile_read_classes() -> dict:
    """{class: {timed launches, ms, timed flops, launches, flops}} for every class; resets them."""
    out = {}
    for i, name in enumerate(PROFILE_CLASSES):
        n, ms, fl, na, fa = C.c_int64(), C.c_double(), C.c_double(), C.c_int64(), C.c_double()
        _check(load().rgf_profile_read_class(i, C.byref(n), C.byref(ms), C.byref(fl), C.byref(na), C.byref(fa)))
        out[name] = {"timed_launches": n.value, "ms": ms.value, "timed_flops": fl.value,
                     "launches": na.value, "flops": fa.value}
    return out


def get_tile(precision="fp64") -> int:
    t = C.c_int32()
    _check(load().rgf_get_tile(PRECISION[precision], C.byref(t)))
    return t.value


def set_tile(precision, tile: int):
    _check(load().rgf_set_tile(PRECISION[precision], int(tile)))


def set_graphs(enable: bool):
    """Capture each chunk's sweep into a HIP graph on first use and replay it on later calls."""
    _check(load().rgf_set_graphs(1 if enable else 0))


def get_graphs() -> bool:
    return bool(load().rgf_get_graphs())


def get_tuning(M: int, precision="fp64") -> Tuple[int, int]:
    """(tile, lanes) in effect for block size M (defaults resolved)."""
    t, n = C.c_int32(), C.c_int32()
    _check(load().rgf_get_tuning(int(M), PRECISION[precision], C.byref(t), C.byref(n)))
    return t.value, n.value


def set_tuning(M: int, precision, tile: int = 0, lanes: int = 0):
    """Tile (0/64/128) and lanes (0..4) for block size M's class; 0 restores the default."""
    _check(load().rgf_set_tuning(int(M), PRECISION[precision], int(tile), int(lanes)))


def autotune(M: int, precision="fp64", batch: int = 64) -> dict:
    """Time the (tile, lanes) choices for block size M on the GPU, keep the fastest.

    Returns {"M", "precision", "tile", "lanes", "ms": {(tile, lanes): ms}}.
    """
    t, n = C.c_int32(), C.c_int32()
    ms = (C.c_double * 4)()
    _check(load().rgf_autotune(int(M), PRECISION[precision], int(batch), C.byref(t), C.byref(n), ms))
    keys = [(64, 1), (64, 2), (128, 1), (128, 2)]
    return {"M": int(M), "precision": precision, "tile": t.value, "lanes": n.value,
            "ms": {k: ms[i] for i, k in enumerate(keys) if ms[i] >= 0}}


def save_tuning(path: str, sizes, precisions=("fp64", "mixed")):
    """Write the table entries in effect for the given block sizes to a JSON file."""
    import json
    rows = []
    for M in sizes:
        for p in precisions:
            tile, lanes = get_tuning(M, p)
            rows.append({"M": int(M), "precision": p, "tile": tile, "lanes": lanes})
    with open(path, "w") as f:
        json.dump({"librgf": version(), "entries": rows}, f, indent=1)


def load_tuning(path: str) -> int:
    """Apply the entries of a file written by save_tuning; returns how many were applied."""
    import json
    with open(path) as f:
        data = json.load(f)
    for r in data["entries"]:
        set_tuning(r["M"], r["precision"], r["tile"], r["lanes"])
    return len(data["entries"])


MIXED_SWEEP, MIXED_LU, MIXED_SOLVE, MIXED_ALL = 1, 2, 4, 7


def set_mixed_parts(parts: int):
    """Which block products run in FP32 on the matrix cores for precision="mixed" (bit mask)."""
    _check(load().rgf_set_mixed_parts(int(parts)))


def get_mixed_parts() -> int:
    return int(load().rgf_get_mixed_parts())


def version() -> str:
    return load().rgf_version().decode()


class Server:
    """Continuous-batching transmission server (transport_open/submit/poll/close).

    submit() takes HOST numpy arrays (complex128 blocks, float64 energies); they
    are copied before it returns.  poll() returns None while the request runs,
    else (T, info, latency_s) as numpy arrays / float.
    """

    def __init__(self, hbm_budget_bytes: int = 0, lead_cache_bytes: int = 0, max_slots: int = 0):
        lib = load()
        self._lib = lib
        opts = rgf_server_opts(int(hbm_budget_bytes), int(lead_cache_bytes), int(max_slots))
        h = C.c_void_p()
        _check(lib.transport_open(C.byref(opts), C.byref(h)))
        self._h = h
        self._n = {}

    def submit(self, hd, hu, sd, su, left, right, E, eta: float, precision="fp64",
               lead_key_L: int = 0, lead_key_R: int = 0) -> int:
        """Blocks as numpy complex128 arrays (hd, sd: [N, M, M]; hu, su: [N-1, M, M]; left/right:
        (H00, H01, S00, S01)); E float64 [nE].  Equal lead keys must mean identical lead blocks."""
        import numpy as np
        arrs = [np.ascontiguousarray(x, dtype=np.complex128) for x in (hd, hu, sd, su)]
        la = [np.ascontiguousarray(x, dtype=np.complex128) for x in left]
        ra = [np.ascontiguousarray(x, dtype=np.complex128) for x in right]
        E = np.ascontiguousarray(E, dtype=np.float64)
        N, M = arrs[0].shape[0], arrs[0].shape[-1]
        p = lambda a: a.ctypes.data if a.size else None
        d = rgf_device(N, M, p(arrs[0]), p(arrs[1]), p(arrs[2]), p(arrs[3]),
                       rgf_lead(M, *[p(a) for a in la]), rgf_lead(M, *[p(a) for a in ra]))
        t = C.c_uint64()
        _check(self._lib.transport_submit(self._h, C.byref(d), int(lead_key_L), int(lead_key_R), E.ctypes.data,
                                          len(E), float(eta), PRECISION[precision], C.byref(t)))
        self._n[t.value] = len(E)
        return t.value

    def poll(self, ticket: int):
        import numpy as np
        n = self._n[ticket]
        T = np.empty(n, np.float64)
        info = np.empty(n, np.int32)
        lat = C.c_double()
        rc = self._lib.transport_poll(self._h, C.c_uint64(ticket), T.ctypes.data, info.ctypes.data, C.byref(lat))
        if rc == RGF_EAGAIN:
            return None
        self._n.pop(ticket, None)
        _check(rc)
        return T, info, lat.value

    def wait(self, ticket: int, poll_s: float = 0.002):
        import time
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            time.sleep(poll_s)

    def stats(self) -> dict:
        s = rgf_server_stats()
        _check(self._lib.transport_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in rgf_server_stats._fields_}

    def close(self):
        if self._h:
            _check(self._lib.transport_close(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
