"""Seeded synthetic inputs for the RGF transmission path.

This module only *builds inputs*: block-tridiagonal nonorthogonal devices
(H, S), lead principal layers and energy grids.  It holds none of the
transport arithmetic (no Green's functions, no self-energies, no
transmission), so both the CPU oracle and the GPU harness can draw their
inputs from it without sharing any of the method.

Conventions (stated once, used everywhere):

* A block is an M x M complex128 array, row-major.
* ``Hu[i]`` couples layer i to layer i+1 (rows in layer i, columns in
  layer i+1), so H_{i+1,i} = Hu[i]^dagger; the same holds for S.
* A lead is one principal layer (H00, H01, S00, S01) repeated; H01/S01
  couple lead layer n to n+1 in the +z direction for *both* leads.  The
  left lead's surface layer couples to device layer 0 through its own
  (H01, S01); device layer N-1 couples to the right lead's surface layer
  through the right lead's (H01, S01).

The paper (Methods; Results on Pt-Si-Pt and Pt-Si:P-Pt devices) works
with DFT Hamiltonians that are not available here; these seeded random
blocks stand in for them with the shapes of the benchmark workloads.
Random numbers come from ``numpy.random.default_rng(SeedSequence([seed,
layer, kind]))`` with kind 0: H_ii, 1: H_i,i+1, 2: S_ii, 3: S_i,i+1,
4: dopants, so any layer can be rebuilt on its own.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

KIND_HD, KIND_HU, KIND_SD, KIND_SU, KIND_DOPE = 0, 1, 2, 3, 4
DECAY_LENGTH = 32.0


def _rng(seed: int, layer: int, kind: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(layer), int(kind)]))


def complex_normal(rng: np.random.Generator, shape) -> np.ndarray:
    """(a + i b)/sqrt(2), a, b ~ N(0,1): unit complex variance."""
    a = rng.standard_normal(shape)
    b = rng.standard_normal(shape)
    return (a + 1j * b) / np.sqrt(2.0)


def gue(rng: np.random.Generator, m: int) -> np.ndarray:
    """Hermitian matrix with N(0,1) diagonal and unit-variance complex off-diagonals."""
    x = complex_normal(rng, (m, m))
    return (x + x.conj().T) / np.sqrt(2.0)


def goe(rng: np.random.Generator, m: int) -> np.ndarray:
    z = rng.standard_normal((m, m))
    return (z + z.T) / np.sqrt(2.0)


def spd_perturbation(rng: np.random.Generator, m: int) -> np.ndarray:
    b = rng.standard_normal((m, m))
    return (b @ b.T) / m


def decay_weights(m: int, length: float = DECAY_LENGTH) -> np.ndarray:
    j = np.arange(m)
    return np.exp(-np.abs(j[:, None] - j[None, :]) / length)


@dataclass
class Lead:
    """One principal layer of a semi-infinite electrode."""
    H00: np.ndarray
    H01: np.ndarray
    S00: np.ndarray
    S01: np.ndarray

    @property
    def M(self) -> int:
        return self.H00.shape[0]

    def mirrored(self) -> "Lead":
        """The same electrode seen with the transport direction reversed."""
        return Lead(self.H00, self.H01.conj().T.copy(), self.S00, self.S01.conj().T.copy())


@dataclass
class Device:
    """Block-tridiagonal device; blocks are either stored or rebuilt per layer.

    ``Hd(i)``, ``Sd(i)`` for i in [0, N) and ``Hu(i)``, ``Su(i)`` for i in
    [0, N-1) return M x M complex128 blocks.  A device built from one
    repeated principal layer keeps only that layer (``base``) plus the
    per-layer on-site shifts (``shifts``), so a 400-layer, M = 1024 device
    costs four blocks of host memory.
    """
    N: int
    M: int
    left: Lead
    right: Lead
    _hd: Optional[List[np.ndarray]] = None
    _hu: Optional[List[np.ndarray]] = None
    _sd: Optional[List[np.ndarray]] = None
    _su: Optional[List[np.ndarray]] = None
    base: Optional[Lead] = None
    shifts: Dict[int, float] = field(default_factory=dict)
    name: str = ""

    def Hd(self, i: int) -> np.ndarray:
        if self._hd is not None:
            return self._hd[i]
        h = self.base.H00
        if i in self.shifts:
            h = h + self.shifts[i] * np.eye(self.M)
        return h

    def Sd(self, i: int) -> np.ndarray:
        return self._sd[i] if self._sd is not None else self.base.S00

    def Hu(self, i: int) -> np.ndarray:
        return self._hu[i] if self._hu is not None else self.base.H01

    def Su(self, i: int) -> np.ndarray:
        return self._su[i] if self._su is not None else self.base.S01

    def stacked(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
        """(Hd[N], Hu[N-1], Sd[N], Su[N-1]) as contiguous complex128 arrays."""
        N, M = self.N, self.M
        hd = np.empty((N, M, M), np.complex128)
        sd = np.empty((N, M, M), np.complex128)
        hu = np.empty((max(N - 1, 0), M, M), np.complex128)
        su = np.empty((max(N - 1, 0), M, M), np.complex128)
        for i in range(N):
            hd[i] = self.Hd(i)
            sd[i] = self.Sd(i)
        for i in range(N - 1):
            hu[i] = self.Hu(i)
            su[i] = self.Su(i)
        return hd, hu, sd, su

    def mirrored(self) -> "Device":
        """Layers reversed and the leads swapped: transport from right to left.

        Hu'[j] = Hu[N-2-j]^dagger; the new left lead is the old right lead
        seen backwards (H01 -> H01^dagger) and vice versa.
        """
        N = self.N
        hd = [self.Hd(N - 1 - j) for j in range(N)]
        sd = [self.Sd(N - 1 - j) for j in range(N)]
        hu = [self.Hu(N - 2 - j).conj().T.copy() for j in range(N - 1)]
        su = [self.Su(N - 2 - j).conj().T.copy() for j in range(N - 1)]
        return Device(N, self.M, self.right.mirrored(), self.left.mirrored(),
                      hd, hu, sd, su, name=self.name + "-mirrored")

    def with_basis_change(self, V: np.ndarray) -> "Device":
        """Every block X -> V^dagger X V, leads included (a congruence)."""
        f = lambda X: V.conj().T @ X @ V
        N = self.N
        lead = lambda L: Lead(f(L.H00), f(L.H01), f(L.S00), f(L.S01))
        return Device(N, self.M, lead(self.left), lead(self.right),
                      [f(self.Hd(i)) for i in range(N)], [f(self.Hu(i)) for i in range(N - 1)],
                      [f(self.Sd(i)) for i in range(N)], [f(self.Su(i)) for i in range(N - 1)],
                      name=self.name + "-basis")


def device_from_blocks(hd, hu, sd, su, left: Lead, right: Lead, name: str = "") -> Device:
    hd = [np.asarray(x, np.complex128) for x in hd]
    sd = [np.asarray(x, np.complex128) for x in sd]
    hu = [np.asarray(x, np.complex128) for x in hu]
    su = [np.asarray(x, np.complex128) for x in su]
    return Device(len(hd), hd[0].shape[0], left, right, hd, hu, sd, su, name=name)


def repeated_device(layer: Lead, N: int, shifts: Optional[Dict[int, float]] = None,
                    name: str = "") -> Device:
    """A device made of one principal layer repeated N times; the same layer is both leads."""
    return Device(N, layer.M, layer, layer, base=layer, shifts=dict(shifts or {}), name=name)


# ----------------------------------------------------------------------------
# Principal-layer recipes
# ----------------------------------------------------------------------------

def layer_c1(seed: int = 1, m: int = 4) -> Lead:
    """C1 recipe: H00 GUE, H01 0.5 complex N(0,1), S00 = I + 0.05 GOE, S01 = 0.02 N(0,1)."""
    H00 = gue(_rng(seed, 0, KIND_HD), m)
    H01 = 0.5 * complex_normal(_rng(seed, 0, KIND_HU), (m, m))
    S00 = np.eye(m) + 0.05 * goe(_rng(seed, 0, KIND_SD), m)
    S01 = 0.02 * _rng(seed, 0, KIND_SU).standard_normal((m, m))
    return Lead(H00, H01, S00.astype(np.complex128), S01.astype(np.complex128))


def decay_layer(seed: int, layer: int, m: int) -> Lead:
    """C2-C5 recipe for one principal layer (decay-weighted random blocks).

    H_ii = GUE * W, H_i,i+1 = 0.5 complex N(0,1) * W, S_ii = I + 0.1 P (P SPD),
    S_i,i+1 = 0.02 N(0,1) * W with W_jk = exp(-|j-k|/32).
    """
    W = decay_weights(m)
    H00 = gue(_rng(seed, layer, KIND_HD), m) * W
    H01 = 0.5 * complex_normal(_rng(seed, layer, KIND_HU), (m, m)) * W
    S00 = np.eye(m) + 0.1 * spd_perturbation(_rng(seed, layer, KIND_SD), m)
    S01 = 0.02 * _rng(seed, layer, KIND_SU).standard_normal((m, m)) * W
    return Lead(H00, H01, S00.astype(np.complex128), S01.astype(np.complex128))


def dopant_shifts(dope_seed: int, N: int, fraction: float = 0.05, sigma: float = 0.3) -> Dict[int, float]:
    """A seeded 5% of the interior layers (0-based 1..N-2) get an on-site shift delta ~ N(0, sigma^2)."""
    rng = _rng(dope_seed, 0, KIND_DOPE)
    n = int(round(fraction * N))
    layers = np.sort(rng.choice(np.arange(1, N - 1), size=n, replace=False))
    deltas = rng.normal(0.0, sigma, size=n)
    return {int(l): float(d) for l, d in zip(layers, deltas)}


# ----------------------------------------------------------------------------
# The benchmark configurations
# ----------------------------------------------------------------------------

@dataclass
class Config:
    name: str
    device: Device
    energies: np.ndarray
    eta: float


def config_c1() -> Config:
    """Tiny pristine case: 20 layers, M = 4, 200 energies on [-4, 4], eta = 1e-6."""
    layer = layer_c1(seed=1, m=4)
    return Config("c1", repeated_device(layer, 20, name="c1"), np.linspace(-4.0, 4.0, 200), 1e-6)


def config_c2(n_layers: int = 60, m: int = 256, n_e: int = 1000) -> Config:
    """Junction-like case: 60 random decay-weighted layers, M = 256, a separate seeded lead."""
    lead = decay_layer(102, 0, m)
    layers = [decay_layer(2, i, m) for i in range(n_layers)]
    dev = device_from_blocks([l.H00 for l in layers], [l.H01 for l in layers[:-1]],
                             [l.S00 for l in layers], [l.S01 for l in layers[:-1]],
                             lead, lead, name="c2")
    return Config("c2", dev, np.linspace(-2.0, 2.0, n_e), 1e-6)


def config_doped(seed: int, dope_seed: int, n_layers: int, m: int, n_e: int, name: str,
                 doped: bool = True) -> Config:
    layer = decay_layer(seed, 0, m)
    shifts = dopant_shifts(dope_seed, n_layers) if doped else {}
    dev = repeated_device(layer, n_layers, shifts, name=name)
    return Config(name, dev, np.linspace(-2.0, 2.0, n_e), 1e-6)


def config_c3(doped: bool = True) -> Config:
    """Doped channel: 200 layers, M = 512, 5% doped layers, 2000 energies."""
    return config_doped(3, 303, 200, 512, 2000, "c3", doped)


def config_c4(doped: bool = True, n_e: int = 512) -> Config:
    """Beyond 10,000 atoms: 400 layers, M = 1024, 5% doped layers, 512 energies."""
    return config_doped(4, 404, 400, 1024, n_e, "c4", doped)


C5_BLOCK_SIZES = (128, 256, 512, 1024)
C5_GRID = np.linspace(-2.0, 2.0, 1024)


@dataclass
class Request:
    index: int
    arrival_s: float
    device: Device
    energies: np.ndarray
    lead_key: int


def phase_vectors(n: int, R: int, seed: int) -> np.ndarray:
    """R random-phase vectors of length n (columns; E[r r^dagger] = I), the KPM trace estimator's
    inputs: entries exp(2 pi i u), u uniform on [0, 1) from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return np.exp(2j * np.pi * rng.random((n, R)))


def kpm_bounds(layer: Lead, shifts: Optional[Dict[int, float]] = None, margin: float = 1.01):
    """Spectral bounds +-e for a device repeating `layer` with on-site shifts: |e| <= ||H||_2 /
    lambda_min(S) with ||H||_2 <= ||H00|| + 2 ||H01|| + max |shift| and lambda_min(S) >=
    lambda_min(S00) - 2 ||S01|| (Weyl's inequality), times `margin`."""
    norm2 = lambda X: np.linalg.norm(X, 2)
    h = norm2(layer.H00) + 2 * norm2(layer.H01) + max([abs(v) for v in (shifts or {}).values()] + [0.0])
    s_min = np.linalg.eigvalsh(layer.S00)[0] - 2 * norm2(layer.S01)
    if s_min <= 0:
        raise ValueError("the overlap bound is not positive")
    e = margin * h / s_min
    return -e, e


def c5_lead(m: int) -> Lead:
    """The lead type of block size m (4 seeded lead types, one per block size)."""
    return decay_layer(500 + m, 0, m)


def c5_requests(n_req: int = 128, qps: float = 1.0, sizes=C5_BLOCK_SIZES, n_layers=(20, 400),
                n_e=(64, 1024), seed: int = 5, repeated: bool = False) -> List[Request]:
    """Serving mix: Poisson arrivals; M from ``sizes``, N ~ U[20, 400], nE ~ U[64, 1024].

    Request r draws its device from seed 5000 + r (decay-layer recipe per
    layer) and its energies as a sorted seeded subset of the common
    1024-point grid on [-2, 2]; lead type = block-size class.  With
    ``repeated`` the device is instead layer 0 of that recipe repeated N
    times with 5% seeded dopant shifts (the C3/C4 recipe): the same shapes
    and work, without drawing N random layers on the host.
    """
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0, 0]))
    gaps = rng.exponential(1.0 / qps, size=n_req)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for r in range(n_req):
        rr = np.random.default_rng(np.random.SeedSequence([5000 + r, 0, 0]))
        m = int(rr.choice(sizes))
        N = int(rr.integers(n_layers[0], n_layers[1] + 1))
        ne = int(rr.integers(n_e[0], min(n_e[1], len(C5_GRID)) + 1))
        idx = np.sort(rr.choice(len(C5_GRID), size=ne, replace=False))
        lead = c5_lead(m)
        if repeated:
            base = decay_layer(5000 + r, 0, m)
            shifts = dopant_shifts(5000 + r, N) if N > 2 else {}
            dev = Device(N, m, lead, lead, base=base, shifts=shifts, name=f"c5-r{r}")
        else:
            layers = [decay_layer(5000 + r, i, m) for i in range(N)]
            dev = device_from_blocks([l.H00 for l in layers], [l.H01 for l in layers[:-1]],
                                     [l.S00 for l in layers], [l.S01 for l in layers[:-1]],
                                     lead, lead, name=f"c5-r{r}")
        out.append(Request(r, float(arrivals[r]), dev, C5_GRID[idx].copy(), lead_key=m))
    return out


# ----------------------------------------------------------------------------
# Systems with closed-form answers (inputs only; the answers live in the tests)
# ----------------------------------------------------------------------------

def chain_lead(eps0: float, t: float, s: float = 0.0) -> Lead:
    """1D tight-binding chain, one orbital per layer: H00 = eps0, H01 = t, S00 = 1, S01 = s."""
    c = lambda x: np.array([[x]], np.complex128)
    return Lead(c(eps0), c(t), c(1.0), c(s))


def chain_device(N: int, eps0: float = 0.0, t: float = -1.0, s: float = 0.0,
                 impurity: Optional[Tuple[int, float]] = None) -> Device:
    """A pristine chain of N sites, optionally with one on-site impurity (site, U)."""
    lead = chain_lead(eps0, t, s)
    hd = [np.array([[eps0]], np.complex128) for _ in range(N)]
    if impurity is not None:
        site, U = impurity
        hd[site] = hd[site] + U
    return device_from_blocks(hd, [lead.H01] * (N - 1), [lead.S00] * N, [lead.S01] * (N - 1),
                              lead, lead, name="chain")


def decoupled_chains(eps: np.ndarray, t: np.ndarray, N: int) -> Device:
    """M independent orthogonal chains (eps_m, t_m), diagonal blocks."""
    H00 = np.diag(np.asarray(eps, float)).astype(np.complex128)
    H01 = np.diag(np.asarray(t, float)).astype(np.complex128)
    M = len(eps)
    lead = Lead(H00, H01, np.eye(M, dtype=np.complex128), np.zeros((M, M), np.complex128))
    return repeated_device(lead, N, name="chains")


def random_basis(M: int, seed: int, scale: float = 0.3) -> np.ndarray:
    """A well-conditioned random invertible complex matrix I + scale * complex N(0,1)/sqrt(M)."""
    rng = _rng(seed, 0, 0)
    return np.eye(M) + scale * complex_normal(rng, (M, M)) / np.sqrt(M)


def random_small_device(N: int, M: int, seed: int, real: bool = False,
                        coupling: float = 0.5, distinct_leads: bool = False) -> Device:
    """Independent random layers (GUE on-site, complex couplings) and a separate random lead."""
    def layer(sd, i):
        rng_h = _rng(sd, i, KIND_HD)
        rng_u = _rng(sd, i, KIND_HU)
        rng_s = _rng(sd, i, KIND_SD)
        rng_v = _rng(sd, i, KIND_SU)
        if real:
            H00 = goe(rng_h, M).astype(np.complex128)
            H01 = (coupling * rng_u.standard_normal((M, M))).astype(np.complex128)
        else:
            H00 = gue(rng_h, M)
            H01 = coupling * complex_normal(rng_u, (M, M))
        S00 = (np.eye(M) + 0.05 * goe(rng_s, M)).astype(np.complex128)
        S01 = (0.02 * rng_v.standard_normal((M, M))).astype(np.complex128)
        return Lead(H00, H01, S00, S01)
    lead = layer(seed + 1000, 0)
    lead_r = layer(seed + 2000, 0) if distinct_leads else lead
    layers = [layer(seed, i) for i in range(N)]
    return device_from_blocks([l.H00 for l in layers], [l.H01 for l in layers[:-1]],
                              [l.S00 for l in layers], [l.S01 for l in layers[:-1]],
                              lead, lead_r, name=f"rand{N}x{M}")


# ----------------------------------------------------------------------------
# Transverse lattice images (inputs of k-point sampling)
# ----------------------------------------------------------------------------

KIND_IMAGE = 5


def transverse_images(base: Device, seed: int, scale: float = 0.1, directions=((1, 0), (0, 1))):
    """Real-space images of a transversely periodic device: (images, R).

    images[0] is ``base`` at R = (0, 0).  For each direction d and the pair
    +-d, on-site blocks (H_ii, S_ii and the electrodes' H00, S00) get a
    seeded complex image X(+d) with X(-d) = X(+d)^dagger, so every X(k) is
    Hermitian; coupling blocks (H_i,i+1, S_i,i+1, H01, S01) get independent
    seeded images for +d and -d.  H images are ``scale`` x decay-weighted
    complex N(0,1), S images a tenth of that.  One electrode serves both sides.
    """
    N, M = base.N, base.M
    W = decay_weights(M)
    dag = lambda x: x.conj().T
    images, R = [base], [(0, 0)]
    for j, d in enumerate(directions):
        rng = lambda layer, kind, sign: _rng(seed, layer, 16 * (KIND_IMAGE + kind) + 4 * j + sign)
        cn = lambda r, s: s * complex_normal(r, (M, M)) * W
        hd_p = [cn(rng(i, 0, 0), scale) for i in range(N)]
        sd_p = [cn(rng(i, 1, 0), 0.1 * scale) for i in range(N)]
        hu = [[cn(rng(i, 2, sg), scale) for i in range(N - 1)] for sg in (0, 1)]
        su = [[cn(rng(i, 3, sg), 0.1 * scale) for i in range(N - 1)] for sg in (0, 1)]
        l00, ls00 = cn(rng(N, 4, 0), scale), cn(rng(N, 5, 0), 0.1 * scale)
        l01 = [cn(rng(N, 6, sg), scale) for sg in (0, 1)]
        ls01 = [cn(rng(N, 7, sg), 0.1 * scale) for sg in (0, 1)]
        plus_lead = Lead(l00, l01[0], ls00, ls01[0])
        minus_lead = Lead(dag(l00), l01[1], dag(ls00), ls01[1])
        images.append(device_from_blocks(hd_p, hu[0], sd_p, su[0], plus_lead, plus_lead))
        images.append(device_from_blocks([dag(x) for x in hd_p], hu[1], [dag(x) for x in sd_p], su[1],
                                         minus_lead, minus_lead))
        R += [tuple(d), (-d[0], -d[1])]
    return images, R
