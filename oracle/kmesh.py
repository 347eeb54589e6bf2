"""FP64 reference for transverse k-point sampling of the transmission.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed
----------------
The paper's devices are periodic across the transport direction and their
transmissions are sampled on transverse k-point meshes (Method: 7x7x1,
9x9x1 and 11x11x1 meshes for the three device classes; the per-stage cost
is O(N_z M_b^3) per energy and per transverse k-point, Results).  The
textbook construction, used here: every block (device on-site and coupling
blocks, electrode blocks, H and S alike) is given in real space for a set of
transverse lattice images R = (R_1, R_2), and at the fractional transverse
wavevector k = (k_1, k_2)

    X(k) = sum_R X(R) exp(2 pi i (k_1 R_1 + k_2 R_2)),

the k-resolved transmission T_k(E) is the Caroli transmission of the
device built from the X(k), and T(E) = sum_k w_k T_k(E) with the mesh
weights w_k (summing to one).
"""
from __future__ import annotations

import numpy as np

from .rgf_oracle import transmission


def bloch_sum(blocks, R, k):
    """sum_r blocks[r] exp(2 pi i k . R_r) for blocks [nR, ...] and R [nR, 2]."""
    ph = np.exp(2j * np.pi * (np.asarray(R, float) @ np.asarray(k, float)))
    return np.tensordot(ph, np.asarray(blocks), axes=(0, 0))


def device_at_k(images, R, k):
    """The device of transverse wavevector k from its real-space images (synth.Device each)."""
    import synth
    N = images[0].N
    hd = bloch_sum(np.array([[im.Hd(i) for i in range(N)] for im in images]), R, k)
    sd = bloch_sum(np.array([[im.Sd(i) for i in range(N)] for im in images]), R, k)
    hu = bloch_sum(np.array([[im.Hu(i) for i in range(N - 1)] for im in images]), R, k) if N > 1 else []
    su = bloch_sum(np.array([[im.Su(i) for i in range(N - 1)] for im in images]), R, k) if N > 1 else []
    lead = lambda side: synth.Lead(*(bloch_sum(np.array([getattr(getattr(im, side), name) for im in images]), R, k)
                                     for name in ("H00", "H01", "S00", "S01")))
    return synth.device_from_blocks(list(hd), list(hu), list(sd), list(su), lead("left"), lead("right"))


def transmission_kmesh(images, R, kpts, weights, energies, eta: float, method: str = "auto"):
    """(T(E) = sum_k w_k T_k(E), T_k [nk, nE]) over the transverse mesh."""
    kpts = np.asarray(kpts, float).reshape(-1, 2)
    weights = np.asarray(weights, float)
    Tk = np.array([transmission(device_at_k(images, R, k), energies, eta, method=method) for k in kpts])
    return weights @ Tk, Tk


def monkhorst_pack(n1: int, n2: int):
    """Uniform n1 x n2 mesh of fractional k = ((i + 1/2)/n1 - 1/2, (j + 1/2)/n2 - 1/2), equal weights."""
    k1 = (np.arange(n1) + 0.5) / n1 - 0.5
    k2 = (np.arange(n2) + 0.5) / n2 - 0.5
    kk = np.array([(a, b) for a in k1 for b in k2])
    return kk, np.full(len(kk), 1.0 / len(kk))
