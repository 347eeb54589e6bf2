"""FP64 reference for the orbital-resolved local density of states of the device.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed
----------------
The paper reports the spatially resolved local density of states (LDOS) of
its devices, at zero and at finite bias with the zero-bias Hamiltonian
(Discussion, the paragraph on finite-bias transport).  It prints no
formula, so the textbook NEGF definitions are used (Datta, *Electronic
Transport in Mesoscopic Systems*, ch. 8; the Mulliken projection for a
nonorthogonal basis):

* G = (z S - H - Sigma_L (+) 0 (+) Sigma_R)^-1 on the device, z = E + i eta;
* the spectral function A = i (G - G^dagger), and the electrode-injected
  spectral functions A_X = G Gamma_X G^dagger, Gamma_X = i (Sigma_X -
  Sigma_X^dagger) placed on the contact layer of electrode X;
* LDOS of orbital mu:          rho_mu   = (1 / 2 pi) Re [A S]_mu,mu
  electrode-injected LDOS:     rho^X_mu = (1 / 2 pi) Re [A_X S]_mu,mu
  with S the device overlap (the projection stays inside the device: the
  overlap between device and electrode orbitals is not part of it).

Identities that follow from the definition (used as pins):
  G^-1 - G^-dagger = 2 i eta S + i (Gamma_L + Gamma_R), hence
  A = A_L + A_R + 2 eta G S G^dagger, so rho = rho^L + rho^R + (eta/pi) Re diag(G S G^dagger S);
  sum_mu rho_mu = -(1/pi) Im Tr[G S]; for an isolated device with
  generalized eigenvalues e_n of (H, S) this is sum_n (eta/pi) / ((E - e_n)^2 + eta^2);
  for S = I, rho_mu = -(1/pi) Im G_mu,mu.

Two formulations: ``ldos_dense`` inverts the whole device matrix (small
devices); ``ldos_layers`` solves the block-tridiagonal system for the block
columns it needs (block Thomas: block LU from the first layer, then
back-substitution), for selected layers of large devices.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .rgf_oracle import broadening, self_energies


def device_matrix(dev, z: complex, sigma_l, sigma_r):
    """Dense (z S - H - Sigma_L (+) 0 (+) Sigma_R) and the dense device overlap S."""
    N, M = dev.N, dev.M
    A = np.zeros((N * M, N * M), np.complex128)
    S = np.zeros((N * M, N * M), np.complex128)
    for i in range(N):
        blk = slice(i * M, (i + 1) * M)
        A[blk, blk] = z * dev.Sd(i) - dev.Hd(i)
        S[blk, blk] = dev.Sd(i)
        if i + 1 < N:
            nxt = slice((i + 1) * M, (i + 2) * M)
            A[blk, nxt] = z * dev.Su(i) - dev.Hu(i)
            A[nxt, blk] = z * dev.Su(i).conj().T - dev.Hu(i).conj().T
            S[blk, nxt] = dev.Su(i)
            S[nxt, blk] = dev.Su(i).conj().T
    A[:M, :M] -= sigma_l
    A[(N - 1) * M:, (N - 1) * M:] -= sigma_r
    return A, S


def _mulliken(X, S) -> np.ndarray:
    """(1 / 2 pi) Re diag(X S)."""
    return np.real(np.einsum("ij,ji->i", X, S)) / (2.0 * np.pi)


def ldos_dense(dev, z: complex, sigma_l, sigma_r):
    """(rho, rho_L, rho_R), each [N, M], from the dense inverse of the device matrix."""
    N, M = dev.N, dev.M
    A, S = device_matrix(dev, z, sigma_l, sigma_r)
    G = np.linalg.inv(A)
    spec = 1j * (G - G.conj().T)
    gam_l = np.zeros_like(A)
    gam_r = np.zeros_like(A)
    gam_l[:M, :M] = broadening(sigma_l)
    gam_r[(N - 1) * M:, (N - 1) * M:] = broadening(sigma_r)
    a_l = G @ gam_l @ G.conj().T
    a_r = G @ gam_r @ G.conj().T
    shape = (N, M)
    return (_mulliken(spec, S).reshape(shape), _mulliken(a_l, S).reshape(shape),
            _mulliken(a_r, S).reshape(shape))


class _BlockThomas:
    """Block LU of the block-tridiagonal device matrix, kept for many right-hand sides."""

    def __init__(self, dev, z: complex, sigma_l, sigma_r):
        N = dev.N
        self.N, self.M = N, dev.M
        self.diag = [z * dev.Sd(i) - dev.Hd(i) for i in range(N)]
        self.diag[0] = self.diag[0] - sigma_l
        self.diag[N - 1] = self.diag[N - 1] - sigma_r
        self.up = [z * dev.Su(i) - dev.Hu(i) for i in range(N - 1)]
        self.lo = [z * dev.Su(i).conj().T - dev.Hu(i).conj().T for i in range(N - 1)]
        # D'_0 = A_00, D'_i = A_ii - L_i D'_{i-1}^-1 U_{i-1}
        self.lus = []
        for i in range(N):
            D = self.diag[i]
            if i > 0:
                D = D - self.lo[i - 1] @ sla.lu_solve(self.lus[i - 1], self.up[i - 1])
            self.lus.append(sla.lu_factor(D))

    def block_column(self, q: int):
        """The q-th block column of G: solve A X = e_q (x) I."""
        N, M = self.N, self.M
        y = [np.zeros((M, M), np.complex128) for _ in range(N)]
        y[q] = np.eye(M, dtype=np.complex128)
        for i in range(q + 1, N):  # forward elimination of the right-hand side (zero above row q)
            y[i] = y[i] - self.lo[i - 1] @ sla.lu_solve(self.lus[i - 1], y[i - 1])
        x = [None] * N
        x[N - 1] = sla.lu_solve(self.lus[N - 1], y[N - 1])
        for i in range(N - 2, -1, -1):
            x[i] = sla.lu_solve(self.lus[i], y[i] - self.up[i] @ x[i + 1])
        return x


def _s_block(dev, p: int, q: int):
    """Device overlap block S_pq (zero unless |p - q| <= 1)."""
    if p == q:
        return dev.Sd(p)
    if q == p + 1:
        return dev.Su(p)
    if q == p - 1:
        return dev.Su(q).conj().T
    return None


def ldos_layers(dev, z: complex, sigma_l, sigma_r, layers):
    """(rho, rho_L, rho_R) for the given layers only, each [len(layers), M], from block columns."""
    N = dev.N
    bt = _BlockThomas(dev, z, sigma_l, sigma_r)
    cols = {}

    def col(q):
        if q not in cols:
            cols[q] = bt.block_column(q)
        return cols[q]

    first, last = col(0), col(N - 1)
    gam_l, gam_r = broadening(sigma_l), broadening(sigma_r)
    rho, rho_l, rho_r = [], [], []
    for p in layers:
        near = [q for q in (p - 1, p, p + 1) if 0 <= q < N]
        # [A S]_pp = sum_q i (G_pq - (G_qp)^dagger) S_qp
        AS = sum(1j * (col(q)[p] - col(p)[q].conj().T) @ _s_block(dev, q, p) for q in near)
        # [A_X S]_pp = sum_q G_p,c Gamma_X (G_q,c)^dagger S_qp, c the contact layer of X
        ALS = sum(first[p] @ gam_l @ first[q].conj().T @ _s_block(dev, q, p) for q in near)
        ARS = sum(last[p] @ gam_r @ last[q].conj().T @ _s_block(dev, q, p) for q in near)
        for out, X in ((rho, AS), (rho_l, ALS), (rho_r, ARS)):
            out.append(np.real(np.diag(X)) / (2.0 * np.pi))
    return np.array(rho), np.array(rho_l), np.array(rho_r)


def local_dos(dev, energies, eta: float, method: str = "auto", layers=None):
    """(rho, rho_L, rho_R) as [nE, N or len(layers), M] over the energies."""
    energies = np.atleast_1d(np.asarray(energies, np.float64))
    if method == "auto":
        method = "dense" if dev.N * dev.M <= 1200 and layers is None else "layers"
    out = []
    for E in energies:
        z = complex(E, eta)
        sl, sr, _ = self_energies(dev.left, dev.right, z)
        if method == "dense":
            r = ldos_dense(dev, z, sl, sr)
            if layers is not None:
                r = tuple(x[list(layers)] for x in r)
        else:
            r = ldos_layers(dev, z, sl, sr, range(dev.N) if layers is None else layers)
        out.append(r)
    return tuple(np.array([o[k] for o in out]) for k in range(3))
