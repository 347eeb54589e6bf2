"""FP64 reference for the nonorthogonal kernel polynomial method (KPM) Fermi level.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed
----------------
The paper finds the Fermi level of the central region without
diagonalisation (Introduction; Results, the workflow paragraph and the
per-stage scaling O(N_mom N_rand N)): the generalized problem H c = e S c
is mapped onto the rescaled operator  A~ = S^-1 (H - b S) / a,  whose action
on a vector is a product with (H - b S) followed by a solve with S (S^-1 is
never formed); its Chebyshev moments, estimated with random vectors, give
the density of states, and the Fermi level follows from the electron-number
constraint.  The textbook KPM (Weisse, Wellein, Alvermann, Fehske, Rev. Mod.
Phys. 78, 275 (2006)) fixes the rest:

* a = (e_max - e_min) / (2 - eps), b = (e_max + e_min) / 2 for spectral
  bounds [e_min, e_max] (so the spectrum of A~ lies inside [-1, 1]);
* moments mu_n = Tr T_n(A~) = sum_k T_n(x_k), x_k = (e_k - b) / a, estimated
  as mu_n = (1/R) Re sum_r r^dagger T_n(A~) r over R random vectors
  (E[r r^dagger] = I), with T_0 r = r, T_1 r = A~ r, T_{n+1} r = 2 A~ T_n r - T_{n-1} r;
* the Jackson kernel g_n damps the Gibbs oscillations of the truncated series;
* the number of states below x:
  N(x) = g_0 mu_0 (pi - acos x) / pi - (2 / pi) sum_{n>=1} g_n mu_n sin(n acos x) / n;
* the Fermi level e_F = a x_F + b with N(x_F) = n_states (the number of
  occupied states, spin not counted), found by bisection;
* the density of states per unit energy rho(e) = (1/a) [g_0 mu_0 + 2 sum g_n mu_n T_n(x)] / (pi sqrt(1 - x^2)).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

KPM_EPS = 0.01


def scaling(e_min: float, e_max: float, eps: float = KPM_EPS):
    """(a, b) of the map x = (e - b) / a."""
    return (e_max - e_min) / (2.0 - eps), (e_max + e_min) / 2.0


def central_matrices(dev):
    """Dense H and S of the central region (the device blocks; the electrodes do not enter)."""
    N, M = dev.N, dev.M
    H = np.zeros((N * M, N * M), np.complex128)
    S = np.zeros((N * M, N * M), np.complex128)
    for i in range(N):
        blk = slice(i * M, (i + 1) * M)
        H[blk, blk] = dev.Hd(i)
        S[blk, blk] = dev.Sd(i)
        if i + 1 < N:
            nxt = slice((i + 1) * M, (i + 2) * M)
            H[blk, nxt] = dev.Hu(i)
            H[nxt, blk] = dev.Hu(i).conj().T
            S[blk, nxt] = dev.Su(i)
            S[nxt, blk] = dev.Su(i).conj().T
    return H, S


def moments(dev, e_min: float, e_max: float, n_mom: int, vectors, eps: float = KPM_EPS):
    """mu_0 .. mu_{n_mom-1} from the random vectors (columns of `vectors`, [N M, R])."""
    H, S = central_matrices(dev)
    a, b = scaling(e_min, e_max, eps)
    lu = sla.lu_factor(S)
    apply = lambda v: sla.lu_solve(lu, (H - b * S) @ v) / a
    r = np.asarray(vectors, np.complex128)
    R = r.shape[1]
    mu = np.empty(n_mom)
    v_prev, v = r, apply(r)
    mu[0] = np.real(np.vdot(r, r)) / R
    if n_mom > 1:
        mu[1] = np.real(np.vdot(r, v)) / R
    for n in range(2, n_mom):
        v_prev, v = v, 2.0 * apply(v) - v_prev
        mu[n] = np.real(np.vdot(r, v)) / R
    return mu


def jackson(n_mom: int) -> np.ndarray:
    """Jackson kernel g_0 .. g_{n_mom-1}."""
    n = np.arange(n_mom)
    q = np.pi / (n_mom + 1)
    return ((n_mom - n + 1) * np.cos(q * n) + np.sin(q * n) / np.tan(q)) / (n_mom + 1)


def states_below(mu, x) -> np.ndarray:
    """N(x): the kernel-smoothed number of states below x (x in [-1, 1])."""
    mu = np.asarray(mu, float)
    g = jackson(len(mu))
    th = np.arccos(np.clip(np.atleast_1d(np.asarray(x, float)), -1.0, 1.0))
    n = np.arange(1, len(mu))
    out = g[0] * mu[0] * (np.pi - th) / np.pi
    out = out - (2.0 / np.pi) * np.sum((g[1:] * mu[1:] / n)[None, :] * np.sin(np.outer(th, n)), axis=1)
    return out


def fermi_level(mu, e_min: float, e_max: float, n_states: float, eps: float = KPM_EPS, iters: int = 200) -> float:
    """e_F with N(x_F) = n_states, by bisection on [-1, 1]."""
    a, b = scaling(e_min, e_max, eps)
    lo, hi = -1.0, 1.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if states_below(mu, mid)[0] < n_states:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 1e-15:
            break
    return a * 0.5 * (lo + hi) + b


def dos(mu, e_min: float, e_max: float, energies, eps: float = KPM_EPS) -> np.ndarray:
    """Kernel-smoothed density of states per unit energy at the given energies."""
    mu = np.asarray(mu, float)
    a, b = scaling(e_min, e_max, eps)
    x = (np.atleast_1d(np.asarray(energies, float)) - b) / a
    g = jackson(len(mu))
    th = np.arccos(np.clip(x, -1.0, 1.0))
    n = np.arange(1, len(mu))
    s = g[0] * mu[0] + 2.0 * np.sum((g[1:] * mu[1:])[None, :] * np.cos(np.outer(th, n)), axis=1)
    return s / (np.pi * np.sqrt(np.maximum(1.0 - x * x, 1e-300)) * a)
