"""FP64 reference implementation of the transmission path, written for clarity.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
uses this module.

What is computed, and where it comes from
-----------------------------------------
The paper (Introduction; Results, the paragraph on the linear-scaling cost
of each stage; Fig. 1(b)) evaluates the zero-bias transmission T(E) of a
device with a static, nonorthogonal Hamiltonian (H, S) coupled to two
semi-infinite electrodes whose self-energies come from the bulk electrode,
using the recursive Green's function method over N_z principal layers of
M_b orbitals, at a cost of O(N_z M_b^3) per energy.  It prints no formula
for this stage, so the definitions below are the textbook ones:

* retarded device Green's function G = (z S - H - Sigma_L (+) Sigma_R)^-1,
  z = E + i eta, with eta entering both the device and the leads and
  multiplying S (Datta, *Electronic Transport in Mesoscopic Systems*);
* lead surface Green's functions by Lopez Sancho - Lopez Sancho - Rubio
  decimation (J. Phys. F 15, 851 (1985)), cross-checked against the Bloch
  (transfer-matrix) construction from the modes of the lead;
* Sigma_L = L_L g_L U_L, Sigma_R = U_R g_R L_R, with U = z S01 - H01 and
  L = z S01^dagger - H01^dagger of the lead, Gamma = i (Sigma - Sigma^dagger);
* Caroli formula T = Re Tr[Gamma_L G_1N Gamma_R G_1N^dagger]
  (Caroli et al., J. Phys. C 4, 916 (1971); Meir-Wingreen, PRL 68, 2512).

RGF reaches exactly the result of dense linear algebra (it is block
Gaussian elimination), so the oracle computes that plain definition: by a
dense solve of the whole (z S - H - Sigma) for small devices, and by a
block-Thomas direct solve (block LU of the tridiagonal system, then block
back-substitution for one block column) for large ones.  Every solve is a
LAPACK call through numpy/scipy; nothing is blocked, fused or reordered.
Sancho-Rubio is an iteration, so it is written out step by step.

Block conventions match ``synth``: Hu[i] = H_{i,i+1}; lead H01 couples
layer n to n+1 in +z for both leads; device layer 0 couples to the left
lead's surface through the left lead's (H01, S01), and device layer N-1 to
the right lead's surface through the right lead's (H01, S01).
"""
from __future__ import annotations

from typing import Tuple

import numpy as np
import scipy.linalg as sla

SR_TOL = 1e-14
SR_MAXIT = 100


def lead_operators(lead, z: complex):
    """D = z S00 - H00, U = z S01 - H01 (layer n -> n+1), L = z S01^+ - H01^+ (n+1 -> n)."""
    D = z * lead.S00 - lead.H00
    U = z * lead.S01 - lead.H01
    L = z * lead.S01.conj().T - lead.H01.conj().T
    return D, U, L


def sancho_rubio(lead, z: complex, tol: float = SR_TOL, maxit: int = SR_MAXIT):
    """Surface Green's functions of a semi-infinite lead by decimation.

    Returns (g_left, g_right, iterations, converged):
    g_right is the surface GF of a lead whose bulk lies at +z (used for the
    right electrode), g_left of a lead whose bulk lies at -z (left electrode).

    Each step eliminates every other layer of the chain: with the effective
    on-site block eps and couplings alpha (towards +z), beta (towards -z),
        eps_R <- eps_R - alpha eps^-1 beta
        eps_L <- eps_L - beta eps^-1 alpha
        eps   <- eps - alpha eps^-1 beta - beta eps^-1 alpha
        alpha <- -alpha eps^-1 alpha,  beta <- -beta eps^-1 beta
    (the sign of alpha, beta is immaterial).  It stops when
    ||alpha||_F + ||beta||_F <= tol * max(1, ||D||_F).
    """
    D, U, L = lead_operators(lead, z)
    eps = D.copy()
    eps_r = D.copy()
    eps_l = D.copy()
    alpha = U.copy()
    beta = L.copy()
    scale = max(1.0, np.linalg.norm(D))
    converged = False
    it = 0
    while it < maxit:
        it += 1
        lu = sla.lu_factor(eps)
        x_alpha = sla.lu_solve(lu, alpha)
        x_beta = sla.lu_solve(lu, beta)
        a_xb = alpha @ x_beta
        b_xa = beta @ x_alpha
        eps_r = eps_r - a_xb
        eps_l = eps_l - b_xa
        eps = eps - a_xb - b_xa
        alpha = -(alpha @ x_alpha)
        beta = -(beta @ x_beta)
        if np.linalg.norm(alpha) + np.linalg.norm(beta) <= tol * scale:
            converged = True
            break
    g_left = np.linalg.inv(eps_l)
    g_right = np.linalg.inv(eps_r)
    return g_left, g_right, it, converged


def surface_gf_bloch(lead, z: complex) -> Tuple[np.ndarray, np.ndarray]:
    """Surface GFs from the lead's Bloch modes (independent of decimation).

    A solution psi_n = lambda^n c of the lead equations satisfies
    (L + lambda D + lambda^2 U) c = 0.  Linearised as the 2M x 2M pencil
    [[0, I], [-L, -D]] v = lambda [[I, 0], [0, U]] v with v = (c, lambda c).
    For eta > 0 exactly M modes decay towards +z (|lambda| < 1); with them
    F = C Lambda C^-1 propagates psi_n -> psi_{n+1} and the right surface GF
    is (D + U F)^-1.  The M modes with |lambda| > 1 decay towards -z and give
    F~ = C Lambda^-1 C^-1 (psi_n -> psi_{n-1}), left surface GF (D + L F~)^-1.
    """
    D, U, L = lead_operators(lead, z)
    M = D.shape[0]
    I = np.eye(M)
    Z = np.zeros((M, M))
    A = np.block([[Z, I], [-L, -D]])
    B = np.block([[I, Z], [Z, U]])
    lam, vec = sla.eig(A, B)
    mag = np.abs(lam)
    order = np.argsort(mag)
    inner = order[:M]
    outer = order[M:]
    if not (np.all(mag[inner] < 1.0) and np.all(mag[outer] > 1.0)):
        raise ValueError("Bloch modes do not split into M decaying + M growing modes")
    C_in = vec[:M, inner]
    F = C_in @ np.diag(lam[inner]) @ np.linalg.inv(C_in)
    C_out = vec[:M, outer]
    F_back = C_out @ np.diag(1.0 / lam[outer]) @ np.linalg.inv(C_out)
    g_right = np.linalg.inv(D + U @ F)
    g_left = np.linalg.inv(D + L @ F_back)
    return g_left, g_right


def dyson_residual(lead, z: complex, g: np.ndarray, side: str) -> float:
    """|| g (D - X g Y) - I ||_F for the surface Dyson equation of one side.

    Right surface (bulk at +z): g = (D - U g L)^-1; left surface: g = (D - L g U)^-1.
    """
    D, U, L = lead_operators(lead, z)
    if side == "right":
        r = g @ (D - U @ g @ L)
    else:
        r = g @ (D - L @ g @ U)
    return float(np.linalg.norm(r - np.eye(D.shape[0])))


def self_energies(left_lead, right_lead, z: complex, tol: float = SR_TOL,
                  maxit: int = SR_MAXIT, method: str = "sancho_rubio"):
    """Sigma_L = L_L g_L U_L and Sigma_R = U_R g_R L_R (device-side blocks).

    Returns (Sigma_L, Sigma_R, info) with info = {"iters_left", "iters_right",
    "converged_left", "converged_right"}.
    """
    info = {}
    if method == "bloch":
        gl, _ = surface_gf_bloch(left_lead, z)
        _, gr = surface_gf_bloch(right_lead, z)
        info.update(iters_left=0, iters_right=0, converged_left=True, converged_right=True)
    else:
        gl, gr_same, itl, okl = sancho_rubio(left_lead, z, tol, maxit)
        if right_lead is left_lead:
            gr, itr, okr = gr_same, itl, okl
        else:
            _, gr, itr, okr = sancho_rubio(right_lead, z, tol, maxit)
        info.update(iters_left=itl, iters_right=itr, converged_left=okl, converged_right=okr)
    _, UL, LL = lead_operators(left_lead, z)
    _, UR, LR = lead_operators(right_lead, z)
    sigma_l = LL @ gl @ UL
    sigma_r = UR @ gr @ LR
    return sigma_l, sigma_r, info


def broadening(sigma: np.ndarray) -> np.ndarray:
    """Gamma = i (Sigma - Sigma^dagger)."""
    return 1j * (sigma - sigma.conj().T)


def _device_ops(dev, z: complex, i: int):
    """A_ii, U_i = A_{i,i+1}, L_{i+1} = A_{i+1,i} of the device (z S - H)."""
    A = z * dev.Sd(i) - dev.Hd(i)
    if i < dev.N - 1:
        U = z * dev.Su(i) - dev.Hu(i)
        L = z * dev.Su(i).conj().T - dev.Hu(i).conj().T
    else:
        U = L = None
    return A, U, L


def _caroli(gamma_a, G, gamma_b) -> complex:
    """Tr[Gamma_a G Gamma_b G^dagger] (complex; the real part is the transmission)."""
    return np.trace(gamma_a @ G @ gamma_b @ G.conj().T)


def transmission_dense(dev, z: complex, sigma_l, sigma_r, direction: str = "LR") -> complex:
    """Caroli transmission from a dense solve of the whole device (small devices only).

    Builds the NM x NM matrix (z S - H - Sigma_L (+) 0 (+) Sigma_R) and solves
    for the last block column (LR: G_1N) or the first (RL: G_N1).
    """
    N, M = dev.N, dev.M
    A = np.zeros((N * M, N * M), np.complex128)
    for i in range(N):
        Aii, U, L = _device_ops(dev, z, i)
        A[i * M:(i + 1) * M, i * M:(i + 1) * M] = Aii
        if U is not None:
            A[i * M:(i + 1) * M, (i + 1) * M:(i + 2) * M] = U
            A[(i + 1) * M:(i + 2) * M, i * M:(i + 1) * M] = L
    A[:M, :M] -= sigma_l
    A[(N - 1) * M:, (N - 1) * M:] -= sigma_r
    gl, gr = broadening(sigma_l), broadening(sigma_r)
    rhs = np.zeros((N * M, M), np.complex128)
    if direction == "LR":
        rhs[(N - 1) * M:] = np.eye(M)
        col = np.linalg.solve(A, rhs)
        return _caroli(gl, col[:M], gr)
    rhs[:M] = np.eye(M)
    col = np.linalg.solve(A, rhs)
    return _caroli(gr, col[(N - 1) * M:], gl)


def transmission_block_thomas(dev, z: complex, sigma_l, sigma_r, direction: str = "LR") -> complex:
    """Caroli transmission from a block-tridiagonal direct solve.

    LR: block LU from the top, D'_0 = A_00 - Sigma_L,
    D'_i = A_ii - L_i D'_{i-1}^-1 U_{i-1} (- Sigma_R at i = N-1), keeping each
    LU factorisation; then back-substitution for the last block column,
    X_{N-1} = D'_{N-1}^-1, X_i = -D'_i^-1 U_i X_{i+1}; G_1N = X_0.
    RL: the same from the bottom for the first block column; G_N1 = X_{N-1}.
    Every inverse is applied as an LU solve; none is formed explicitly.
    """
    N, M = dev.N, dev.M
    gam_l, gam_r = broadening(sigma_l), broadening(sigma_r)
    ops = [_device_ops(dev, z, i) for i in range(N)]
    I = np.eye(M)
    if direction == "LR":
        lus = []
        for i in range(N):
            Dp = ops[i][0].copy()
            if i == 0:
                Dp = Dp - sigma_l
            else:
                Dp = Dp - ops[i - 1][2] @ sla.lu_solve(lus[i - 1], ops[i - 1][1])
            if i == N - 1:
                Dp = Dp - sigma_r
            lus.append(sla.lu_factor(Dp))
        X = sla.lu_solve(lus[N - 1], I)
        for i in range(N - 2, -1, -1):
            X = -sla.lu_solve(lus[i], ops[i][1] @ X)
        return _caroli(gam_l, X, gam_r)
    lus = [None] * N
    for i in range(N - 1, -1, -1):
        Dp = ops[i][0].copy()
        if i == N - 1:
            Dp = Dp - sigma_r
        else:
            Dp = Dp - ops[i][1] @ sla.lu_solve(lus[i + 1], ops[i][2])
        if i == 0:
            Dp = Dp - sigma_l
        lus[i] = sla.lu_factor(Dp)
    X = sla.lu_solve(lus[0], I)
    for i in range(1, N):
        X = -sla.lu_solve(lus[i], ops[i - 1][2] @ X)
    return _caroli(gam_r, X, gam_l)


def transmission(dev, energies, eta: float, method: str = "auto", direction: str = "LR",
                 sigma_method: str = "sancho_rubio", return_info: bool = False, sr_maxit: int = SR_MAXIT):
    """T(E) = Re Tr[Gamma_L G_1N Gamma_R G_1N^dagger] at each energy (eta > 0).

    method: "dense" (full solve), "thomas" (block-tridiagonal solve) or
    "auto" (dense when N*M <= 600).  sr_maxit caps the decimation (the last
    iterate is used, and the info reports it unconverged).  Returns a float64
    array, and with ``return_info`` also the complex traces and the
    decimation info.
    """
    energies = np.atleast_1d(np.asarray(energies, np.float64))
    if method == "auto":
        method = "dense" if dev.N * dev.M <= 600 else "thomas"
    fn = transmission_dense if method == "dense" else transmission_block_thomas
    out = np.empty(len(energies), np.complex128)
    infos = []
    for k, E in enumerate(energies):
        z = complex(E, eta)
        sl, sr, info = self_energies(dev.left, dev.right, z, maxit=sr_maxit, method=sigma_method)
        out[k] = fn(dev, z, sl, sr, direction)
        infos.append(info)
    if return_info:
        return out.real.copy(), out, infos
    return out.real.copy()


def lead_bands(lead, nk: int = 4096) -> Tuple[np.ndarray, np.ndarray]:
    """Bands E_n(k) of the periodic lead from H(k) c = E S(k) c on k in (-pi, pi].

    H(k) = H00 + H01 e^{ik} + H01^+ e^{-ik}, S(k) likewise.
    """
    ks = -np.pi + 2.0 * np.pi * (np.arange(nk) + 1) / nk
    bands = np.empty((nk, lead.M))
    for j, k in enumerate(ks):
        ph = np.exp(1j * k)
        Hk = lead.H00 + lead.H01 * ph + lead.H01.conj().T / ph
        Sk = lead.S00 + lead.S01 * ph + lead.S01.conj().T / ph
        bands[j] = sla.eigh(Hk, Sk, eigvals_only=True)
    return ks, bands


def channel_count(lead, energies, nk: int = 4096, bands=None) -> np.ndarray:
    """Number of right-moving Bloch channels N_ch(E): upward crossings of E by the bands.

    With n(k) = #{bands below E at k}, each upward crossing as k increases
    lowers n by one, so N_ch = sum over the periodic k loop of max(0, n_j - n_{j+1}).
    """
    if bands is None:
        _, bands = lead_bands(lead, nk)
    energies = np.atleast_1d(energies)
    out = np.empty(len(energies), np.int64)
    for i, E in enumerate(energies):
        n = np.sum(bands < E, axis=1)
        out[i] = int(np.sum(np.maximum(0, n - np.roll(n, -1))))
    return out


def band_extrema(lead, nk: int = 4096, bands=None) -> np.ndarray:
    """Energies of local band extrema on the k grid (where channel counts jump)."""
    if bands is None:
        _, bands = lead_bands(lead, nk)
    prev = np.roll(bands, 1, axis=0)
    nxt = np.roll(bands, -1, axis=0)
    ext = ((bands >= prev) & (bands >= nxt)) | ((bands <= prev) & (bands <= nxt))
    return np.unique(bands[ext])
