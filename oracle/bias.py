"""FP64 reference for finite-bias transport with the zero-bias Hamiltonian, and the current.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed
----------------
The paper's current formula (Method, eq. (1)) is the Landauer integral

    I(V_b) = (2e/h) * integral dE [f(E, mu_L) - f(E, mu_R)] T(E, V_b),

with f the Fermi-Dirac distribution of each electrode at its
electrochemical potential.  For weakly nonlinear devices the paper feeds the
zero-bias Hamiltonian H0 straight into the NEGF solver at finite bias
(Method, the paragraph after eq. (1)), i.e. no self-consistent potential is
computed.  The reading taken here (it is not spelled out in the paper):

* the device blocks stay those of H0;
* each electrode is rigidly shifted by the bias part of its potential
  energy, u_X = mu_X - E_F (u_L = +V_b/2, u_R = -V_b/2 for a symmetric
  bias): H00 -> H00 + u_X S00 and H01 -> H01 + u_X S01 (S unchanged), so its
  self-energy is the zero-bias one evaluated at E - u_X;
* T(E, V_b) is the Caroli transmission with these self-energies;
* the occupations use the electrochemical potentials mu_X = E_F + u_X;
* energies are in eV, so with G0 = 2 e^2 / h (conductance quantum including
  spin, exact SI constants) the current in amperes is G0 times the integral
  taken in eV;
* the integral is the trapezoid rule on the caller's ascending energy grid,
  which must cover the bias window plus several kT on each side.
"""
from __future__ import annotations

import numpy as np

from .rgf_oracle import (self_energies, transmission_block_thomas, transmission_dense)

E_CHARGE = 1.602176634e-19  # C (exact)
H_PLANCK = 6.62607015e-34   # J s (exact)
G0 = 2.0 * E_CHARGE ** 2 / H_PLANCK  # S: 2e^2/h, the spin-degenerate conductance quantum


def shifted_lead(lead, u: float):
    """The electrode rigidly shifted by u: H00 + u S00, H01 + u S01 (S unchanged)."""
    return type(lead)(lead.H00 + u * lead.S00, lead.H01 + u * lead.S01, lead.S00, lead.S01)


def transmission_bias(dev, energies, eta: float, u_l: float, u_r: float, method: str = "auto"):
    """T(E, V_b) of the H0 device between electrodes shifted by u_l (left) and u_r (right), in eV."""
    energies = np.atleast_1d(np.asarray(energies, np.float64))
    if method == "auto":
        method = "dense" if dev.N * dev.M <= 600 else "thomas"
    fn = transmission_dense if method == "dense" else transmission_block_thomas
    left = shifted_lead(dev.left, u_l)
    right = shifted_lead(dev.right, u_r)
    out = np.empty(len(energies))
    for k, E in enumerate(energies):
        z = complex(E, eta)
        sl, sr, _ = self_energies(left, right, z)
        out[k] = fn(dev, z, sl, sr).real
    return out


def fermi(E, mu: float, kT: float):
    """Fermi-Dirac occupation; kT = 0 gives the step (1/2 exactly at E = mu)."""
    E = np.asarray(E, np.float64)
    if kT == 0.0:
        return np.where(E < mu, 1.0, np.where(E > mu, 0.0, 0.5))
    x = (E - mu) / kT
    # 1 / (1 + e^x) written so that neither branch overflows
    return np.where(x > 0, np.exp(-np.abs(x)) / (1.0 + np.exp(-np.abs(x))), 1.0 / (1.0 + np.exp(-np.abs(x))))


def landauer_current(energies, T, mu_l: float, mu_r: float, kT: float) -> float:
    """I = G0 * trapezoid over the ascending grid of (f_L - f_R) T, in amperes."""
    energies = np.asarray(energies, np.float64)
    g = (fermi(energies, mu_l, kT) - fermi(energies, mu_r, kT)) * np.asarray(T, np.float64)
    dE = np.diff(energies)
    return float(G0 * np.sum(dE * (g[:-1] + g[1:]) / 2.0))


def current(dev, energies, eta: float, e_fermi: float, v_bias: float, kT: float, method: str = "auto"):
    """(T(E, V_b), I) for a symmetric bias: mu_L,R = E_F +- V_b/2, electrodes shifted by +-V_b/2."""
    T = transmission_bias(dev, energies, eta, v_bias / 2.0, -v_bias / 2.0, method)
    I = landauer_current(energies, T, e_fermi + v_bias / 2.0, e_fermi - v_bias / 2.0, kT)
    return T, I
