"""Pins of the LDOS oracle (CPU).

The oracle computes the Mulliken-projected spectral function of the device,
rho_mu = (1/2pi) Re[A S]_mu,mu with A = i (G - G^dagger), and the
electrode-injected parts rho^X from A_X = G Gamma_X G^dagger.  Each pin is
fixed by algebra or by a closed form: the Lorentzian sum over the
generalized eigenvalues of an isolated device, the 1D-chain density of
states, decoupled chains under a change of basis, the exact sum rule
A = A_L + A_R + 2 eta G S G^dagger, the orthogonal special case and the
mirror.  Planted mistakes at the end show that the pins constrain it.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle.ldos as ol
import synth

ETA = 1e-6


def _chain_dos(E, eps, t):
    """Site DOS of an infinite orthogonal chain: 1 / (pi sqrt(4 t^2 - (E - eps)^2)) in band, else 0."""
    w = 4.0 * t * t - (E - eps) ** 2
    return np.where(w > 0, 1.0 / (np.pi * np.sqrt(np.abs(w))), 0.0)


def _isolated(dev):
    """The same device with electrodes that do not couple (H01 = S01 = 0, so Sigma = 0)."""
    z = np.zeros((dev.M, dev.M), np.complex128)
    lead = synth.Lead(dev.left.H00, z, dev.left.S00, z)
    return synth.device_from_blocks([dev.Hd(i) for i in range(dev.N)], [dev.Hu(i) for i in range(dev.N - 1)],
                                    [dev.Sd(i) for i in range(dev.N)], [dev.Su(i) for i in range(dev.N - 1)],
                                    lead, lead)


def test_isolated_device_total_dos_is_the_lorentzian_sum():
    dev = _isolated(synth.random_small_device(3, 4, seed=21))
    eta = 0.05
    Afull, S = ol.device_matrix(dev, 0.0 + 0j, np.zeros((4, 4)), np.zeros((4, 4)))
    H = -Afull  # at z = 0 the device matrix is -H
    ev = sla.eigh(H, S, eigvals_only=True)
    for E in (-1.3, -0.2, 0.45, 1.7):
        rho, rl, rr = ol.local_dos(dev, [E], eta)
        expect = np.sum((eta / np.pi) / ((E - ev) ** 2 + eta ** 2))
        assert abs(rho.sum() - expect) <= 1e-10 * expect
        assert np.all(rl == 0) and np.all(rr == 0)


@pytest.mark.parametrize("E", [-1.7, -0.4, 0.3, 1.2])
def test_perfect_chain_site_dos(E):
    rho, rl, rr = ol.local_dos(synth.chain_device(6), [E], ETA)
    expect = _chain_dos(E, 0.0, -1.0)
    assert np.allclose(rho, expect, rtol=1e-5)
    # each injected wave decays by about 2 eta / v per site (absorption by the device's eta),
    # so over 6 sites the two halves differ from rho / 2 by ~1e-5 relative
    assert np.allclose(rl, expect / 2, rtol=1e-4) and np.allclose(rr, expect / 2, rtol=1e-4)


def test_perfect_chain_outside_the_band_has_no_states():
    # only the Lorentzian tails of width eta remain (Gamma itself is O(eta) outside the band)
    rho, rl, rr = ol.local_dos(synth.chain_device(5), [2.6], ETA)
    assert np.all(np.abs(rho) < 1e-5) and np.all(np.abs(rl) < 1e-5) and np.all(np.abs(rr) < 1e-5)


@pytest.mark.parametrize("E", [-1.3, 0.5])
def test_chain_with_one_electrode_ends_like_a_semi_infinite_chain(E):
    """Left electrode attached, right one decoupled: the last site is the end of a
    semi-infinite chain, rho_end = sqrt(4 t^2 - E^2) / (2 pi t^2), all of it injected from the left."""
    chain = synth.chain_device(5)
    zero = np.zeros((1, 1), np.complex128)
    right = synth.Lead(chain.right.H00, zero, chain.right.S00, zero)
    dev = synth.device_from_blocks([chain.Hd(i) for i in range(5)], [chain.Hu(i) for i in range(4)],
                                   [chain.Sd(i) for i in range(5)], [chain.Su(i) for i in range(4)],
                                   chain.left, right)
    rho, rl, rr = ol.local_dos(dev, [E], ETA)
    assert abs(rho[0, -1, 0] - np.sqrt(4.0 - E * E) / (2.0 * np.pi)) <= 1e-5 * rho[0, -1, 0]
    assert np.all(rr == 0) and np.allclose(rl, rho, rtol=1e-4)


def test_decoupled_chains_under_a_basis_change_give_chain_dos_per_layer():
    eps = np.array([-0.5, 0.0, 0.4, 1.1])
    t = np.array([-1.0, -0.6, -0.8, -0.5])
    dev = synth.decoupled_chains(eps, t, 5).with_basis_change(synth.random_basis(4, seed=12))
    for E in (-0.9, 0.2, 1.0):
        rho, rl, rr = ol.local_dos(dev, [E], ETA)
        expect = sum(_chain_dos(E, e, tt) for e, tt in zip(eps, t))
        assert np.allclose(rho[0].sum(axis=1), expect, rtol=1e-5)
        assert np.allclose(rl[0].sum(axis=1), expect / 2, rtol=1e-4)
        assert np.allclose(rr[0].sum(axis=1), expect / 2, rtol=1e-4)


def test_sum_rule_with_the_device_broadening():
    """rho - rho_L - rho_R = (eta / pi) Re diag(G S G^dagger S), exactly."""
    dev = synth.random_small_device(4, 5, seed=31, distinct_leads=True)
    eta = 0.02
    for E in (-0.8, 0.6):
        z = complex(E, eta)
        sl, sr, _ = ol.self_energies(dev.left, dev.right, z)
        Afull, S = ol.device_matrix(dev, z, sl, sr)
        G = np.linalg.solve(Afull, np.eye(len(Afull)))
        extra = (eta / np.pi) * np.real(np.diag(G @ S @ G.conj().T @ S)).reshape(dev.N, dev.M)
        rho, rl, rr = ol.local_dos(dev, [E], eta)
        assert np.allclose(rho[0] - rl[0] - rr[0], extra, rtol=0, atol=1e-11 * np.abs(rho).max())


def test_orthogonal_basis_reduces_to_minus_im_g_over_pi():
    base = synth.random_small_device(3, 4, seed=41, distinct_leads=True)
    eye, zero = np.eye(4, dtype=np.complex128), np.zeros((4, 4), np.complex128)
    lead = lambda L: synth.Lead(L.H00, L.H01, eye, zero)
    dev = synth.device_from_blocks([base.Hd(i) for i in range(3)], [base.Hu(i) for i in range(2)],
                                   [eye] * 3, [zero] * 2, lead(base.left), lead(base.right))
    E = 0.35
    z = complex(E, ETA)
    sl, sr, _ = ol.self_energies(dev.left, dev.right, z)
    Afull, _ = ol.device_matrix(dev, z, sl, sr)
    g_diag = np.diag(np.linalg.solve(Afull, np.eye(12)))
    rho, _, _ = ol.local_dos(dev, [E], ETA)
    assert np.allclose(rho[0].ravel(), -g_diag.imag / np.pi, rtol=1e-12, atol=0)


def test_mirror_exchanges_the_injecting_electrodes():
    dev = synth.random_small_device(4, 3, seed=51, distinct_leads=True)
    E = [-0.6, 0.9]
    rho, rl, rr = ol.local_dos(dev, E, ETA)
    mrho, mrl, mrr = ol.local_dos(dev.mirrored(), E, ETA)
    assert np.allclose(mrho[:, ::-1], rho, rtol=1e-9) and np.allclose(mrl[:, ::-1], rr, rtol=1e-9)
    assert np.allclose(mrr[:, ::-1], rl, rtol=1e-9)


def test_total_injected_dos_is_nonnegative():
    dev = synth.random_small_device(5, 6, seed=61, distinct_leads=True)
    rho, rl, rr = ol.local_dos(dev, np.linspace(-2, 2, 9), ETA)
    assert np.all(rl.sum(axis=(1, 2)) >= -1e-12) and np.all(rr.sum(axis=(1, 2)) >= -1e-12)
    assert np.all(rho.sum(axis=(1, 2)) >= -1e-12)


def test_block_columns_equal_the_dense_inverse():
    dev = synth.random_small_device(6, 7, seed=71, distinct_leads=True)
    E = [-1.1, 0.2, 1.4]
    d = ol.local_dos(dev, E, ETA, method="dense")
    b = ol.local_dos(dev, E, ETA, method="layers")
    for x, y in zip(d, b):
        assert np.allclose(x, y, rtol=1e-9, atol=1e-12 * np.abs(x).max())
    sel = ol.local_dos(dev, E, ETA, method="layers", layers=[0, 3, 5])
    for x, y in zip(d, sel):
        assert np.allclose(x[:, [0, 3, 5]], y, rtol=1e-9, atol=1e-12 * np.abs(x).max())


# ------------------------------------------------------------- planted mistakes
def _pins_hold() -> bool:
    try:
        test_isolated_device_total_dos_is_the_lorentzian_sum()
        for E in (-1.7, 0.3):
            test_perfect_chain_site_dos(E)
        test_decoupled_chains_under_a_basis_change_give_chain_dos_per_layer()
        test_chain_with_one_electrode_ends_like_a_semi_infinite_chain(0.5)
        test_mirror_exchanges_the_injecting_electrodes()
        test_total_injected_dos_is_nonnegative()
    except AssertionError:
        return False
    return True


def test_pins_hold_for_the_oracle():
    assert _pins_hold()


def test_planted_mistakes_are_caught(monkeypatch):
    orig_mulliken, orig_broadening, orig_matrix = ol._mulliken, ol.broadening, ol.device_matrix
    # the projection without the overlap
    monkeypatch.setattr(ol, "_mulliken", lambda X, S: np.real(np.diag(X)) / (2 * np.pi))
    assert not _pins_hold()
    monkeypatch.setattr(ol, "_mulliken", orig_mulliken)
    # Gamma with the wrong sign
    monkeypatch.setattr(ol, "broadening", lambda s: -orig_broadening(s))
    assert not _pins_hold()
    monkeypatch.setattr(ol, "broadening", orig_broadening)
    # the projection with a transposed overlap
    monkeypatch.setattr(ol, "_mulliken", lambda X, S: orig_mulliken(X, S.T))
    assert not _pins_hold()
    monkeypatch.setattr(ol, "_mulliken", orig_mulliken)

    # the electrodes' self-energies attached to the opposite ends
    def swapped(dev, z, sl, sr):
        return orig_matrix(dev, z, sr, sl)
    monkeypatch.setattr(ol, "device_matrix", swapped)
    assert not _pins_hold()
    monkeypatch.setattr(ol, "device_matrix", orig_matrix)
    assert _pins_hold()
