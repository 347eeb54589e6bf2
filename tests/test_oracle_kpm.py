"""Pins of the nonorthogonal KPM oracle (CPU).

The oracle estimates Chebyshev moments of A~ = S^-1 (H - b S) / a with
random vectors, damps them with the Jackson kernel and finds the Fermi level
from the electron-number constraint.  The pins: with the unit vectors as
"random" vectors the moments are exactly sum_k T_n(x_k) over the generalized
eigenvalues; the Jackson kernel's reconstruction of one level is
nonnegative with the published width; the state count is exact in gaps; the
Fermi level lands in the gap that the state count selects; random-phase
vectors converge to the exact moments; the density of states integrates to
the dimension.  Planted mistakes at the end show that the pins constrain it.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle.kpm as ok
import synth


def _device(seed=5, N=3, M=4):
    return synth.random_small_device(N, M, seed=seed)


def _spectrum(dev):
    """Generalized eigenvalues of (H, S) of the central region, assembled here from the blocks."""
    N, M = dev.N, dev.M
    H = np.zeros((N * M, N * M), np.complex128)
    S = np.zeros_like(H)
    for i in range(N):
        H[i * M:(i + 1) * M, i * M:(i + 1) * M] = dev.Hd(i)
        S[i * M:(i + 1) * M, i * M:(i + 1) * M] = dev.Sd(i)
    for i in range(N - 1):
        H[i * M:(i + 1) * M, (i + 1) * M:(i + 2) * M] = dev.Hu(i)
        S[i * M:(i + 1) * M, (i + 1) * M:(i + 2) * M] = dev.Su(i)
    H = np.triu(H) + np.triu(H, 1).conj().T
    S = np.triu(S) + np.triu(S, 1).conj().T
    return sla.eigh(H, S, eigvals_only=True)


def _exact_vectors(n):
    """sqrt(n) e_j, j = 1..n: (1/n) sum_j r_j r_j^dagger = I exactly, so the estimate is the trace."""
    return np.sqrt(n) * np.eye(n)


def _bounds(ev, pad=0.05):
    return ev[0] - pad, ev[-1] + pad


def test_unit_vectors_give_the_exact_moments():
    dev = _device()
    ev = _spectrum(dev)
    lo, hi = _bounds(ev)
    a, b = ok.scaling(lo, hi)
    x = (ev - b) / a
    n_mom = 60
    mu = ok.moments(dev, lo, hi, n_mom, _exact_vectors(len(ev)))
    exact = np.array([np.sum(np.cos(n * np.arccos(x))) for n in range(n_mom)])
    assert np.allclose(mu, exact, rtol=0, atol=1e-10 * len(ev))
    assert np.all(np.abs(x) < 1)


def test_jackson_reconstruction_of_one_level_is_nonnegative_with_the_published_width():
    n_mom = 128
    for x0 in (0.0, 0.5, -0.7):
        mu = np.cos(np.arange(n_mom) * np.arccos(x0))  # one level at x0
        g = ok.jackson(n_mom)
        assert g[0] == pytest.approx(1.0, abs=1e-15)
        x = np.linspace(-0.999, 0.999, 4001)
        dens = ok.dos(mu, -1.0 * (2 - ok.KPM_EPS) / 2, (2 - ok.KPM_EPS) / 2, x * (2 - ok.KPM_EPS) / 2)
        assert np.all(dens >= -1e-10)
        # variance of the kernel-broadened level: (pi / N)^2 [1 - x0^2 + (3 x0^2 - 2) / N] (Weisse et al.)
        w = dens * (1 - 0)  # density in x up to the constant Jacobian
        w = w / np.trapezoid(w, x)
        var = np.trapezoid(w * (x - x0) ** 2, x)
        expect = (np.pi / n_mom) ** 2 * (1 - x0 ** 2 + (3 * x0 ** 2 - 2) / n_mom)
        assert var == pytest.approx(expect, rel=0.1)


def test_state_count_is_exact_in_gaps():
    dev = _device(seed=7)
    ev = _spectrum(dev)
    lo, hi = _bounds(ev)
    a, b = ok.scaling(lo, hi)
    mu = ok.moments(dev, lo, hi, 400, _exact_vectors(len(ev)))
    gaps = np.diff(ev)
    for k in np.argsort(gaps)[-3:]:
        if gaps[k] < 0.1 * a:
            continue
        mid = 0.5 * (ev[k] + ev[k + 1])
        assert ok.states_below(mu, (mid - b) / a)[0] == pytest.approx(k + 1, abs=2e-2)
    assert ok.states_below(mu, -1.0)[0] == pytest.approx(0.0, abs=1e-12)
    assert ok.states_below(mu, 1.0)[0] == pytest.approx(len(ev), rel=1e-12)


def test_fermi_level_lands_in_the_selected_gap():
    dev = _device(seed=11, N=4, M=3)
    ev = _spectrum(dev)
    lo, hi = _bounds(ev)
    mu = ok.moments(dev, lo, hi, 500, _exact_vectors(len(ev)))
    k = int(np.argmax(np.diff(ev)))
    ef = ok.fermi_level(mu, lo, hi, k + 1)
    assert ev[k] < ef < ev[k + 1]


def test_random_phase_vectors_converge_to_the_exact_moments():
    dev = _device(seed=13)
    ev = _spectrum(dev)
    lo, hi = _bounds(ev)
    n = len(ev)
    rng = np.random.default_rng(3)
    R = 3000
    r = np.exp(2j * np.pi * rng.random((n, R)))
    mu = ok.moments(dev, lo, hi, 12, r)
    exact = ok.moments(dev, lo, hi, 12, _exact_vectors(n))
    # a sample r^dagger X r of a random-phase vector has variance sum_{j != k} |X_jk|^2 <= n^2
    # (|T_n(A~)| entries are O(1)), so the mean over R has sigma <= n / sqrt(R)
    assert np.allclose(mu, exact, atol=5 * n / np.sqrt(R))
    assert mu[0] == pytest.approx(n)   # |r_j| = 1 exactly


def test_dos_integrates_to_the_dimension():
    dev = _device(seed=17)
    ev = _spectrum(dev)
    lo, hi = _bounds(ev)
    a, b = ok.scaling(lo, hi)
    mu = ok.moments(dev, lo, hi, 200, _exact_vectors(len(ev)))
    th = np.linspace(1e-6, np.pi - 1e-6, 20001)
    e = a * np.cos(th) + b
    # integral of rho de = integral of rho(x) a sin(th) dth over th in (0, pi)
    integral = np.trapezoid(ok.dos(mu, lo, hi, e) * a * np.sin(th), th)
    assert integral == pytest.approx(len(ev), rel=1e-6)


# ------------------------------------------------------------- planted mistakes
def _pins_hold() -> bool:
    try:
        test_unit_vectors_give_the_exact_moments()
        test_jackson_reconstruction_of_one_level_is_nonnegative_with_the_published_width()
        test_state_count_is_exact_in_gaps()
        test_fermi_level_lands_in_the_selected_gap()
        test_dos_integrates_to_the_dimension()
    except AssertionError:
        return False
    return True


def test_pins_hold_for_the_oracle():
    assert _pins_hold()


def test_planted_mistakes_are_caught(monkeypatch):
    orig_central, orig_jackson, orig_scaling = ok.central_matrices, ok.jackson, ok.scaling
    # the overlap left out of the operator (A~ = (H - b) / a)
    monkeypatch.setattr(ok, "central_matrices",
                        lambda dev: (orig_central(dev)[0], np.eye(dev.N * dev.M, dtype=np.complex128)))
    assert not _pins_hold()
    monkeypatch.setattr(ok, "central_matrices", orig_central)
    # no kernel (Dirichlet truncation)
    monkeypatch.setattr(ok, "jackson", lambda n: np.ones(n))
    assert not _pins_hold()
    monkeypatch.setattr(ok, "jackson", orig_jackson)
    # the spectral centre with the wrong sign
    monkeypatch.setattr(ok, "scaling", lambda lo, hi, eps=ok.KPM_EPS: (orig_scaling(lo, hi, eps)[0],
                                                                        -orig_scaling(lo, hi, eps)[1]))
    assert not _pins_hold()
    monkeypatch.setattr(ok, "scaling", orig_scaling)
    assert _pins_hold()
