"""Pins of the oracle's behaviour in the cases the per-energy status bits report.

The library reports, per energy, decimation that hit its iteration cap, an
exactly zero pivot (with the layer) and a non-finite result.  The oracle has
the same three cases; these pins fix what it does in each, against brute
force, so the GPU status tests can compare with it.
"""
import warnings

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth

ETA = 1e-6


def _finite_chain(lead, z, n):
    """Dense matrix of n lead layers: D on the diagonal, U = A_{n,n+1} above, L below."""
    D, U, L = oracle.lead_operators(lead, z)
    M = D.shape[0]
    A = np.zeros((n * M, n * M), np.complex128)
    for i in range(n):
        A[i * M:(i + 1) * M, i * M:(i + 1) * M] = D
        if i + 1 < n:
            A[i * M:(i + 1) * M, (i + 1) * M:(i + 2) * M] = U
            A[(i + 1) * M:(i + 2) * M, i * M:(i + 1) * M] = L
    return A


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_capped_decimation_is_the_finite_chain(k):
    """After k steps (cap k), decimation has eliminated every layer between the surface and
    layer 2^k: its surface GFs are those of a finite chain of 2^k layers, g_right = G_00 and
    g_left = G_last,last, by dense inversion; the oracle flags the result unconverged."""
    lead = synth.random_small_device(2, 3, seed=41).left
    z = complex(0.37, ETA)
    gl, gr, it, ok = oracle.sancho_rubio(lead, z, maxit=k)
    assert it == k and not ok
    n = 2 ** k
    G = np.linalg.inv(_finite_chain(lead, z, n))
    M = lead.M
    assert np.allclose(gr, G[:M, :M], rtol=1e-10, atol=1e-12)
    assert np.allclose(gl, G[-M:, -M:], rtol=1e-10, atol=1e-12)


def test_capped_transmission_differs_and_reports():
    """A cap far below convergence changes T and the info says which sides did not converge;
    the default cap converges on the same device."""
    dev = synth.random_small_device(3, 4, seed=12, distinct_leads=True)
    E = np.array([-0.8, 0.4])
    T0, _, info0 = oracle.transmission(dev, E, ETA, return_info=True)
    T3, _, info3 = oracle.transmission(dev, E, ETA, return_info=True, sr_maxit=3)
    assert all(i["converged_left"] and i["converged_right"] for i in info0)
    assert all(not i["converged_left"] and not i["converged_right"] and i["iters_left"] == 3 for i in info3)
    assert np.max(np.abs(T3 - T0)) > 1e-6


def _cut_layer(dev, k):
    """Layer k emptied (H_kk = S_kk = 0) and both its couplings zeroed: block row k of z S - H is
    zero, so the device matrix is exactly singular."""
    hd, hu, sd, su = dev.stacked()
    hd[k] = 0.0
    sd[k] = 0.0
    hu[k - 1] = 0.0
    su[k - 1] = 0.0
    hu[k] = 0.0
    su[k] = 0.0
    return synth.device_from_blocks(hd, hu, sd, su, dev.left, dev.right)


def test_empty_layer_is_an_exactly_singular_device():
    """The dense solve refuses the matrix; the block-Thomas elimination meets an exactly zero
    pivot at that layer (LAPACK's warning on the factorisation of D'_k) and has no finite
    result after it (its next solve refuses the non-finite factors)."""
    dev = _cut_layer(synth.random_small_device(4, 3, seed=5), 2)
    E = np.array([0.3])
    with pytest.raises(np.linalg.LinAlgError):
        oracle.transmission(dev, E, ETA, method="dense")
    with warnings.catch_warnings(record=True) as w:
        warnings.simplefilter("always")
        with pytest.raises(ValueError, match="infs or NaNs"):
            oracle.transmission(dev, E, ETA, method="thomas")
    assert any(issubclass(x.category, sla.LinAlgWarning) for x in w)
    # the same device with the layer kept has a finite T: the failure is the empty layer's
    assert np.isfinite(oracle.transmission(synth.random_small_device(4, 3, seed=5), E, ETA)[0])


def test_nan_entry_has_no_finite_transmission():
    dev = synth.random_small_device(3, 4, seed=6)
    hd, hu, sd, su = dev.stacked()
    hd[1][2, 1] = np.nan
    bad = synth.device_from_blocks(hd, hu, sd, su, dev.left, dev.right)
    with pytest.raises(ValueError, match="infs or NaNs"):
        oracle.transmission(bad, np.array([0.1, 0.9]), ETA, method="thomas")
    with np.errstate(invalid="ignore"):
        T = oracle.transmission(bad, np.array([0.1, 0.9]), ETA, method="dense")
    assert not np.any(np.isfinite(T))
