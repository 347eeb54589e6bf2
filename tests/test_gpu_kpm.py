"""Nonorthogonal KPM on the GPU against the FP64 oracle, through the C-ABI.

The moments of S^-1 (H - b S) / a from the same random vectors must agree
with the oracle's dense-solve recursion element by element: a moment is a
sum over N M R terms of magnitude <= |r|^2 |T_n| <= 1 after the division by
R, and the Chebyshev recursion is stable on [-1, 1] (errors grow at most
linearly in n), so the bar is |mu_gpu - mu_oracle| <= 1e-10 N M.  The Fermi
level is the bisection of the Jackson-smoothed state count; on the GPU's own
moments it must equal the oracle's bisection to 1e-9 (the count is a fixed
function of the moments, evaluated in another summation order).
"""
import numpy as np
import pytest

import oracle.kpm as ok
import synth
from gpu_helpers import log, stage

pytestmark = pytest.mark.gpu


def _device(N, M, seed):
    """Decay-weighted random layers (the C2 recipe) with a positive-definite overlap."""
    layers = [synth.decay_layer(seed, i, M) for i in range(N)]
    return synth.device_from_blocks([l.H00 for l in layers], [l.H01 for l in layers[:-1]],
                                    [l.S00 for l in layers], [l.S01 for l in layers[:-1]],
                                    layers[0], layers[0])


def _vectors(n, R, seed):
    rng = np.random.default_rng(seed)
    return np.exp(2j * np.pi * rng.random((n, R)))


def _bounds(dev):
    import scipy.linalg as sla
    H, S = ok.central_matrices(dev)
    ev = sla.eigh(H, S, eigvals_only=True)
    return ev[0] - 0.1, ev[-1] + 0.1, ev


@pytest.mark.parametrize("N,M,R,n_mom", [(1, 5, 3, 40), (3, 16, 8, 64), (4, 40, 70, 50), (3, 70, 16, 33),
                                         (2, 130, 5, 20)])
def test_kpm_moments_match_oracle(lib, N, M, R, n_mom):
    import torch
    dev = _device(N, M, seed=900 + M)
    lo, hi, _ = _bounds(dev)
    r = _vectors(N * M, R, seed=M)
    mu = lib.kpm_moments(stage(dev), lo, hi, n_mom, torch.as_tensor(r).cuda())
    torch.cuda.synchronize()
    ref = ok.moments(dev, lo, hi, n_mom, r)
    err = np.abs(mu.cpu().numpy() - ref)
    log(f"[kpm] N={N} M={M} R={R} n_mom={n_mom}: max |dmu| {err.max():.2e} (mu_0 {ref[0]:.3f})")
    assert np.all(err <= 1e-10 * N * M)


def test_kpm_fermi_level_and_dos_match_oracle(lib):
    import torch
    dev = _device(4, 12, seed=77)
    lo, hi, ev = _bounds(dev)
    n = dev.N * dev.M
    r = np.sqrt(n) * np.eye(n, dtype=np.complex128)  # exact trace
    n_mom = 300
    mu = lib.kpm_moments(stage(dev), lo, hi, n_mom, torch.as_tensor(r).cuda())
    k = int(np.argmax(np.diff(ev)))
    ef = lib.kpm_fermi(mu, lo, hi, k + 1)
    E = torch.linspace(lo + 0.05, hi - 0.05, 37, dtype=torch.float64, device="cuda")
    rho = lib.kpm_dos(mu, lo, hi, E)
    torch.cuda.synchronize()
    mu_h = mu.cpu().numpy()
    ef_ref = ok.fermi_level(mu_h, lo, hi, k + 1)
    log(f"[kpm] e_F gpu {ef.item():.12f} oracle {ef_ref:.12f}, gap ({ev[k]:.4f}, {ev[k + 1]:.4f})")
    assert abs(ef.item() - ef_ref) <= 1e-9 * max(1.0, abs(ef_ref))
    assert ev[k] < ef.item() < ev[k + 1]
    rho_ref = ok.dos(mu_h, lo, hi, E.cpu().numpy())
    assert np.allclose(rho.cpu().numpy(), rho_ref, rtol=1e-10, atol=1e-12 * np.abs(rho_ref).max())


def test_kpm_moments_are_deterministic(lib):
    import torch
    dev = _device(5, 24, seed=3)
    lo, hi, _ = _bounds(dev)
    dev_t = stage(dev)
    r = torch.as_tensor(_vectors(5 * 24, 10, seed=1)).cuda()
    a = lib.kpm_moments(dev_t, lo, hi, 30, r)
    b = lib.kpm_moments(dev_t, lo, hi, 30, r)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_kpm_argument_errors(lib):
    import torch
    dt = stage(synth.random_small_device(2, 4, seed=2))
    r = torch.ones((8, 2), dtype=torch.complex128, device="cuda")
    with pytest.raises(lib.RgfError):
        lib.kpm_moments(dt, 1.0, -1.0, 10, r)
    with pytest.raises(lib.RgfError):
        lib.kpm_moments(dt, -1.0, 1.0, 0, r)
    with pytest.raises(ValueError):
        lib.kpm_moments(dt, -1.0, 1.0, 10, r[:7])
