"""Finite-bias transmission and the Landauer current on the GPU against the FP64 oracle.

The electrodes are rigidly shifted by +-V_b/2 while the device keeps its
zero-bias blocks; the current is eq. (1) of the paper by the trapezoid rule.
FP64 bar for T as for zero bias; the current within 1e-10 relative (the
Fermi factors use the device exp, the oracle numpy's).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import fp64_close, force_batched_path, log, stage

pytestmark = pytest.mark.gpu


def _bias(lib, dt, E, eta, ul, ur, precision="fp64"):
    import torch
    T, info = lib.transmission_bias(dt, torch.as_tensor(E).cuda(), eta, ul, ur, precision)
    torch.cuda.synchronize()
    return T.cpu().numpy(), info.cpu().numpy()


@pytest.mark.parametrize("N,M,distinct", [(8, 4, False), (5, 9, True), (4, 40, False), (3, 130, True),
                                          (2, 300, False)])
def test_bias_transmission_matches_oracle(lib, N, M, distinct):
    dev = synth.random_small_device(N, M, seed=300 + M, distinct_leads=distinct)
    dt = stage(dev)
    E = np.array([-1.7, -0.6, 0.2, 1.1, 2.2])
    for ul, ur in ((0.15, -0.15), (-0.3, 0.05)):
        T, info = _bias(lib, dt, E, 1e-6, ul, ur)
        ref = oracle.transmission_bias(dev, E, 1e-6, ul, ur)
        ok, rel, ab = fp64_close(T, ref)
        log(f"[bias] N={N} M={M} u=({ul},{ur}): max rel {rel:.2e}")
        assert ok and np.all(info == 0)


def _decay_device(N, M, seed):
    """Decay-weighted random layers with a separate electrode (the C2 recipe: S positive definite)."""
    layers = [synth.decay_layer(seed, i, M) for i in range(N)]
    lead = synth.decay_layer(seed + 100, 0, M)
    return synth.device_from_blocks([l.H00 for l in layers], [l.H01 for l in layers[:-1]],
                                    [l.S00 for l in layers], [l.S01 for l in layers[:-1]], lead, lead)


@pytest.mark.parametrize("N,M", [(4, 40), (3, 130)])
def test_bias_mixed_precision_within_the_mixed_bar(lib, N, M):
    """The precision form at finite bias: |dT| <= 1e-4 against the FP64 oracle (on the
    well-conditioned decay-weighted recipe the bar is stated for)."""
    dev = _decay_device(N, M, seed=350 + M)
    E = np.array([-1.2, -0.3, 0.4, 1.3])
    T, info = _bias(lib, stage(dev), E, 1e-6, 0.1, -0.1, "mixed")
    ref = oracle.transmission_bias(dev, E, 1e-6, 0.1, -0.1)
    log(f"[bias] mixed N={N} M={M}: max |dT| {np.abs(T - ref).max():.2e}")
    assert np.all(np.abs(T - ref) <= 1e-4) and np.all(info == 0)


def test_bias_small_block_path_and_batched_path_agree(lib):
    dev = synth.random_small_device(6, 7, seed=71)
    dt = stage(dev)
    E = np.array([-1.0, 0.3, 1.6])
    a, _ = _bias(lib, dt, E, 1e-6, 0.2, -0.2)
    with force_batched_path():
        b, _ = _bias(lib, dt, E, 1e-6, 0.2, -0.2)
    ref = oracle.transmission_bias(dev, E, 1e-6, 0.2, -0.2)
    assert fp64_close(a, ref)[0] and fp64_close(b, ref)[0]


def test_zero_bias_is_rgf_transmission_bitwise(lib):
    import torch
    dev = synth.random_small_device(4, 70, seed=5, distinct_leads=True)
    dt = stage(dev)
    E = torch.as_tensor(np.array([-0.8, 0.4, 1.3])).cuda()
    T0, _ = lib.transmission(dt, E, 1e-6)
    T1, _ = lib.transmission_bias(dt, E, 1e-6, 0.0, 0.0)
    torch.cuda.synchronize()
    assert torch.equal(T0, T1)


def test_current_matches_oracle(lib):
    import torch
    dev = synth.random_small_device(5, 24, seed=88, distinct_leads=True)
    dt = stage(dev)
    E = np.linspace(-0.6, 0.6, 121)
    EF, V, kT = 0.05, 0.4, 0.025
    T, info, I = lib.current(dt, torch.as_tensor(E).cuda(), 1e-6, EF, V, kT)
    torch.cuda.synchronize()
    T_ref, I_ref = oracle.current(dev, E, 1e-6, EF, V, kT)
    log(f"[bias] current {I.item():.6e} A vs oracle {I_ref:.6e} A")
    assert fp64_close(T.cpu().numpy(), T_ref)[0]
    assert abs(I.item() - I_ref) <= 1e-10 * abs(I_ref)


def test_landauer_kernel_unit_transmission(lib):
    import torch
    E = torch.linspace(-1.0, 1.0, 40001, dtype=torch.float64, device="cuda")
    T = torch.ones_like(E)
    for ml, mr, kT in ((0.1, -0.1, 0.0259), (0.05, -0.15, 0.01)):
        I = lib.landauer_current(E, T, ml, mr, kT).item()
        assert abs(I - oracle.G0 * (ml - mr)) <= 1e-9 * oracle.G0 * abs(ml - mr)
    assert lib.landauer_current(E, T, 0.1, 0.1, 0.02).item() == 0.0
    assert lib.landauer_current(E[:1], T[:1], 0.1, -0.1, 0.02).item() == 0.0
