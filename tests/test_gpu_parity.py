"""GPU parity: the HIP path against the FP64 oracle, element by element.

FP64 bar: |T_gpu - T_oracle| <= 1e-8 |T_oracle| + 1e-12 on every energy.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import fp64_close, force_batched_path, gpu_transmission, log, stage

pytestmark = pytest.mark.gpu


def _check(dev, E, eta, tag, method="auto"):
    log(f"[parity] {tag}: N={dev.N} M={dev.M} nE={len(E)}")
    dt = stage(dev)
    T, info = gpu_transmission(dt, E, eta)
    ref = oracle.transmission(dev, E, eta, method=method)
    ok, rel, ab = fp64_close(T, ref)
    log(f"[parity] {tag}: max rel {rel:.3e} max abs {ab:.3e} info max {int(info.max())}")
    assert np.all(info == 0), info
    assert ok, (T, ref)


def test_c1_small_fused(lib):
    cfg = synth.config_c1()
    _check(cfg.device, cfg.energies, cfg.eta, "c1-small", method="dense")


def test_c1_batched_path(lib):
    cfg = synth.config_c1()
    with force_batched_path():
        _check(cfg.device, cfg.energies, cfg.eta, "c1-batched", method="dense")


@pytest.mark.parametrize("N,M", [(1, 5), (2, 9), (5, 13), (1, 20), (3, 40), (6, 70), (4, 130)])
def test_random_devices_distinct_leads(lib, N, M):
    dev = synth.random_small_device(N, M, seed=100 + 7 * N + M, distinct_leads=True)
    E = np.array([-2.3, -1.1, -0.37, 0.52, 1.4, 2.6])
    _check(dev, E, 1e-6, f"rand-{N}x{M}")


def test_mirror_equals_oracle_reverse(lib):
    dev = synth.random_small_device(5, 24, seed=77, distinct_leads=True)
    E = np.array([-1.6, -0.2, 0.9])
    T, _ = gpu_transmission(stage(dev.mirrored()), E, 1e-6)
    ref = oracle.transmission(dev, E, 1e-6, direction="RL")
    ok, rel, ab = fp64_close(T, ref)
    log(f"[parity] mirror: max rel {rel:.3e}")
    assert ok


def test_lead_self_energy_matches_oracle(lib):
    import torch
    from paper_2609_37058_amd import rgf, staging
    lead = synth.decay_layer(102, 0, 72)
    lt = staging.stage_lead(lead.H00, lead.H01, lead.S00, lead.S01)
    E = np.array([-1.5, -0.1, 0.8, 1.9])
    Et = torch.as_tensor(E).cuda()
    for side in (rgf.RGF_LEFT, rgf.RGF_RIGHT):
        sig, info = rgf.lead_self_energy(lt, side, Et, 1e-6)
        torch.cuda.synchronize()
        sig = sig.cpu().numpy()
        for k, e in enumerate(E):
            sl, sr, _ = oracle.self_energies(lead, lead, complex(e, 1e-6))
            ref = sl if side == rgf.RGF_LEFT else sr
            err = np.linalg.norm(sig[k] - ref) / np.linalg.norm(ref)
            log(f"[parity] sigma side={side} E={e}: rel {err:.2e}")
            assert err < 1e-9
        assert np.all(info.cpu().numpy() == 0)


def test_blocks_above_1024(lib):
    """M = 1100 (padded 1152: the four-rows-per-thread panel) against the oracle; a broad eta keeps
    the oracle's decimation of the 1100-orbital electrode short."""
    layers = [synth.decay_layer(61, i, 1100) for i in range(2)]
    lead = synth.decay_layer(161, 0, 1100)
    dev = synth.device_from_blocks([l.H00 for l in layers], [layers[0].H01], [l.S00 for l in layers],
                                   [layers[0].S01], lead, lead)
    E = np.array([-0.4, 0.7])
    T, info = gpu_transmission(stage(dev), E, 0.05)
    ref = oracle.transmission(dev, E, 0.05, method="thomas")
    ok, rel, ab = fp64_close(T, ref)
    log(f"[parity] M=1100: max rel {rel:.2e} max abs {ab:.2e}")
    assert ok and np.all(info == 0)


def test_input_checks(lib):
    """rgf_check_device accepts the Hermitian test devices and names the first block that is
    not Hermitian or whose overlap diagonal is not positive; with rgf_set_checks(1) the
    transmission call fails the same way, and without it runs."""
    import torch
    dev = synth.random_small_device(4, 70, seed=12, distinct_leads=True)
    E = torch.linspace(-1.0, 1.0, 3, dtype=torch.float64, device="cuda")
    dt = stage(dev)
    assert lib.check_device(dt) <= 1e-14
    bad = stage(dev)
    bad.Hd[2, 5, 9] += 0.3  # breaks H_22 = H_22^+
    with pytest.raises(lib.RgfError, match="H_ii of layer 2"):
        lib.check_device(bad)
    neg = stage(dev)
    neg.Sd[1].mul_(-1.0)  # Hermitian, but not positive
    with pytest.raises(lib.RgfError, match="overlap diagonal"):
        lib.check_device(neg)
    T0, _ = lib.transmission(bad, E, 1e-6)  # unchecked calls run on any input
    torch.cuda.synchronize()
    lib.set_checks(True)
    try:
        with pytest.raises(lib.RgfError, match="not Hermitian"):
            lib.transmission(bad, E, 1e-6)
        T, _ = lib.transmission(dt, E, 1e-6)
        torch.cuda.synchronize()
        assert torch.isfinite(T).all()
        r = torch.ones((dev.N * dev.M, 2), dtype=torch.complex128, device="cuda")
        with pytest.raises(lib.RgfError, match="overlap diagonal"):
            lib.kpm_moments(neg, -10.0, 10.0, 4, r)
    finally:
        lib.set_checks(False)


@pytest.mark.parametrize("M", [8, 40])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_zero_coupling_block_gives_zero(lib, M, precision):
    """A device cut in two by a zero coupling block (H_{2,3} = S_{2,3} = 0) transmits nothing:
    T = 0 exactly on every energy (the oracle's pin of the same case), with no info bit set."""
    import torch
    from paper_2609_37058_amd import staging
    dev = synth.random_small_device(5, M, seed=300 + M, distinct_leads=True)
    hd, hu, sd, su = dev.stacked()
    hu[2] = 0.0
    su[2] = 0.0
    L, R = dev.left, dev.right
    dt = staging.stage_blocks(hd, hu, sd, su, staging.stage_lead(L.H00, L.H01, L.S00, L.S01),
                              staging.stage_lead(R.H00, R.H01, R.S00, R.S01))
    E = torch.as_tensor(np.array([-1.7, -0.4, 0.3, 1.2])).cuda()
    T, info = lib.transmission(dt, E, 1e-6, precision)
    torch.cuda.synchronize()
    log(f"[parity] zero coupling M={M} {precision}: T={T.cpu().numpy()}")
    assert torch.all(T == 0.0) and torch.all(info == 0)


def test_empty_energy_grid(lib):
    """nE = 0 is legal: nothing is launched and the outputs are empty."""
    import torch
    dt = stage(synth.random_small_device(3, 20, seed=5))
    T, info = lib.transmission(dt, torch.empty(0, dtype=torch.float64, device="cuda"), 1e-6)
    torch.cuda.synchronize()
    assert T.numel() == 0 and info.numel() == 0


@pytest.mark.parametrize("M,lanes", [(300, "1"), (520, "2")])
def test_lu_lookahead_equals_plain(lib, M, lanes, monkeypatch):
    """RGF_LOOKAHEAD=1: the blocked LU updates the columns beyond the next pair of panels on a
    side stream (per lane) while the lane factors that pair; the results are the same bits as
    without it, and match the oracle."""
    dev = synth.random_small_device(3, M, seed=500 + M)
    E = np.linspace(-1.0, 1.0, 8)
    st = stage(dev)
    monkeypatch.setenv("RGF_LANES", lanes)
    plain, info0 = gpu_transmission(st, E, 1e-6)
    monkeypatch.setenv("RGF_LOOKAHEAD", "1")
    log(f"[parity] look-ahead M={M} lanes={lanes}")
    ahead, info1 = gpu_transmission(st, E, 1e-6)
    assert np.all(info0 == 0) and np.all(info1 == 0)
    assert np.array_equal(plain, ahead)
    ok, rel, ab = fp64_close(ahead[:3], oracle.transmission(dev, E[:3], 1e-6))
    assert ok, rel
