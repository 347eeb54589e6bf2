"""The batching form on the GPU: many devices of uneven size in one call, and the autotuner.

rgf_transmission_batch must give, for every device, exactly (bitwise) what
rgf_transmission gives for that device alone, and both must meet the FP64
oracle bar.  The small-block devices share one persistent launch whose
workgroups draw (device, energy) items from a work counter.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import fp64_close, log, stage

pytestmark = pytest.mark.gpu


def _single(lib, dev_t, E, eta, precision="fp64"):
    import torch
    T, info = lib.transmission(dev_t, torch.as_tensor(E).cuda(), eta, precision)
    torch.cuda.synchronize()
    return T.cpu().numpy(), info.cpu().numpy()


def _batch(lib, devs_t, Es, eta, precision="fp64"):
    import torch
    res = lib.transmission_batch(devs_t, [torch.as_tensor(E).cuda() for E in Es], eta, precision)
    torch.cuda.synchronize()
    return [(T.cpu().numpy(), i.cpu().numpy()) for T, i in res]


def _mix(specs, seed):
    rng = np.random.default_rng(seed)
    devs, Es = [], []
    for k, (N, M, nE) in enumerate(specs):
        devs.append(synth.random_small_device(N, M, seed=seed + 31 * k + M, distinct_leads=bool(k % 2)))
        Es.append(np.sort(rng.uniform(-2.5, 2.5, nE)))
    return devs, Es


def test_small_devices_share_one_persistent_launch(lib):
    specs = [(20, 4, 37), (1, 1, 5), (7, 16, 11), (3, 9, 1), (30, 2, 23), (12, 13, 8), (2, 16, 40), (5, 7, 3)]
    devs, Es = _mix(specs, 900)
    dts = [stage(d) for d in devs]
    got = _batch(lib, dts, Es, 1e-6)
    for (N, M, nE), d, dt, E, (T, info) in zip(specs, devs, dts, Es, got):
        Ts, infos = _single(lib, dt, E, 1e-6)
        ref = oracle.transmission(d, E, 1e-6)
        ok, rel, ab = fp64_close(T, ref)
        log(f"[batch] small N={N} M={M} nE={nE}: bitwise={np.array_equal(T, Ts)} max rel {rel:.2e}")
        assert np.array_equal(T, Ts) and np.array_equal(info, infos)
        assert ok and np.all(info == 0)


def test_mixed_sizes_match_single_calls_and_oracle(lib):
    specs = [(4, 130, 5), (6, 70, 9), (20, 4, 12), (3, 40, 7), (2, 200, 4), (9, 11, 6)]
    devs, Es = _mix(specs, 1700)
    dts = [stage(d) for d in devs]
    got = _batch(lib, dts, Es, 1e-6)
    for (N, M, nE), d, dt, E, (T, info) in zip(specs, devs, dts, Es, got):
        Ts, _ = _single(lib, dt, E, 1e-6)
        ref = oracle.transmission(d, E, 1e-6)
        ok, rel, ab = fp64_close(T, ref)
        log(f"[batch] mixed N={N} M={M} nE={nE}: bitwise={np.array_equal(T, Ts)} max rel {rel:.2e}")
        assert np.array_equal(T, Ts)
        assert ok and np.all(info == 0)


def test_batch_mixed_precision_equals_single_calls(lib):
    specs = [(3, 70, 4), (2, 130, 3), (5, 8, 5)]
    devs, Es = _mix(specs, 2500)
    dts = [stage(d) for d in devs]
    got = _batch(lib, dts, Es, 1e-6, "mixed")
    for d, dt, E, (T, info) in zip(devs, dts, Es, got):
        Ts, _ = _single(lib, dt, E, 1e-6, "mixed")
        assert np.array_equal(T, Ts)
        ref = oracle.transmission(d, E, 1e-6)
        assert np.max(np.abs(T - ref)) <= 1e-4


def test_batch_argument_errors(lib):
    import torch
    assert lib.load().rgf_transmission_batch(None, -1, None, None, 1e-6, 0, None, None, None) == lib.RGF_EINVAL
    assert lib.load().rgf_transmission_batch(None, 0, None, None, 1e-6, 0, None, None, None) == lib.RGF_OK
    d = stage(synth.random_small_device(2, 5, seed=3))
    with pytest.raises(lib.RgfError):
        lib.transmission_batch([d], [torch.zeros(2, dtype=torch.float64, device="cuda")], -1.0)


def test_autotune_picks_a_measured_choice_and_keeps_results(lib):
    dev = synth.random_small_device(4, 100, seed=41, distinct_leads=True)
    dt = stage(dev)
    E = np.array([-1.3, -0.4, 0.6, 1.7])
    before, _ = _single(lib, dt, E, 1e-6)
    try:
        r = lib.autotune(100, "fp64", batch=16)
        log(f"[tune] M=100 fp64: tile {r['tile']} lanes {r['lanes']} ms {r['ms']}")
        assert r["tile"] in (64, 128) and r["lanes"] in (1, 2)
        assert len(r["ms"]) == 4 and all(v > 0 for v in r["ms"].values())
        assert r["ms"][(r["tile"], r["lanes"])] == min(r["ms"].values())
        assert lib.get_tuning(100, "fp64") == (r["tile"], r["lanes"])
        for tile in (64, 128):
            lib.set_tuning(100, "fp64", tile, 1)
            after, _ = _single(lib, dt, E, 1e-6)
            log(f"[tune] tile {tile}: max |dT| vs default {np.max(np.abs(after - before)):.2e}")
            assert np.allclose(after, before, rtol=1e-12, atol=1e-14)
    finally:
        lib.set_tuning(100, "fp64", 0, 0)
    assert lib.get_tuning(100, "fp64") == (128, 1)


@pytest.mark.parametrize("N,M,nE", [(6, 70, 5), (3, 300, 4)])
def test_graph_replays_equal_eager_results(lib, N, M, nE):
    """Captured sweeps: every replay equals the eager path bitwise, with eager work in between.

    M = 300 pads to 320 and splits over two lanes, so each lane captures its own graph.
    """
    import torch
    dev = synth.random_small_device(N, M, seed=60 + M, distinct_leads=True)
    dt = stage(dev)
    rng = np.random.default_rng(M)
    grids = [np.sort(rng.uniform(-2.0, 2.0, nE)) for _ in range(4)]
    eager = [_single(lib, dt, E, 1e-6)[0] for E in grids]
    try:
        lib.set_graphs(True)
        assert lib.get_graphs()
        for rep in range(2):
            for k, E in enumerate(grids):
                T, info = _single(lib, dt, E, 1e-6)
                log(f"[graph] N={N} M={M} rep {rep} grid {k}: bitwise={np.array_equal(T, eager[k])}")
                assert np.array_equal(T, eager[k]) and np.all(info == 0)
                lib.set_graphs(False)  # eager work between replays
                Te, _ = _single(lib, dt, grids[(k + 1) % 4], 1e-6)
                assert np.array_equal(Te, eager[(k + 1) % 4])
                torch.cuda.synchronize()
                lib.set_graphs(True)
        ref = oracle.transmission(dev, grids[0], 1e-6)
        assert fp64_close(eager[0], ref)[0]
    finally:
        lib.set_graphs(False)


def test_profile_samples_every_nth_launch(lib):
    """rgf_profile(n) times one block-product launch in n: the recorded count is the ceiling of
    the full count over n, and the results do not change while profiling."""
    dev = synth.random_small_device(7, 130, seed=41)
    E = np.linspace(-1.5, 1.5, 6)
    dt = stage(dev)
    T0, _ = _single(lib, dt, E, 1e-6)
    counts = {}
    for every in (1, 3, 4):
        lib.profile(True, every)
        lib.profile_read()
        T, _ = _single(lib, dt, E, 1e-6)
        n, ms, flops = lib.profile_read()
        lib.profile(False)
        counts[every] = n
        log(f"[profile] every {every}: {n} launches, {ms:.3f} ms, {flops:.3e} flops")
        assert np.array_equal(T, T0)
        assert n == 0 or (ms > 0 and flops > 0)
    assert counts[1] > 0
    for every in (3, 4):
        assert counts[every] == -(-counts[1] // every)


def test_decimation_flops_count_the_iterations_each_energy_ran(lib, monkeypatch):
    """With the class profile on, the decimation class counts only the iterations each energy ran
    (later launches skip a converged energy in-kernel).  Energies a few times beyond the lead's
    bands converge in about five iterations, band energies at eta = 1e-6 need about 26 (the
    oracle's counts on this lead); a count of whole launches would charge the former the latter's
    iterations whenever both share a call.  The executed work is per energy, so a call of both
    sets counts the sum of the two sets' calls."""
    from oracle import rgf_oracle
    monkeypatch.setenv("RGF_LANES", "1")
    dev = synth.random_small_device(3, 64, seed=43)  # S(k) positive definite at this size
    _, bands = rgf_oracle.lead_bands(dev.left, 64)
    emax = np.max(np.abs(bands))
    gap = np.array([3.0 * emax, 4.0 * emax])
    band = np.percentile(bands, [40.0, 60.0])
    dt = stage(dev)

    def lead_flops(E):
        lib.profile_classes(True, 1)
        lib.profile_read_classes()
        T, info = _single(lib, dt, E, 1e-6)
        c = lib.profile_read_classes()["lead"]
        lib.profile_classes(False)
        assert np.all(info == 0), (E, info)
        return c["flops"]

    f_gap, f_band = lead_flops(gap), lead_flops(band)
    f_both = lead_flops(np.concatenate([gap, band]))
    log(f"[profile] decimation flops: gap {f_gap:.4e}, band {f_band:.4e}, both {f_both:.4e}")
    assert 0 < f_gap < f_band
    assert abs(f_both - (f_gap + f_band)) <= 1e-9 * f_both
