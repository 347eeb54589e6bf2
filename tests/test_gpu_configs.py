"""GPU parity at the full workload sizes, against stored oracle values.

The expected values in tests/golden/<cfg>.json were written by
tests/golden/make_golden.py, which calls only the FP64 oracle.  The GPU runs
each workload in the configuration the benchmark times (whole energy batches,
full layer count and block size) and the sampled energies are compared
element by element: C2 all 1000 energies, C3 128 and C4 16 (each with the 8
grid energies nearest the lead's band extrema); C4 runs in the benchmark's step
(256 energies on one lane).

FP64 bar: |T_gpu - T_oracle| <= 1e-8 |T_oracle| + 1e-12.  Where the golden also
holds other oracle values of the same T (C4, at every sample: from the
Bloch-mode lead construction, from the same construction under other BLAS
threading, and from the device and electrodes with every block times 3, which
leaves T unchanged in exact arithmetic but changes every rounding), twice the
largest spread |T_oracle - T_other| is added: where the lead's bands have
sharp features, T is reproducible in FP64 only to that spread (at the C4
grid point E = 1.6712 the decimation and Bloch-mode constructions of Sigma
differ by 2.7e-8 and 7.6e-8 relative), and a correct GPU result can lie that
far from any one oracle value; elsewhere the spread is far below the bar.
At that grid point the oracle's constructions agree within 2.5e-9; the FP64
path's decimation substitutes with the diagonal blocks of U there (explicit
inverses of those blocks had put T 2.0e-8 off).
Mixed bar: |T_gpu - T_oracle| <= 1e-4.  The FP32 matrix-core form does not
reach it on these workloads (FP32 accumulation leaves ~1e-6 relative error
per product and the near-singular layer blocks at eta = 1e-6 amplify it), so
those tests are strict expected failures that log the measured |dT|.

The forms beyond T(E) are checked at the block sizes the benchmark times,
reduced only in the layer count: finite bias at M = 1024, the 7 x 7
transverse k-mesh at M = 256 and the KPM moments at M = 1024.
"""
import json
import os

import numpy as np
import pytest

import synth
from gpu_helpers import FP64_ATOL, FP64_RTOL, MIXED_ATOL, fp64_close, gpu_transmission, log, stage

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
MIXED_UNMET = ("the FP32 matrix-core form gives |dT| of order 1e-3 on this workload (eta = 1e-6); the 1e-4 "
               "bar is not met")


def golden(name):
    path = os.path.join(GOLDEN, f"{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as f:
        return json.load(f)


def _compare(tag, T, g, precision):
    ref = np.array(g["T"])
    err = np.abs(T - ref)
    # the oracle's own FP64 spread at each sample: T from Bloch-mode leads, from the same
    # construction under other BLAS threading, and from the device with every block scaled
    spread = np.abs(ref - np.array(g["T_bloch"])) if "T_bloch" in g else np.zeros_like(ref)
    pos = {i: k for k, i in enumerate(g["indices"])}
    for kind in ("rethread", "scaled"):
        for i, t in zip(g.get(f"{kind}_indices", []), g.get(f"T_{kind}", [])):
            spread[pos[i]] = max(spread[pos[i]], abs(ref[pos[i]] - t))
    E = np.array(g["E"])
    if precision == "fp64":
        ok = err <= FP64_RTOL * np.abs(ref) + FP64_ATOL + 2.0 * spread
    else:
        ok = err <= MIXED_ATOL
    log(f"[config] {tag} {precision}: max |dT| {err.max():.3e}, p99 {np.percentile(err, 99):.3e}, "
        f"mean |dT| {err.mean():.3e}, max rel {np.max(err / np.abs(ref)):.3e}, "
        f"T range [{ref.min():.3g}, {ref.max():.3g}], {len(ref)} energies; "
        f"oracle construction spread max rel {np.max(spread / np.abs(ref)):.2e}")
    assert np.all(ok), [(e, d, r) for e, d, r, o in zip(E, err, ref, ok) if not o][:10]


@pytest.fixture(scope="module")
def c2_dev():
    cfg = synth.config_c2()
    return cfg, stage(cfg.device)


def _precision_param():
    return pytest.mark.parametrize("precision", [
        "fp64", pytest.param("mixed", marks=pytest.mark.xfail(strict=True, reason=MIXED_UNMET))])


@_precision_param()
def test_c2_all_energies(lib, c2_dev, precision):
    """60 layers, M = 256: all 1000 energies in one call, every one compared."""
    cfg, dt = c2_dev
    g = golden("c2")
    log(f"[config] c2 {precision}: N={cfg.device.N} M={cfg.device.M} nE={len(cfg.energies)}")
    T, info = gpu_transmission(dt, cfg.energies, cfg.eta, precision)
    assert np.all(info == 0)
    _compare("c2", T[g["indices"]], g, precision)


@_precision_param()
def test_c3_sampled(lib, precision):
    """200 layers, M = 512, 5% doped layers: the 128 sampled energies in two 64-energy batches."""
    cfg = synth.config_c3()
    g = golden("c3")
    dt = stage(cfg.device)
    E = np.array(g["E"])
    log(f"[config] c3 {precision}: N={cfg.device.N} M={cfg.device.M} energies={len(E)}")
    T = np.concatenate([gpu_transmission(dt, E[i:i + 64], cfg.eta, precision)[0] for i in range(0, len(E), 64)])
    _compare("c3", T, g, precision)


@pytest.fixture(scope="module")
def c4_dev():
    cfg = synth.config_c4()
    dt = stage(cfg.device)
    yield cfg, dt
    del dt
    import torch
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def c4_runs():
    return {}


def _c4_result(lib, c4_dev, c4_runs, precision):
    """T at the 16 sampled energies inside one 256-energy call on one energy lane, the benchmark's
    step (run once per precision and shared by the tests below)."""
    from paper_2609_37058_amd import rgf
    if precision not in c4_runs:
        cfg, dt = c4_dev
        idx = np.array(golden("c4")["indices"])
        batch = np.concatenate([cfg.energies[idx], cfg.energies[100:100 + 256 - len(idx)]])
        log(f"[config] c4 {precision}: N={cfg.device.N} M={cfg.device.M} batch={len(batch)}, one lane")
        rgf.set_tuning(cfg.device.M, precision, 0, 1)
        try:
            T, info = gpu_transmission(dt, batch, cfg.eta, precision)
        finally:
            rgf.set_tuning(cfg.device.M, precision, 0, 0)
        c4_runs[precision] = (T[:len(idx)], info)
    return c4_runs[precision]


@_precision_param()
def test_c4_sampled(lib, c4_dev, c4_runs, precision):
    """400 layers, M = 1024 (25 GiB of blocks): the 16 sampled energies inside a 256-energy call
    on one energy lane, the benchmark's step."""
    g = golden("c4")
    T, info = _c4_result(lib, c4_dev, c4_runs, precision)
    assert np.all(info == 0)
    _compare("c4", T, g, precision)


def test_batch_invariance_and_determinism(lib, c2_dev):
    """A result does not depend on the batch it runs in, and reruns are bitwise equal."""
    cfg, dt = c2_dev
    E = cfg.energies[::37]
    T_all, _ = gpu_transmission(dt, E, cfg.eta)
    T_again, _ = gpu_transmission(dt, E, cfg.eta)
    T_alone = np.array([gpu_transmission(dt, E[k:k + 1], cfg.eta)[0][0] for k in (0, 7, len(E) - 1)])
    T_rev, _ = gpu_transmission(dt, np.ascontiguousarray(E[::-1]), cfg.eta)
    assert np.array_equal(T_all, T_again)
    assert np.array_equal(T_all[[0, 7, len(E) - 1]], T_alone)
    assert np.array_equal(T_all, T_rev[::-1])


def test_c1_pristine_integer_channels_on_gpu(lib):
    """The GPU's T for the pristine C1 device equals the leads' channel count away from band edges."""
    import oracle
    cfg = synth.config_c1()
    T, info = gpu_transmission(stage(cfg.device), cfg.energies, cfg.eta)
    nch = oracle.channel_count(cfg.device.left, cfg.energies)
    ext = oracle.band_extrema(cfg.device.left)
    keep = np.array([np.min(np.abs(ext - e)) > 1e-2 for e in cfg.energies])
    assert np.max(np.abs(T - nch)[keep]) <= 1e-3


# ---------------------------------------------------------------- the NEXT rows at bench shapes

def _golden_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(GOLDEN, "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bias_at_block_1024(lib):
    """Finite bias (electrodes shifted by +-0.1 eV) on the C4 device's first 3 layers, M = 1024."""
    import torch
    g = golden("bias_m1024")
    cfg, dev = _golden_module().bias_device()
    E = torch.as_tensor(np.array(g["E"])).cuda()
    log(f"[config] bias M={dev.M} N={dev.N} energies={len(g['E'])}")
    T, info = lib.transmission_bias(stage(dev), E, cfg.eta, g["V"] / 2, -g["V"] / 2)
    torch.cuda.synchronize()
    ok, rel, ab = fp64_close(T.cpu().numpy(), np.array(g["T"]))
    log(f"[config]   max |dT| {ab:.2e} (rel {rel:.2e})")
    assert ok and int(info.abs().sum()) == 0


def test_kmesh_at_block_256_on_7x7(lib):
    """The k-mesh workload's recipe at M = 256 on the full 7 x 7 mesh (N = 4): every T_k and the
    weighted average."""
    import torch
    g = golden("kmesh_m256")
    cfg, images, R, kk, w, E = _golden_module().kmesh_device()
    imgs = [stage(im) for im in images]
    log(f"[config] kmesh M={g['M']} N={g['N']} {len(kk)} k-points, {len(E)} energies")
    T, Tk, info = lib.transmission_kmesh(imgs, R, kk, w, torch.as_tensor(E).cuda(), cfg.eta)
    torch.cuda.synchronize()
    okk, relk, abk = fp64_close(Tk.cpu().numpy(), np.array(g["Tk"]))
    ok, rel, ab = fp64_close(T.cpu().numpy(), np.array(g["T"]))
    log(f"[config]   max |dT_k| {abk:.2e}, max |dT| {ab:.2e}")
    assert okk and ok and int(info.abs().sum()) == 0


def test_kpm_at_block_1024(lib):
    """KPM moments of the C4 central region's first 4 layers (M = 1024, N M = 4096) from 4
    random-phase vectors, against the dense-solve oracle: |dmu| <= 1e-10 N M."""
    import torch
    g = golden("kpm_m1024")
    dev, lo, hi, r = _golden_module().kpm_device()
    log(f"[config] kpm M={dev.M} N={dev.N} R={g['R']} n_mom={g['n_mom']}")
    mu = lib.kpm_moments(stage(dev), lo, hi, g["n_mom"], torch.as_tensor(r).cuda())
    torch.cuda.synchronize()
    err = np.abs(mu.cpu().numpy() - np.array(g["mu"]))
    log(f"[config]   max |dmu| {err.max():.2e} (bar {1e-10 * dev.N * dev.M:.1e})")
    assert np.all(err <= 1e-10 * dev.N * dev.M)
