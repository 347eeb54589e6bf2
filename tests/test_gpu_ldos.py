"""Orbital-resolved LDOS on the GPU against the FP64 oracle, through the C-ABI.

The library runs, per direction, a pass that keeps the end-connected
inverse of every layer and a pass that walks the layers forming G's blocks
next to the diagonal and the contact's block column; the oracle inverts the
whole device (small cases) or solves for block columns (sampled layers of a
C2-sized device).  FP64 bar element by element: |x - ref| <= 1e-8 |ref| plus
an absolute floor of 1e-10 times the largest |ref| of that energy (a value
is a sum of about 3M products of the energy's G and S entries, so its
rounding error scales with the largest of them, not with the value itself).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import log, stage

pytestmark = pytest.mark.gpu

ETA = 1e-6


def ldos_close(x, ref):
    scale = np.abs(ref).reshape(ref.shape[0], -1).max(axis=1).reshape(-1, *([1] * (ref.ndim - 1)))
    err = np.abs(x - ref)
    bound = 1e-8 * np.abs(ref) + 1e-10 * scale
    return bool(np.all(err <= bound)), float(np.max(err / (np.abs(ref) + 1e-300))), float(np.max(err / scale))


def run(lib, dev_t, E, parts=("dos", "left", "right")):
    import torch
    out = lib.ldos(dev_t, torch.as_tensor(np.asarray(E, np.float64)).cuda(), ETA, parts)
    torch.cuda.synchronize()
    return [None if t is None else t.cpu().numpy() for t in out]


@pytest.mark.parametrize("N,M,distinct", [(1, 5, True), (3, 16, False), (4, 40, True), (3, 70, True),
                                          (2, 130, False), (5, 24, True)])
def test_ldos_matches_oracle(lib, N, M, distinct):
    dev = synth.random_small_device(N, M, seed=700 + M, distinct_leads=distinct)
    E = np.array([-1.3, -0.2, 0.6, 1.5])
    dos, adl, adr, info = run(lib, stage(dev), E)
    ref = oracle.local_dos(dev, E, ETA, method="dense")
    ok = []
    for name, x, r in zip(("dos", "left", "right"), (dos, adl, adr), ref):
        good, rel, absn = ldos_close(x, r)
        log(f"[ldos] N={N} M={M} distinct={distinct} {name}: max rel {rel:.2e}, max err/scale {absn:.2e}")
        ok.append(good)
    assert all(ok) and np.all(info == 0)


def test_ldos_perfect_chain_closed_form(lib):
    E = np.array([-1.7, -0.4, 0.3, 1.2])
    dos, adl, adr, info = run(lib, stage(synth.chain_device(6)), E)
    expect = 1.0 / (np.pi * np.sqrt(4.0 - E ** 2))
    log(f"[ldos] chain: max rel {np.max(np.abs(dos[..., 0] / expect[:, None] - 1)):.2e}")
    assert np.allclose(dos[..., 0], expect[:, None], rtol=1e-5)
    assert np.allclose(adl[..., 0], expect[:, None] / 2, rtol=1e-4)
    assert np.allclose(adr[..., 0], expect[:, None] / 2, rtol=1e-4)


def test_ldos_sampled_layers_of_a_c2_sized_device(lib):
    """C2's device (60 layers, M = 256): sampled layers against the oracle's block-column solve."""
    cfg = synth.config_c2()
    dev = cfg.device
    E = np.array([0.4])
    layers = [0, 30, 59]
    dos, adl, adr, info = run(lib, stage(dev), E)
    ref = oracle.local_dos(dev, E, ETA, method="layers", layers=layers)
    ok = []
    for name, x, r in zip(("dos", "left", "right"), (dos, adl, adr), ref):
        good, rel, absn = ldos_close(x[:, layers], r)
        log(f"[ldos] c2 layers {layers} {name}: max rel {rel:.2e}, max err/scale {absn:.2e}")
        ok.append(good)
    assert all(ok) and np.all(info == 0)


def test_ldos_parts_chunks_and_lanes_are_bitwise_equal(lib, monkeypatch):
    dev_t = stage(synth.random_small_device(4, 40, seed=81, distinct_leads=True))
    E = np.linspace(-1.0, 1.0, 7)
    full = run(lib, dev_t, E)
    for parts in (("dos",), ("left",), ("right",), ("dos", "right")):
        sub = run(lib, dev_t, E, parts)
        for name, a, b in zip(("dos", "left", "right"), full[:3], sub[:3]):
            if name in parts:
                assert np.array_equal(a, b), (parts, name)
    for chunk, lanes in (("3", "1"), ("2", "2"), ("7", "3")):
        monkeypatch.setenv("RGF_MAX_CHUNK", chunk)
        monkeypatch.setenv("RGF_LANES", lanes)
        chunked = run(lib, dev_t, E)
        for a, b in zip(full, chunked):
            assert np.array_equal(a, b), (chunk, lanes)


def test_ldos_argument_errors(lib):
    import torch
    dt = stage(synth.random_small_device(2, 4, seed=2))
    E = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        lib.ldos(dt, E, ETA, ())
    with pytest.raises(lib.RgfError):
        lib.ldos(dt, E, -1.0)
