"""Transverse k-point sampling on the GPU against the FP64 oracle.

Blocks are given for transverse lattice images; the library forms X(k) with
a Bloch-sum kernel, runs the k-resolved transmissions of all k-points as one
grouped batch (the fused small-block kernel's multi-device batch for tiny
blocks) and averages them with the mesh weights.  FP64 bar element by
element on every T_k and on the average.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import fp64_close, log, stage

pytestmark = pytest.mark.gpu


def _images(N, M, seed, distinct=False):
    """R = 0 plus a +-R pair along direction 1 with X(-R) = X(R)^+ on-site, free couplings."""
    d0 = synth.random_small_device(N, M, seed=seed, distinct_leads=distinct)
    rng = np.random.default_rng(seed)
    c = lambda *s: 0.15 * (rng.standard_normal(s) + 1j * rng.standard_normal(s))
    dag = lambda x: np.conj(np.swapaxes(x, -1, -2))
    hd, sd = c(N, M, M), 0.1 * c(N, M, M)
    hu_p, hu_m = c(max(N - 1, 1), M, M)[:N - 1], c(max(N - 1, 1), M, M)[:N - 1]
    su_p, su_m = 0.1 * c(max(N - 1, 1), M, M)[:N - 1], 0.1 * c(max(N - 1, 1), M, M)[:N - 1]
    lp = [c(M, M), c(M, M), 0.1 * c(M, M), 0.1 * c(M, M)]
    lm = [dag(lp[0]), c(M, M), dag(lp[2]), 0.1 * c(M, M)]
    lead_p, lead_m = synth.Lead(*lp), synth.Lead(*lm)
    plus = synth.device_from_blocks(list(hd), list(hu_p), list(sd), list(su_p), lead_p, lead_p)
    minus = synth.device_from_blocks(list(dag(hd)), list(hu_m), list(dag(sd)), list(su_m), lead_m, lead_m)
    # with distinct=True only the R = 0 image has two different electrodes, which is
    # enough to make every k-point's left and right electrode differ
    return [d0, plus, minus], [[0, 0], [1, 0], [-1, 0]]


def _stage_images(images):
    return [stage(im) for im in images]


@pytest.mark.parametrize("N,M,distinct", [(4, 3, False), (3, 16, False), (3, 40, False), (2, 70, False),
                                          (3, 16, True), (3, 40, True)])
def test_kmesh_matches_oracle(lib, N, M, distinct):
    import torch
    images, R = _images(N, M, seed=500 + M, distinct=distinct)
    kk, w = oracle.monkhorst_pack(3, 2)
    E = np.array([-1.2, -0.3, 0.5, 1.4])
    T, Tk, info = lib.transmission_kmesh(_stage_images(images), R, kk, w, torch.as_tensor(E).cuda(), 1e-6)
    torch.cuda.synchronize()
    T_ref, Tk_ref = oracle.transmission_kmesh(images, R, kk, w, E, 1e-6)
    ok_k, rel_k, _ = fp64_close(Tk.cpu().numpy().ravel(), Tk_ref.ravel())
    ok, rel, _ = fp64_close(T.cpu().numpy(), T_ref)
    log(f"[kmesh] N={N} M={M} distinct={distinct} nk={len(kk)}: T_k max rel {rel_k:.2e}, T max rel {rel:.2e}")
    assert ok_k and ok and np.all(info.cpu().numpy() == 0)


def test_kmesh_chunks_across_k_points_are_bitwise_equal(lib, monkeypatch):
    """Energy chunks and lanes that start inside a k-point's energies give the same bits."""
    import torch
    images, R = _images(3, 40, seed=611)
    kk, w = oracle.monkhorst_pack(3, 3)
    E = torch.as_tensor(np.linspace(-1.0, 1.0, 5)).cuda()
    staged = _stage_images(images)
    T0, Tk0, i0 = lib.transmission_kmesh(staged, R, kk, w, E, 1e-6)
    torch.cuda.synchronize()
    for chunk, lanes in (("3", "1"), ("7", "2"), ("2", "3")):
        monkeypatch.setenv("RGF_MAX_CHUNK", chunk)
        monkeypatch.setenv("RGF_LANES", lanes)
        T1, Tk1, i1 = lib.transmission_kmesh(staged, R, kk, w, E, 1e-6)
        torch.cuda.synchronize()
        log(f"[kmesh] chunk {chunk} lanes {lanes}: equal {torch.equal(Tk0, Tk1)}")
        assert torch.equal(Tk0, Tk1) and torch.equal(T0, T1) and torch.equal(i0, i1)


def test_single_image_equals_plain_transmission(lib):
    import torch
    dev = synth.random_small_device(5, 24, seed=9, distinct_leads=True)
    dt = stage(dev)
    E = torch.as_tensor(np.array([-0.9, 0.2, 1.1])).cuda()
    T, Tk, _ = lib.transmission_kmesh([dt], [[0, 0]], [[0.1, -0.2], [0.3, 0.4]], [0.25, 0.75], E, 1e-6)
    T0, _ = lib.transmission(dt, E, 1e-6)
    torch.cuda.synchronize()
    assert torch.equal(Tk[0], T0) and torch.equal(Tk[1], T0)
    assert torch.allclose(T, T0, rtol=1e-15, atol=0)


def test_kmesh_argument_errors(lib):
    import torch
    dt = stage(synth.random_small_device(2, 4, seed=2))
    E = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.RgfError):
        lib.transmission_kmesh([dt] * 33, [[0, 0]] * 33, [[0, 0]], [1.0], E, 1e-6)
    with pytest.raises(lib.RgfError):
        lib.transmission_kmesh([dt, stage(synth.random_small_device(3, 4, seed=2))], [[0, 0], [1, 0]],
                               [[0, 0]], [1.0], E, 1e-6)
