"""Pins of the transverse k-point oracle (CPU).

X(k) = sum_R X(R) exp(2 pi i k . R) for every block; T(E) = sum_k w_k T_k(E).
Pinned by: a single image (T_k = T), an orthogonal device with on-site
transverse hopping (an exact energy shift of the zero-k transmission, with
different hoppings along the two transverse directions), time reversal for
real images, and band folding in a transverse supercell, built independently
in real space.
"""
import numpy as np
import pytest

import oracle
import oracle.kmesh as km
import synth

ETA = 1e-6


def orthogonal(dev):
    """The device with S = I on-site and no overlap between layers (leads too)."""
    N, M = dev.N, dev.M
    I, Z = np.eye(M, dtype=complex), np.zeros((M, M), complex)
    lead = lambda L: synth.Lead(L.H00, L.H01, I, Z)
    return synth.device_from_blocks([dev.Hd(i) for i in range(N)], [dev.Hu(i) for i in range(N - 1)],
                                    [I] * N, [Z] * (N - 1), lead(dev.left), lead(dev.right))


def onsite_image(dev, t):
    """An image whose only blocks are t * I on the device and electrode on-site H blocks."""
    N, M = dev.N, dev.M
    I, Z = np.eye(M, dtype=complex), np.zeros((M, M), complex)
    lead = synth.Lead(t * I, Z, Z, Z)
    return synth.device_from_blocks([t * I] * N, [Z] * (N - 1), [Z] * N, [Z] * (N - 1), lead, lead)


def test_single_image_gives_the_plain_transmission():
    dev = synth.random_small_device(4, 3, seed=5, distinct_leads=True)
    kk, w = km.monkhorst_pack(3, 2)
    E = np.array([-1.1, 0.2, 1.3])
    T, Tk = km.transmission_kmesh([dev], [[0, 0]], kk, w, E, ETA)
    ref = oracle.transmission(dev, E, ETA)
    assert np.allclose(Tk, ref[None, :], rtol=1e-13, atol=1e-15) and np.allclose(T, ref, rtol=1e-13, atol=1e-15)


def test_onsite_transverse_hopping_is_an_energy_shift():
    """Orthogonal device, hoppings t1, t2 along the two transverse directions:
    T_k(E) = T_0(E - 2 t1 cos(2 pi k1) - 2 t2 cos(2 pi k2))."""
    dev = orthogonal(synth.random_small_device(4, 3, seed=12, distinct_leads=True))
    t1, t2 = 0.13, -0.21
    images = [dev, onsite_image(dev, t1), onsite_image(dev, t1), onsite_image(dev, t2), onsite_image(dev, t2)]
    R = [[0, 0], [1, 0], [-1, 0], [0, 1], [0, -1]]
    kk = np.array([[0.1, 0.35], [-0.3, 0.05], [0.45, -0.2]])
    E = np.array([-0.9, 0.4, 1.2])
    _, Tk = km.transmission_kmesh(images, R, kk, np.full(3, 1 / 3), E, ETA)
    for (k1, k2), row in zip(kk, Tk):
        shift = 2 * t1 * np.cos(2 * np.pi * k1) + 2 * t2 * np.cos(2 * np.pi * k2)
        ref = oracle.transmission(dev, E - shift, ETA)
        assert np.max(np.abs(row - ref)) <= 1e-10 * max(1.0, np.abs(ref).max())


def _real_images(seed):
    """R = 0 real device plus a real image pair X(-R) = X(R)^T along direction 1."""
    d0 = synth.random_small_device(3, 2, seed=seed, real=True, distinct_leads=True)
    rng = np.random.default_rng(seed)
    N, M = d0.N, d0.M
    r = lambda *s: 0.2 * rng.standard_normal(s).astype(complex)
    hd, hu, sd = r(N, M, M), r(N - 1, M, M), 0.02 * r(N, M, M)
    lh00, lh01 = r(M, M), r(M, M)
    plus = synth.device_from_blocks(list(hd), list(hu), list(sd), [np.zeros((M, M), complex)] * (N - 1),
                                    synth.Lead(lh00, lh01, np.zeros((M, M), complex), np.zeros((M, M), complex)),
                                    synth.Lead(lh00, lh01, np.zeros((M, M), complex), np.zeros((M, M), complex)))
    T = lambda x: np.swapaxes(x, -1, -2)
    minus = synth.device_from_blocks(list(T(hd)), list(T(hu)), list(T(sd)),
                                     [np.zeros((M, M), complex)] * (N - 1),
                                     synth.Lead(lh00.T, lh01.T, np.zeros((M, M), complex), np.zeros((M, M), complex)),
                                     synth.Lead(lh00.T, lh01.T, np.zeros((M, M), complex), np.zeros((M, M), complex)))
    return [d0, plus, minus], [[0, 0], [1, 0], [-1, 0]]


def test_time_reversal_for_real_images():
    """On-site images with X(-R) = X(R)^T (Hermitian X(k)) and real blocks: T_k = T_-k."""
    images, R = _real_images(33)
    # keep only on-site-type images Hermitian: the coupling images pair up as X(-R) = X(R)^T as well
    kk = np.array([[0.21, 0.0], [-0.21, 0.0], [0.37, 0.1], [-0.37, -0.1]])
    E = np.array([-2.0, -1.5, -1.0, 2.5])
    # T_k(LR) = T_-k(RL) exactly; T_LR = T_RL up to the eta absorption, so a small eta
    _, Tk = km.transmission_kmesh(images, R, kk, np.full(4, 0.25), E, 1e-9)
    assert Tk.max() > 0.1
    assert np.max(np.abs(Tk[0] - Tk[1])) <= 1e-6 * max(1, np.abs(Tk[0]).max())
    assert np.max(np.abs(Tk[2] - Tk[3])) <= 1e-6 * max(1, np.abs(Tk[2]).max())
    # a complex image breaks it (the pin is not vacuous)
    images[1] = synth.device_from_blocks([images[1].Hd(i) * (1 + 0.5j) for i in range(images[1].N)],
                                         [images[1].Hu(i) for i in range(images[1].N - 1)],
                                         [images[1].Sd(i) for i in range(images[1].N)],
                                         [images[1].Su(i) for i in range(images[1].N - 1)],
                                         images[1].left, images[1].right)
    images[2] = synth.device_from_blocks([images[2].Hd(i) * (1 - 0.5j) for i in range(images[2].N)],
                                         [images[2].Hu(i) for i in range(images[2].N - 1)],
                                         [images[2].Sd(i) for i in range(images[2].N)],
                                         [images[2].Su(i) for i in range(images[2].N - 1)],
                                         images[2].left, images[2].right)
    _, Tk = km.transmission_kmesh(images, R, kk, np.full(4, 0.25), E, 1e-9)
    assert np.max(np.abs(Tk[2] - Tk[3])) > 1e-4


def _supercell(images, R):
    """Images of the transverse supercell doubled along direction 1 (sub-cells a, b in {0, 1}):
    X_sc(R1', R2)[a, b] = X(2 R1' + b - a, R2)."""
    N, M = images[0].N, images[0].M
    lut = {tuple(r): im for r, im in zip(R, images)}
    Z = np.zeros((M, M), complex)

    def get(im, kind, i):
        if im is None:
            return Z
        if kind in ("H00", "H01", "S00", "S01_"):
            raise ValueError
        return getattr(im, kind)(i)

    out_images, out_R = [], []
    R2s = sorted(set(r[1] for r in R))
    for R1p in (-1, 0, 1):
        for R2 in R2s:
            def blk(fn):
                B = np.zeros((2 * M, 2 * M), complex)
                for a in range(2):
                    for b in range(2):
                        im = lut.get((2 * R1p + b - a, R2))
                        if im is not None:
                            B[a * M:(a + 1) * M, b * M:(b + 1) * M] = fn(im)
                return B
            if not any((2 * R1p + b - a, R2) in lut for a in range(2) for b in range(2)):
                continue
            hd = [blk(lambda im, i=i: im.Hd(i)) for i in range(N)]
            sd = [blk(lambda im, i=i: im.Sd(i)) for i in range(N)]
            hu = [blk(lambda im, i=i: im.Hu(i)) for i in range(N - 1)]
            su = [blk(lambda im, i=i: im.Su(i)) for i in range(N - 1)]
            lead = lambda side: synth.Lead(*(blk(lambda im, n=n: getattr(getattr(im, side), n))
                                              for n in ("H00", "H01", "S00", "S01")))
            out_images.append(synth.device_from_blocks(hd, hu, sd, su, lead("left"), lead("right")))
            out_R.append([R1p, R2])
    return out_images, out_R


def test_band_folding_in_a_transverse_supercell():
    """T_sc(k1', k2) = T(k1'/2, k2) + T(k1'/2 + 1/2, k2) for a supercell doubled along direction 1."""
    d0 = synth.random_small_device(3, 2, seed=91, distinct_leads=True)
    rng = np.random.default_rng(91)
    N, M = d0.N, d0.M
    c = lambda *s: 0.15 * (rng.standard_normal(s) + 1j * rng.standard_normal(s))
    hd, hu, sd, su = c(N, M, M), c(N - 1, M, M), 0.1 * c(N, M, M), 0.1 * c(N - 1, M, M)
    l = [c(M, M) for _ in range(4)]
    l[2] *= 0.1
    l[3] *= 0.1
    dag = lambda x: np.conj(np.swapaxes(x, -1, -2))
    plus = synth.device_from_blocks(list(hd), list(hu), list(sd), list(su), synth.Lead(*l), synth.Lead(*l))
    # X(-R) = X(R)^+ for the on-site blocks keeps X(k) Hermitian; for the couplings the image of -R is the
    # coupling from cell R back to 0, whose adjoint pairing is handled by H_{i+1,i}(k) = H_{i,i+1}(k)^+
    minus = synth.device_from_blocks(list(dag(hd)), list(c(N - 1, M, M)), list(dag(sd)), list(0.1 * c(N - 1, M, M)),
                                     synth.Lead(dag(l[0]), c(M, M), dag(l[2]), 0.1 * c(M, M)),
                                     synth.Lead(dag(l[0]), c(M, M), dag(l[2]), 0.1 * c(M, M)))
    images, R = [d0, plus, minus], [[0, 0], [1, 0], [-1, 0]]
    sc_images, sc_R = _supercell(images, R)
    E = np.array([-0.6, 0.3, 1.1])
    for k1p, k2 in ((0.2, 0.0), (-0.34, 0.0)):
        _, Tsc = km.transmission_kmesh(sc_images, sc_R, [[k1p, k2]], [1.0], E, ETA)
        _, Tk = km.transmission_kmesh(images, R, [[k1p / 2, k2], [k1p / 2 + 0.5, k2]], [0.5, 0.5], E, ETA)
        assert np.max(np.abs(Tsc[0] - Tk.sum(axis=0))) <= 1e-9 * max(1.0, np.abs(Tsc).max())


def test_monkhorst_pack_mesh():
    kk, w = km.monkhorst_pack(7, 7)
    assert kk.shape == (49, 2) and abs(w.sum() - 1) < 1e-15
    assert np.allclose(np.sort(kk[:, 0]), np.sort(-kk[:, 0]))  # symmetric about 0


# ---- planted mistakes: each must break a pin ----

def _pins_hold():
    try:
        test_single_image_gives_the_plain_transmission()
        test_onsite_transverse_hopping_is_an_energy_shift()
        test_band_folding_in_a_transverse_supercell()
    except AssertionError:
        return False
    return True


def test_pins_hold_for_the_oracle():
    assert _pins_hold()


@pytest.mark.parametrize("bad", [
    lambda blocks, R, k: np.tensordot(np.exp(1j * (np.asarray(R, float) @ np.asarray(k, float))),
                                      np.asarray(blocks), axes=(0, 0)),                    # no 2 pi
    lambda blocks, R, k: np.tensordot(np.exp(2j * np.pi * (np.asarray(R, float)[:, ::-1] @ np.asarray(k, float))),
                                      np.asarray(blocks), axes=(0, 0)),                    # components swapped
    lambda blocks, R, k: np.tensordot(np.cos(2 * np.pi * (np.asarray(R, float) @ np.asarray(k, float))),
                                      np.asarray(blocks), axes=(0, 0)),                    # phase dropped
])
def test_planted_bloch_sum_mistakes_are_caught(monkeypatch, bad):
    monkeypatch.setattr(km, "bloch_sum", bad)
    assert not _pins_hold()
