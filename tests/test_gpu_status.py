"""Per-energy status bits on the GPU: the small-block kernel, the fused factor-and-solve and the
batched LU.

Each case ends normally with the bits set (no kernel faults): decimation
capped far below convergence (RGF_INFO_SR_LEFT/RIGHT, and the capped T
still equals the oracle's with the same cap), an exactly zero pivot from an
emptied layer (RGF_INFO_SINGULAR with the layer index in bits 8.., T = NaN)
and a NaN entry (RGF_INFO_NONFINITE, T = NaN).  The oracle's behaviour in
the same cases is pinned in test_oracle_status.py.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import fp64_close, force_batched_path, gpu_transmission, log, stage
from test_oracle_status import _cut_layer

pytestmark = pytest.mark.gpu

ETA = 1e-6
SR_LEFT, SR_RIGHT, SINGULAR, NONFINITE = 1, 2, 4, 8


class capped_decimation:
    def __init__(self, lib, k):
        self.lib, self.k = lib, k

    def __enter__(self):
        self.lib.set_sr_maxit(self.k)

    def __exit__(self, *a):
        self.lib.set_sr_maxit(0)


# (M, batched): M <= 16 takes the small-block kernel unless forced onto the batched path; on the
# batched path padded blocks up to 192 take the fused factor-and-solve (M = 4, 40) and larger ones
# the blocked LU with its panel kernel (M = 200, padded to 256)
PATHS = [(4, False), (4, True), (40, True), (200, True)]


@pytest.mark.parametrize("M,batched", PATHS)
@pytest.mark.parametrize("distinct", [False, True])
def test_capped_decimation_sets_bits_and_matches_capped_oracle(lib, M, batched, distinct):
    """Decimation stopped after 3 steps describes leads of 2^3 layers.  At eta = 1e-6 such a lead
    absorbs only through eta: T drops to 1e-8..1e-4 and its relative conditioning to ~1e-7 (at
    M = 200 the two FP64 paths differ by 1e-7 relative), so the comparison runs at eta = 0.05,
    where the truncated leads still absorb and the fixed FP64 bar applies."""
    eta = 0.05
    dev = synth.random_small_device(3, M, seed=70 + M, distinct_leads=distinct)
    E = np.array([-0.9, 0.25, 1.1])
    log(f"[status] sr cap 3: M={M} batched={batched} distinct={distinct} eta={eta}")
    with capped_decimation(lib, 3):
        if batched:
            with force_batched_path():
                T, info = gpu_transmission(stage(dev), E, eta)
        else:
            T, info = gpu_transmission(stage(dev), E, eta)
    ref = oracle.transmission(dev, E, eta, sr_maxit=3)
    ok, rel, ab = fp64_close(T, ref)
    log(f"[status]   info {info.tolist()}, max |dT| {ab:.2e} vs the oracle capped at 3 steps")
    assert np.all(info == SR_LEFT | SR_RIGHT)
    assert ok
    # the default cap converges: no bits
    T2, info2 = gpu_transmission(stage(dev), E, eta)
    assert np.all(info2 == 0)


@pytest.mark.parametrize("M,batched", PATHS)
@pytest.mark.parametrize("k", [1, 2])
def test_empty_layer_reports_singular_with_layer(lib, M, batched, k):
    dev = _cut_layer(synth.random_small_device(4, M, seed=80 + M), k)
    E = np.array([-0.4, 0.3])
    log(f"[status] empty layer {k}: M={M} batched={batched}")
    if batched:
        with force_batched_path():
            T, info = gpu_transmission(stage(dev), E, ETA)
    else:
        T, info = gpu_transmission(stage(dev), E, ETA)
    log(f"[status]   info {[hex(int(i)) for i in info]}")
    assert np.all(info == SINGULAR | (k << 8))
    assert np.all(np.isnan(T))


@pytest.mark.parametrize("M,batched", PATHS)
def test_nan_entry_reports_nonfinite(lib, M, batched):
    dev = synth.random_small_device(3, M, seed=90 + M)
    hd, hu, sd, su = dev.stacked()
    hd[1][2, 1] = np.nan
    bad = synth.device_from_blocks(hd, hu, sd, su, dev.left, dev.right)
    E = np.array([0.1, 0.9])
    log(f"[status] NaN entry: M={M} batched={batched}")
    if batched:
        with force_batched_path():
            T, info = gpu_transmission(stage(bad), E, ETA)
    else:
        T, info = gpu_transmission(stage(bad), E, ETA)
    log(f"[status]   info {info.tolist()}")
    assert np.all(info == NONFINITE)
    assert np.all(np.isnan(T))
