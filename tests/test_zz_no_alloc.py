"""rgf_transmission_noalloc through the C ABI against rgf_transmission.

The allocation-free entry point runs the same kernels in the library's
static device scratch array, so its results must equal those of the
allocating entry point: the FP64 bar, and bitwise since no per-energy step
depends on how energies are chunked.  Two calls in a row, the second on a
smaller input (the array keeps the first call's contents), plus a small-block
device that needs no scratch at all.
"""
import ctypes as C

import numpy as np
import pytest

import synth
from gpu_helpers import fp64_close, log, stage

pytestmark = pytest.mark.gpu

ETA = 1e-6


def _noalloc(lib, dev_t, E):
    """T, info from rgf_transmission_noalloc, called directly through the C ABI."""
    import torch
    T = torch.full((E.numel(),), -1.0, dtype=torch.float64, device="cuda")
    info = torch.full((E.numel(),), -7, dtype=torch.int32, device="cuda")
    d = dev_t.cstruct()
    rc = lib.load().rgf_transmission_noalloc(C.byref(d), E.data_ptr(), E.numel(), ETA, lib.RGF_FP64,
                                             T.data_ptr(), info.data_ptr(),
                                             torch.cuda.current_stream().cuda_stream)
    assert rc == lib.RGF_OK, lib.load().rgf_last_error()
    torch.cuda.synchronize()
    return T.cpu().numpy(), info.cpu().numpy()


@pytest.mark.parametrize("case", [(5, 200, 20, 31), (3, 70, 5, 32), (4, 6, 9, 33)])
def test_noalloc_equals_transmission(lib, case):
    """(N, M, energies, seed) in this order: 20 energies at M = 200 run in three chunks of the
    scratch array, then a smaller device, then a small-block one."""
    import torch
    N, M, nE, seed = case
    dev = synth.random_small_device(N, M, seed=seed, distinct_leads=True)
    dt = stage(dev)
    E = torch.linspace(-1.3, 1.2, nE, dtype=torch.float64, device="cuda")
    log(f"[noalloc] N={N} M={M} nE={nE}")
    T_na, i_na = _noalloc(lib, dt, E)
    T_ref, i_ref = lib.transmission(dt, E, ETA)
    torch.cuda.synchronize()
    T_ref, i_ref = T_ref.cpu().numpy(), i_ref.cpu().numpy()
    ok, rel, ab = fp64_close(T_na, T_ref)
    log(f"[noalloc]   max |dT| {ab:.2e}, bitwise {np.array_equal(T_na, T_ref)}")
    assert ok and np.array_equal(i_na, i_ref) and np.all(i_na == 0)
    assert np.array_equal(T_na, T_ref)


def test_noalloc_twice_second_smaller(lib):
    """Back to back in one process: a large call, then a smaller one, each equal to the
    allocating entry point."""
    import torch
    for N, M, nE, seed in ((4, 150, 12, 41), (2, 40, 3, 42)):
        dev = synth.random_small_device(N, M, seed=seed)
        dt = stage(dev)
        E = torch.linspace(-0.7, 0.9, nE, dtype=torch.float64, device="cuda")
        T_na, _ = _noalloc(lib, dt, E)
        T_ref, _ = lib.transmission(dt, E, ETA)
        torch.cuda.synchronize()
        assert np.array_equal(T_na, T_ref.cpu().numpy()), (N, M)
