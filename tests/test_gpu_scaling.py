"""Linear scaling of the transmission cost with device length (Results: the RGF stage costs
O(N_z M_b^3) per energy, and the workflow's time grows linearly with the number of atoms).

At fixed block size M = 512 the time of rgf_transmission over N in {50, 100, 200, 400} layers
(doped repeated layers, 32 energies, FP64) must fit t = a + b N with R^2 >= 0.99; each point
is the median of three HIP-event-timed calls after a warm-up.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import log

pytestmark = pytest.mark.gpu


def test_time_is_linear_in_layers(lib):
    import torch
    from paper_2609_37058_amd import staging
    layer = synth.decay_layer(3, 0, 512)
    E = torch.linspace(-1.0, 1.0, 32, dtype=torch.float64, device="cuda")
    Ns, ts = [50, 100, 200, 400], []
    for N in Ns:
        dt = staging.stage_repeated(layer.H00, layer.H01, layer.S00, layer.S01, N,
                                    synth.dopant_shifts(303, N))
        lib.transmission(dt, E, 1e-6)  # warm-up (workspaces)
        torch.cuda.synchronize()
        reps = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            lib.transmission(dt, E, 1e-6)
            e1.record()
            e1.synchronize()
            reps.append(e0.elapsed_time(e1))
        ts.append(float(np.median(reps)))
        log(f"[scaling] N={N}: {ts[-1]:.1f} ms")
        del dt
    A = np.vstack([np.ones(len(Ns)), Ns]).T
    coef, *_ = np.linalg.lstsq(A, np.array(ts), rcond=None)
    pred = A @ coef
    r2 = 1.0 - np.sum((np.array(ts) - pred) ** 2) / np.sum((np.array(ts) - np.mean(ts)) ** 2)
    log(f"[scaling] t = {coef[0]:.1f} + {coef[1]:.3f} N ms, R^2 = {r2:.5f}")
    assert r2 >= 0.99 and coef[1] > 0
