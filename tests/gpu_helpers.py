"""Shared helpers of the GPU tests: stage synth devices on the GPU, compare with the oracle."""
from __future__ import annotations

import os
import sys

import numpy as np

FP64_RTOL = 1e-8     # |T_gpu - T_oracle| <= 1e-8 |T_oracle| + 1e-12 (FP64 path)
FP64_ATOL = 1e-12
MIXED_ATOL = 1e-4    # |T_gpu - T_oracle| <= 1e-4 (mixed path)


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def stage(dev, device="cuda"):
    """synth.Device -> DeviceTensors (a repeated layer is replicated on the GPU)."""
    from paper_2609_37058_amd import staging
    if dev.base is not None:
        b = dev.base
        out = staging.stage_repeated(b.H00, b.H01, b.S00, b.S01, dev.N, dev.shifts, device=device)
        if dev.left is not b or dev.right is not b:
            left = staging.stage_lead(dev.left.H00, dev.left.H01, dev.left.S00, dev.left.S01, device)
            right = left if dev.right is dev.left else staging.stage_lead(
                dev.right.H00, dev.right.H01, dev.right.S00, dev.right.S01, device)
            out.left, out.right = left, right
        return out
    left = staging.stage_lead(dev.left.H00, dev.left.H01, dev.left.S00, dev.left.S01, device)
    right = left if dev.right is dev.left else staging.stage_lead(
        dev.right.H00, dev.right.H01, dev.right.S00, dev.right.S01, device)
    hd, hu, sd, su = dev.stacked()
    return staging.stage_blocks(hd, hu, sd, su, left, right, device)


def gpu_transmission(dev_t, energies, eta, precision="fp64"):
    import torch
    from paper_2609_37058_amd import rgf
    E = torch.as_tensor(np.asarray(energies, np.float64)).cuda()
    T, info = rgf.transmission(dev_t, E, eta, precision)
    torch.cuda.synchronize()
    return T.cpu().numpy(), info.cpu().numpy()


def fp64_close(t_gpu, t_ref):
    err = np.abs(t_gpu - t_ref)
    bound = FP64_RTOL * np.abs(t_ref) + FP64_ATOL
    return bool(np.all(err <= bound)), float(np.max(err / (np.abs(t_ref) + 1e-300))), float(np.max(err))


class force_batched_path:
    """Route even tiny blocks through the batched (matrix-core) path for the duration."""

    def __enter__(self):
        self.old = os.environ.get("RGF_SMALL_MAX_M")
        os.environ["RGF_SMALL_MAX_M"] = "0"

    def __exit__(self, *a):
        if self.old is None:
            os.environ.pop("RGF_SMALL_MAX_M", None)
        else:
            os.environ["RGF_SMALL_MAX_M"] = self.old
