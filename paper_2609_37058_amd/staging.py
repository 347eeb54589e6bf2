"""Host-to-device staging of device and lead blocks (input plumbing, no transport arithmetic).

Blocks are complex128, row-major; see ``include/rgf.h`` for the orientation
conventions.  A device made of one principal layer repeated N times (plus
per-layer on-site shifts) is replicated on the GPU from that one layer, so
a 400-layer M = 1024 device needs only four blocks of host memory.
"""
from __future__ import annotations

from typing import Dict, Optional

import numpy as np
import torch

from .rgf import DeviceTensors, LeadTensors


def _dev(x, device) -> torch.Tensor:
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.complex128)).to(device)


def stage_lead(H00, H01, S00, S01, device="cuda") -> LeadTensors:
    return LeadTensors(_dev(H00, device), _dev(H01, device), _dev(S00, device), _dev(S01, device))


def stage_blocks(hd, hu, sd, su, left: LeadTensors, right: LeadTensors, device="cuda") -> DeviceTensors:
    """Stacked blocks (Hd, Sd: [N, M, M]; Hu, Su: [N-1, M, M]) to the device."""
    return DeviceTensors(_dev(hd, device), _dev(hu, device), _dev(sd, device), _dev(su, device), left, right)


def stage_repeated(H00, H01, S00, S01, N: int, shifts: Optional[Dict[int, float]] = None,
                   device="cuda", lead: Optional[LeadTensors] = None) -> DeviceTensors:
    """N copies of one principal layer; layer l gets H_ll += shifts[l] * I.  The layer is also both leads
    unless ``lead`` is given."""
    layer = stage_lead(H00, H01, S00, S01, device)
    M = layer.M
    Hd = layer.H00.unsqueeze(0).repeat(N, 1, 1)
    Sd = layer.S00.unsqueeze(0).repeat(N, 1, 1)
    Hu = layer.H01.unsqueeze(0).repeat(max(N - 1, 0), 1, 1)
    Su = layer.S01.unsqueeze(0).repeat(max(N - 1, 0), 1, 1)
    if shifts:
        eye = torch.eye(M, dtype=torch.complex128, device=Hd.device)
        for l, d in shifts.items():
            Hd[l] += d * eye
    ld = lead if lead is not None else layer
    return DeviceTensors(Hd, Hu, Sd, Su, ld, ld)
