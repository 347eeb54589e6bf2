"""Write the oracle's expected transmissions for sampled energies of the full-size workloads.

Calls only ``oracle`` and ``synth`` (no GPU code).  Usage:
    python tests/golden/make_golden.py c2 c3 c4
Each output tests/golden/<cfg>.json holds the grid indices, energies and the
FP64 oracle's T_LR (block-Thomas solve, Sancho-Rubio leads) plus the imaginary
part of the trace and the decimation iteration counts.

Samples: C2 -- 16 seeded grid points plus the 8 grid points nearest to the
lead's band extrema (bands on 512 k-points); C3 -- 6 seeded grid points;
C4 -- 2 seeded grid points (about 3 CPU-minutes each on 8 cores).
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

SAMPLES = {"c2": (16, 8), "c3": (6, 0), "c4": (2, 0)}


def sample_indices(cfg, n_rand: int, n_edge: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0, 7]))
    idx = set(rng.choice(len(cfg.energies), size=n_rand, replace=False).tolist())
    if n_edge:
        ext = oracle.band_extrema(cfg.device.left, nk=512)
        dist = np.min(np.abs(cfg.energies[:, None] - ext[None, :]), axis=1)
        for i in np.argsort(dist):
            if len(idx) >= n_rand + n_edge:
                break
            idx.add(int(i))
    return np.array(sorted(idx))


def main(names):
    for name in names:
        cfg = {"c2": synth.config_c2, "c3": synth.config_c3, "c4": synth.config_c4}[name]()
        n_rand, n_edge = SAMPLES[name]
        idx = sample_indices(cfg, n_rand, n_edge, seed={"c2": 2, "c3": 3, "c4": 4}[name])
        E = cfg.energies[idx]
        t0 = time.time()
        T, tr, infos = oracle.transmission(cfg.device, E, cfg.eta, method="thomas", return_info=True)
        out = {
            "config": name,
            "N": cfg.device.N,
            "M": cfg.device.M,
            "eta": cfg.eta,
            "n_grid": len(cfg.energies),
            "indices": idx.tolist(),
            "E": E.tolist(),
            "T": T.tolist(),
            "imag_trace": tr.imag.tolist(),
            "sr_iters": [i["iters_left"] for i in infos],
            "oracle": "oracle.transmission(method='thomas'), FP64, Sancho-Rubio leads",
            "cpu_seconds": round(time.time() - t0, 1),
        }
        path = os.path.join(HERE, f"{name}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(f"{name}: {len(E)} energies in {out['cpu_seconds']} s -> {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c2", "c3", "c4"])
