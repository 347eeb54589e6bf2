"""Write the oracle's expected values for sampled energies of the full-size workloads.

Calls only ``oracle`` and ``synth`` (no GPU code).  Usage:
    python tests/golden/make_golden.py [--jobs N] [name ...]
with names from c2 c3 c4 c4_bloch kmesh_m256 bias_m1024 kpm_m1024
(default: all; c4_bloch, c4_rethread and c4_scaled read c4.json).

Transmission configs (tests/golden/<cfg>.json): grid indices, energies and
the FP64 oracle's T_LR (block-Thomas solve, Sancho-Rubio leads), the
imaginary part of the trace and the decimation iteration counts.
  c2 -- every one of the 1000 grid energies;
  c3 -- 120 seeded grid points plus the 8 grid points nearest the lead's band
        extrema (bands on 512 k-points);
  c4 -- 8 seeded grid points plus the 8 nearest the band extrema (bands on
        256 k-points); about 3 CPU-minutes per energy on 8 cores.
  c4_bloch -- add to c4.json, for every sampled energy, T from the
        Bloch-mode construction of the lead surface GFs (``method="bloch"``,
        an algorithm independent of decimation) on the same block-Thomas
        solve.  Where the lead's bands have sharp features T's FP64 value is
        only reproducible to the spread of such constructions (the tests add
        it to the bar).  One 2M x 2M eigenproblem per energy, about 14 CPU-
        minutes at M = 1024; --jobs N runs N energies at once.
  c4_rethread -- add to c4.json, for every sampled energy, T from the same
        construction as T with the oracle's BLAS limited to 4 threads: a
        different summation order, so the difference from T is the oracle's
        own FP64 reproducibility there (the tests add it to the bar too; on
        this machine it came out bitwise equal to T).
  c4_scaled -- add to c4.json, for every sampled energy, T of the device and
        electrodes with every H and S block times 3: exactly T in exact
        arithmetic (z 3S - 3H = 3 (zS - H) scales G by 1/3 and Sigma, Gamma by
        3), with every rounding changed, so its difference from T is T's FP64
        sensitivity to rounding there (the tests add it to the bar too).
The forms beyond T(E) at the shapes the benchmark times, reduced in the
layer count only:
  kmesh_m256 -- the benchmark's k-mesh recipe (decay-weighted layers of
        M = 256 with transverse images on both in-plane axes) at N = 4 on the
        7 x 7 mesh, 2 energies: every T_k and the average;
  bias_m1024 -- the C4 device's first 3 layers at V_b = 0.2 V (electrodes
        shifted by +-0.1 eV), 3 energies of the bias window;
  kpm_m1024 -- the C4 central region's first 4 layers (N M = 4096), 4
        random-phase vectors, 48 Chebyshev moments with the norm bounds.
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
import oracle.bias as obias  # noqa: E402
import oracle.kmesh as okm  # noqa: E402
import oracle.kpm as okpm  # noqa: E402
import synth  # noqa: E402

# (seeded energies, band-edge energies, k-points for the band extrema); None: every grid point
SAMPLES = {"c2": None, "c3": (120, 8, 512), "c4": (8, 8, 256)}

# the reduced NEXT-row cases (recipe parameters shared with the tests through this module)
KMESH = {"N": 4, "M": 256, "mesh": 7, "image_seed": 77, "grid": (-1.0, 1.0, 16), "pick": [5, 11]}
BIAS = {"N": 3, "V": 0.2, "energies": [-0.35, 0.02, 0.31]}
KPM = {"N": 4, "R": 4, "n_mom": 48, "vector_seed": 2024}


def sample_indices(cfg, n_rand: int, n_edge: int, nk: int, seed: int, edges_only: bool = False) -> np.ndarray:
    """Seeded grid points plus the n_edge grid points nearest the lead's band extrema (those not
    already drawn); edges_only returns the latter alone."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0, 7]))
    idx = set(rng.choice(len(cfg.energies), size=n_rand, replace=False).tolist())
    edge = []
    if n_edge:
        ext = oracle.band_extrema(cfg.device.left, nk=nk)
        dist = np.min(np.abs(cfg.energies[:, None] - ext[None, :]), axis=1)
        for i in np.argsort(dist, kind="stable"):
            if len(idx) >= n_rand + n_edge:
                break
            if int(i) not in idx:
                idx.add(int(i))
                edge.append(int(i))
    return np.array(sorted(edge if edges_only else idx))


def _bloch_T(args):
    name, i = args
    from threadpoolctl import threadpool_limits
    cfg = CONFIGS[name]()
    z = complex(cfg.energies[i], cfg.eta)
    with threadpool_limits(limits=2):
        sl, sr, _ = oracle.self_energies(cfg.device.left, cfg.device.right, z, method="bloch")
        return i, float(oracle.transmission_block_thomas(cfg.device, z, sl, sr).real)


def bloch_spread(name, jobs):
    """T from Bloch-mode leads at every sampled energy of an existing golden (see the header);
    also records which samples are the band-edge picks."""
    import concurrent.futures as cf
    path = os.path.join(HERE, f"{name}.json")
    with open(path) as f:
        out = json.load(f)
    cfg = CONFIGS[name]()
    edge = sample_indices(cfg, *SAMPLES[name], seed=SEEDS[name], edges_only=True).tolist()
    assert all(i in out["indices"] for i in edge)
    t0 = time.time()
    with cf.ProcessPoolExecutor(max_workers=jobs) as ex:
        res = dict(ex.map(_bloch_T, [(name, i) for i in out["indices"]]))
    out["edge_indices"] = edge
    out["T_bloch"] = [res[i] for i in out["indices"]]
    out["bloch_oracle"] = "oracle.self_energies(method='bloch') + oracle.transmission_block_thomas, FP64"
    out["bloch_cpu_seconds"] = round(time.time() - t0, 1)
    write(name, out)


def _rethread_T(args):
    name, i, threads = args
    from threadpoolctl import threadpool_limits
    cfg = CONFIGS[name]()
    with threadpool_limits(limits=threads):
        T = oracle.transmission(cfg.device, cfg.energies[i:i + 1], cfg.eta, method="thomas")
    return i, float(np.real(T[0]))


def rethread_spread(name, jobs, threads=4):
    """T at every sampled energy of an existing golden from the same oracle construction with its
    BLAS limited to `threads` threads (see the header)."""
    import concurrent.futures as cf
    path = os.path.join(HERE, f"{name}.json")
    with open(path) as f:
        out = json.load(f)
    idx = out["indices"]
    t0 = time.time()
    with cf.ProcessPoolExecutor(max_workers=jobs) as ex:
        res = dict(ex.map(_rethread_T, [(name, i, threads) for i in idx]))
    out["rethread_indices"] = idx
    out["T_rethread"] = [res[i] for i in idx]
    out["rethread_oracle"] = f"{out['oracle']}, BLAS limited to {threads} threads"
    out["rethread_cpu_seconds"] = round(time.time() - t0, 1)
    write(name, out)


def scaled_device(dev, c):
    """Every block of the device and its electrodes times c.  Then z cS - cH = c (zS - H), so G
    becomes G / c and Sigma, Gamma become c Sigma, c Gamma: T = Tr[Gamma_L G Gamma_R G^+] is
    unchanged in exact arithmetic, while every rounding of the computation changes."""
    import dataclasses
    sc = lambda L: synth.Lead(c * L.H00, c * L.H01, c * L.S00, c * L.S01)
    if dev.base is not None and dev._hd is None:
        return dataclasses.replace(dev, left=sc(dev.left), right=sc(dev.right), base=sc(dev.base),
                                   shifts={k: c * v for k, v in dev.shifts.items()})
    N = dev.N
    return synth.device_from_blocks([c * dev.Hd(i) for i in range(N)], [c * dev.Hu(i) for i in range(N - 1)],
                                    [c * dev.Sd(i) for i in range(N)], [c * dev.Su(i) for i in range(N - 1)],
                                    sc(dev.left), sc(dev.right), name=dev.name + "-scaled")


SCALE = 3.0


def _scaled_T(args):
    name, i = args
    from threadpoolctl import threadpool_limits
    cfg = CONFIGS[name]()
    with threadpool_limits(limits=4):
        T = oracle.transmission(scaled_device(cfg.device, SCALE), cfg.energies[i:i + 1], cfg.eta, method="thomas")
    return i, float(np.real(T[0]))


def scaled_spread(name, jobs):
    """T at every sampled energy of an existing golden from the device and electrodes scaled by
    SCALE (see the header)."""
    import concurrent.futures as cf
    path = os.path.join(HERE, f"{name}.json")
    with open(path) as f:
        out = json.load(f)
    idx = out["indices"]
    t0 = time.time()
    with cf.ProcessPoolExecutor(max_workers=jobs) as ex:
        res = dict(ex.map(_scaled_T, [(name, i) for i in idx]))
    out["scaled_indices"] = idx
    out["T_scaled"] = [res[i] for i in idx]
    out["scaled_oracle"] = f"{out['oracle']}, every H and S block (device and electrodes) times {SCALE}"
    out["scaled_cpu_seconds"] = round(time.time() - t0, 1)
    write(name, out)


def write(name, out):
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"{name}: {out.get('cpu_seconds')} s -> {path}", flush=True)


CONFIGS = {"c2": synth.config_c2, "c3": synth.config_c3, "c4": synth.config_c4}
SEEDS = {"c2": 2, "c3": 3, "c4": 4}


def transmission_config(name):
    cfg = CONFIGS[name]()
    spec = SAMPLES[name]
    if spec is None:
        idx = np.arange(len(cfg.energies))
    else:
        idx = sample_indices(cfg, *spec, seed=SEEDS[name])
    E = cfg.energies[idx]
    t0 = time.time()
    T, tr, infos = oracle.transmission(cfg.device, E, cfg.eta, method="thomas", return_info=True)
    write(name, {
        "config": name, "N": cfg.device.N, "M": cfg.device.M, "eta": cfg.eta, "n_grid": len(cfg.energies),
        "indices": idx.tolist(), "E": E.tolist(), "T": T.tolist(), "imag_trace": tr.imag.tolist(),
        "sr_iters": [i["iters_left"] for i in infos],
        "band_edge_samples": 0 if spec is None else spec[1],
        "oracle": "oracle.transmission(method='thomas'), FP64, Sancho-Rubio leads",
        "cpu_seconds": round(time.time() - t0, 1)})


def kmesh_device():
    cfg = synth.config_c2(n_layers=KMESH["N"], m=KMESH["M"], n_e=KMESH["grid"][2])
    images, R = synth.transverse_images(cfg.device, seed=KMESH["image_seed"])
    kk, w = okm.monkhorst_pack(KMESH["mesh"], KMESH["mesh"])
    E = np.linspace(*KMESH["grid"])[KMESH["pick"]]
    return cfg, images, R, kk, w, E


def bias_device():
    cfg = synth.config_c4()
    d = cfg.device
    shifts = {k: v for k, v in d.shifts.items() if k < BIAS["N"]}
    return cfg, synth.Device(BIAS["N"], d.M, d.left, d.right, base=d.base, shifts=shifts, name="c4-first3")


def kpm_device():
    cfg = synth.config_c4(n_e=1)
    d = cfg.device
    shifts = {k: v for k, v in d.shifts.items() if k < KPM["N"]}
    sub = synth.Device(KPM["N"], d.M, d.left, d.right, base=d.base, shifts=shifts, name="c4-first4")
    lo, hi = synth.kpm_bounds(d.base, d.shifts)
    r = synth.phase_vectors(KPM["N"] * d.M, KPM["R"], KPM["vector_seed"])
    return sub, lo, hi, r


def main(names, jobs=1):
    for name in names:
        t0 = time.time()
        if name in SAMPLES:
            transmission_config(name)
        elif name.endswith("_bloch") and name[:-6] in SAMPLES:
            bloch_spread(name[:-6], jobs)
        elif name.endswith("_rethread") and name[:-9] in SAMPLES:
            rethread_spread(name[:-9], jobs)
        elif name.endswith("_scaled") and name[:-7] in SAMPLES:
            scaled_spread(name[:-7], jobs)
        elif name == "kmesh_m256":
            cfg, images, R, kk, w, E = kmesh_device()
            T, Tk = okm.transmission_kmesh(images, R, kk, w, E, cfg.eta, method="thomas")
            write(name, {**KMESH, "eta": cfg.eta, "E": E.tolist(), "T": T.tolist(), "Tk": Tk.tolist(),
                         "kpts": kk.tolist(), "weights": w.tolist(), "R": [list(r) for r in R],
                         "oracle": "oracle.kmesh.transmission_kmesh(method='thomas')",
                         "cpu_seconds": round(time.time() - t0, 1)})
        elif name == "bias_m1024":
            cfg, dev = bias_device()
            E = np.array(BIAS["energies"])
            T = obias.transmission_bias(dev, E, cfg.eta, BIAS["V"] / 2, -BIAS["V"] / 2, method="thomas")
            write(name, {**BIAS, "M": dev.M, "eta": cfg.eta, "E": E.tolist(), "T": T.tolist(),
                         "oracle": "oracle.bias.transmission_bias(method='thomas')",
                         "cpu_seconds": round(time.time() - t0, 1)})
        elif name == "kpm_m1024":
            dev, lo, hi, r = kpm_device()
            mu = okpm.moments(dev, lo, hi, KPM["n_mom"], r)
            write(name, {**KPM, "M": dev.M, "bounds": [lo, hi], "mu": mu.tolist(),
                         "oracle": "oracle.kpm.moments (dense S solves)",
                         "cpu_seconds": round(time.time() - t0, 1)})
        else:
            raise SystemExit(f"unknown golden {name}")


if __name__ == "__main__":
    argv = sys.argv[1:]
    jobs = 1
    if "--jobs" in argv:
        k = argv.index("--jobs")
        jobs = int(argv[k + 1])
        del argv[k:k + 2]
    main(argv or ["kpm_m1024", "bias_m1024", "kmesh_m256", "c2", "c3", "c4", "c4_bloch", "c4_rethread", "c4_scaled"],
         jobs)
