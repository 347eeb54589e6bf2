"""Serving on the GPU: continuous batching, lead cache, admission by HBM budget.

Each request's result must equal the same solve run alone through
rgf_transmission (bitwise for FP64), and the oracle within the FP64 bar.
"""
import time

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import fp64_close, gpu_transmission, log, stage

pytestmark = pytest.mark.gpu


def _requests(n, sizes=(64, 128), n_layers=(3, 9), n_e=(4, 12)):
    return synth.c5_requests(n_req=n, qps=50.0, sizes=sizes, n_layers=n_layers, n_e=n_e, seed=55)


def _submit(srv, req, precision="fp64"):
    d = req.device
    hd, hu, sd, su = d.stacked()
    lead = (d.left.H00, d.left.H01, d.left.S00, d.left.S01)
    return srv.submit(hd, hu, sd, su, lead, lead, req.energies, 1e-6, precision,
                      lead_key_L=req.lead_key, lead_key_R=req.lead_key)


def test_mix_equals_alone_and_oracle(lib):
    from paper_2609_37058_amd import rgf
    reqs = _requests(10)
    with rgf.Server(lead_cache_bytes=1 << 30, max_slots=3) as srv:
        t0 = time.time()
        tickets = []
        for r in reqs:   # Poisson arrivals: later requests arrive while earlier ones run
            while time.time() - t0 < r.arrival_s:
                time.sleep(0.001)
            tickets.append(_submit(srv, r))
        results = [srv.wait(t) for t in tickets]
        stats = srv.stats()
    log(f"[serve] stats {stats}")
    assert stats["finished"] == len(reqs)
    for k, (r, (T, info, lat)) in enumerate(zip(reqs, results)):
        alone, info_a = gpu_transmission(stage(r.device), r.energies, 1e-6)
        assert np.all(info == 0)
        assert np.array_equal(T, alone), (r.index, T - alone)
        msg = f"[serve] req {r.index}: N={r.device.N} M={r.device.M} nE={len(r.energies)} latency {lat*1e3:.1f} ms"
        if k < 3:   # the oracle on a few requests keeps the test within its time limit
            ref = oracle.transmission(r.device, r.energies[:4], 1e-6)
            ok, rel, ab = fp64_close(T[:4], ref)
            msg += f" max rel vs oracle {rel:.2e}"
            assert ok
        log(msg)


def test_lead_cache_hits_give_identical_results(lib):
    from paper_2609_37058_amd import rgf
    reqs = _requests(2, sizes=(64,))
    r = reqs[0]
    with rgf.Server(lead_cache_bytes=1 << 30, max_slots=2) as srv:
        T1, _, _ = srv.wait(_submit(srv, r))
        s1 = srv.stats()
        T2, _, _ = srv.wait(_submit(srv, r))
        s2 = srv.stats()
    log(f"[serve] cache stats first {s1} second {s2}")
    assert s2["cache_hits"] - s1["cache_hits"] == len(r.energies)
    assert np.array_equal(T1, T2)


def test_too_big_request_is_rejected(lib):
    from paper_2609_37058_amd import rgf
    r = _requests(1, sizes=(128,))[0]
    with rgf.Server(hbm_budget_bytes=1 << 20, max_slots=1) as srv:
        with pytest.raises(rgf.RgfError) as e:
            _submit(srv, r)
        assert e.value.code == rgf.RGF_ETOOBIG


def test_admission_waits_for_budget(lib):
    """A budget that fits one request at a time: all still finish, peak in-flight bytes stay within it."""
    from paper_2609_37058_amd import rgf
    reqs = _requests(4, sizes=(64,), n_layers=(4, 4), n_e=(8, 8))
    budget = 64 << 20
    with rgf.Server(hbm_budget_bytes=budget, max_slots=4) as srv:
        tickets = [_submit(srv, r) for r in reqs]
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
    log(f"[serve] budget stats {st}")
    assert st["finished"] == 4
    assert st["peak_inflight_bytes"] <= budget
    for r, (T, info, lat) in zip(reqs, res):
        alone, _ = gpu_transmission(stage(r.device), r.energies, 1e-6)
        assert np.array_equal(T, alone)


def _repeated(N, M, seed):
    """A device of one seeded decay-weighted layer repeated N times (also its lead)."""
    return synth.repeated_device(synth.decay_layer(seed, 0, M), N, name=f"rep-{seed}")


def _submit_dev(srv, dev, E, key, precision="fp64"):
    hd, hu, sd, su = dev.stacked()
    lead = (dev.left.H00, dev.left.H01, dev.left.S00, dev.left.S01)
    return srv.submit(hd, hu, sd, su, lead, lead, E, 1e-6, precision, lead_key_L=key, lead_key_R=key)


def test_large_blocks_and_mixed_precision_equal_alone(lib):
    """Requests at M = 256, 512 and 1024 in FP64 and mixed precision, arriving while others run:
    each equals the same solve alone (bitwise, its own precision); FP64 ones also match the oracle."""
    from paper_2609_37058_amd import rgf
    reqs = synth.c5_requests(n_req=6, qps=20.0, sizes=(256, 512, 1024), n_layers=(3, 5), n_e=(6, 12), seed=77)
    precs = ["fp64", "mixed", "fp64", "mixed", "fp64", "mixed"]
    with rgf.Server(lead_cache_bytes=4 << 30, max_slots=3) as srv:
        t0 = time.time()
        tickets = []
        for r, p in zip(reqs, precs):
            while time.time() - t0 < r.arrival_s:
                time.sleep(0.001)
            tickets.append(_submit(srv, r, p))
        results = [srv.wait(t) for t in tickets]
        stats = srv.stats()
    log(f"[serve] large-block stats {stats}")
    checked = 0
    for r, p, (T, info, lat) in zip(reqs, precs, results):
        alone, _ = gpu_transmission(stage(r.device), r.energies, 1e-6, p)
        msg = f"[serve] req {r.index} {p}: N={r.device.N} M={r.device.M} nE={len(r.energies)} {lat:.2f} s"
        assert np.all(info == 0)
        assert np.array_equal(T, alone), (r.index, p, np.max(np.abs(T - alone)))
        if p == "fp64" and checked < 2:
            ref = oracle.transmission(r.device, r.energies[:2], 1e-6, method="thomas")
            ok, rel, ab = fp64_close(T[:2], ref)
            msg += f", max rel vs oracle {rel:.2e}"
            assert ok
            checked += 1
        log(msg)


def test_head_request_is_passed_but_not_starved(lib):
    """The blocks of a large request do not fit next to a long-running one: smaller requests
    behind it are admitted first, but at most 4 of them; it still finishes, and every result
    equals the solve alone."""
    from paper_2609_37058_amd import rgf
    M = 64
    long_dev, big_dev = _repeated(20, M, 601), _repeated(100, M, 602)
    smalls = [_repeated(4, M, 610 + i) for i in range(7)]
    grid = np.linspace(-1.5, 1.5, 1024)
    blk = lambda d: (4 * d.N - 2 + 4) * M * M * 16
    # arenas: half the budget; the other half holds the long request and 4 small ones, or the large one
    room = blk(big_dev) + blk(smalls[0]) // 2
    assert blk(long_dev) + blk(big_dev) > room >= blk(long_dev) + 4 * blk(smalls[0])
    with rgf.Server(hbm_budget_bytes=2 * room, lead_cache_bytes=0, max_slots=2) as srv:
        t_long = _submit_dev(srv, long_dev, grid, 1)
        t_big = _submit_dev(srv, big_dev, grid[::64], 2)
        t_small = [_submit_dev(srv, d, grid[::128], 10 + i) for i, d in enumerate(smalls)]
        res_long, res_big = srv.wait(t_long), srv.wait(t_big)
        res_small = [srv.wait(t) for t in t_small]
        st = srv.stats()
    log(f"[serve] head-of-line stats {st}; latency long {res_long[2]:.2f} s, big {res_big[2]:.2f} s, "
        f"smalls {[round(r[2], 3) for r in res_small]}")
    assert st["finished"] == 9 and st["peak_inflight_bytes"] <= 2 * room
    assert 1 <= st["admitted_ahead"] <= 4
    for dev, E, (T, info, lat) in [(long_dev, grid, res_long), (big_dev, grid[::64], res_big)] + \
            [(d, grid[::128], r) for d, r in zip(smalls, res_small)]:
        alone, _ = gpu_transmission(stage(dev), E, 1e-6)
        assert np.array_equal(T, alone) and np.all(info == 0)


def test_long_request_does_not_hold_a_slot(lib):
    """One worker: a short request submitted right after a long one finishes long before it,
    because work is handed out per item (round-robin over the requests), not per request."""
    from paper_2609_37058_amd import rgf
    long_dev, short_dev = _repeated(20, 64, 701), _repeated(4, 64, 702)
    grid = np.linspace(-1.5, 1.5, 1024)
    with rgf.Server(lead_cache_bytes=0, max_slots=1) as srv:
        t_long = _submit_dev(srv, long_dev, grid, 1)
        t_short = _submit_dev(srv, short_dev, grid[:8], 2)
        T_s, _, lat_s = srv.wait(t_short)
        T_l, _, lat_l = srv.wait(t_long)
    log(f"[serve] one slot: long {lat_l:.3f} s, short {lat_s:.3f} s")
    assert lat_s < 0.5 * lat_l
    assert np.array_equal(T_s, gpu_transmission(stage(short_dev), grid[:8], 1e-6)[0])
