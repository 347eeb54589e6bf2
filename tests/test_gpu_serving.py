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
