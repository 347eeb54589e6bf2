"""Planted mistakes in the oracle (on the CPU) must be caught by its pins.

Each mutation replaces one oracle function by a plausibly wrong variant
(a transposed operand, a dropped term, a wrong sign, the wrong surface);
the pin battery below, a fast subset of ``test_oracle_pins``, must then
fail.  This shows the pins constrain the oracle rather than restate it.
"""
import numpy as np
import pytest

import oracle
import oracle.rgf_oracle as ro
import synth

ETA = 1e-6


def _battery() -> bool:
    """True when every pin in the fast battery holds."""
    ok = True
    # integer channels of the pristine C1 device (complex couplings)
    cfg = synth.config_c1()
    E = cfg.energies[::5]
    T = ro.transmission(cfg.device, E, cfg.eta, method="dense")
    ext = ro.band_extrema(cfg.device.left)
    keep = np.array([np.min(np.abs(ext - e)) > 1e-2 for e in E])
    nch = ro.channel_count(cfg.device.left, E)
    ok &= bool(np.max(np.abs(T - nch)[keep]) <= 1e-3)
    # scalar chain closed forms
    dev = synth.chain_device(10, 0.0, -1.0, 0.1)
    ok &= bool(np.all(np.abs(ro.transmission(dev, [-1.0, 0.6, 1.8], ETA) - 1.0) < 1e-3))
    dev = synth.chain_device(11, 0.0, -1.0, 0.0, impurity=(5, 0.9))
    e = np.array([-1.1, 0.5])
    k = np.arccos(e / -2.0)
    ok &= bool(np.all(np.abs(ro.transmission(dev, e, 1e-7) - 1 / (1 + (0.9 / (2 * np.sin(k))) ** 2)) < 1e-4))
    # decimation versus Bloch modes, both surfaces
    lead = synth.random_small_device(1, 4, seed=64).left
    for en in (-1.1, 0.23, 1.9):
        z = complex(en, ETA)
        gl, gr, _, _ = ro.sancho_rubio(lead, z)
        bl, br = ro.surface_gf_bloch(lead, z)
        ok &= bool(np.linalg.norm(gl - bl) <= 1e-8 * np.linalg.norm(bl))
        ok &= bool(np.linalg.norm(gr - br) <= 1e-8 * np.linalg.norm(br))
    # Gamma is positive semidefinite (a sign flip of both Gammas cancels in T)
    sl, sr, _ = ro.self_energies(lead, lead, complex(0.23, ETA))
    for sg in (sl, sr):
        w = np.linalg.eigvalsh(ro.broadening(sg))
        ok &= bool(w.min() >= -1e-12 * np.abs(w).max())
    # dense versus block-Thomas, both directions, and the mirror identity
    dev = synth.random_small_device(5, 3, seed=45, distinct_leads=True)
    E = np.array([-1.3, 0.4])
    for d in ("LR", "RL"):
        a = ro.transmission(dev, E, ETA, method="dense", direction=d)
        b = ro.transmission(dev, E, ETA, method="thomas", direction=d)
        ok &= bool(np.max(np.abs(a - b)) <= 1e-10 * max(1, np.abs(a).max()))
    a = ro.transmission(dev, E, ETA, direction="RL")
    b = ro.transmission(dev.mirrored(), E, ETA, direction="LR")
    ok &= bool(np.max(np.abs(a - b)) <= 1e-10 * max(1, np.abs(a).max()))
    return ok


def test_battery_passes_on_true_oracle():
    assert _battery()


def _lead_ops_no_conj(lead, z):
    D = z * lead.S00 - lead.H00
    U = z * lead.S01 - lead.H01
    L = z * lead.S01.T - lead.H01.T          # transposed instead of adjoint
    return D, U, L


def _lead_ops_conj_z(lead, z):
    D = z * lead.S00 - lead.H00
    U = z * lead.S01 - lead.H01
    L = np.conj(z) * lead.S01.conj().T - lead.H01.conj().T   # z conjugated in the lower block
    return D, U, L


def _device_ops_swapped(dev, z, i):
    A = z * dev.Sd(i) - dev.Hd(i)
    if i < dev.N - 1:
        L = z * dev.Su(i) - dev.Hu(i)            # upper and lower couplings swapped
        U = z * dev.Su(i).conj().T - dev.Hu(i).conj().T
    else:
        U = L = None
    return A, U, L


def _caroli_no_dagger(ga, G, gb):
    return np.trace(ga @ G @ gb @ G.T)


def _broadening_wrong_sign(s):
    return -1j * (s - s.conj().T)


_orig_sr = ro.sancho_rubio


def _sr_wrong_surface(lead, z, tol=ro.SR_TOL, maxit=ro.SR_MAXIT):
    gl, gr, it, ok = _orig_sr(lead, z, tol, maxit)
    return gr, gl, it, ok                          # surfaces exchanged


def _sr_one_step(lead, z, tol=ro.SR_TOL, maxit=ro.SR_MAXIT):
    return _orig_sr(lead, z, tol, 3)               # stops far too early


_orig_self = ro.self_energies


def _self_energies_swapped(left, right, z, tol=ro.SR_TOL, maxit=ro.SR_MAXIT, method="sancho_rubio"):
    sl, sr, info = _orig_self(left, right, z, tol, maxit, method)
    _, UL, LL = ro.lead_operators(left, z)
    gl = np.linalg.solve(LL, sl) @ np.linalg.inv(UL)
    return UL @ gl @ LL, sr, info                  # U g L on the left instead of L g U


MUTATIONS = {
    "lead_L_transposed_not_adjoint": ("lead_operators", _lead_ops_no_conj),
    "lead_L_conjugated_z": ("lead_operators", _lead_ops_conj_z),
    "device_couplings_swapped": ("_device_ops", _device_ops_swapped),
    "caroli_missing_conjugate": ("_caroli", _caroli_no_dagger),
    "gamma_wrong_sign": ("broadening", _broadening_wrong_sign),
    "sr_surfaces_exchanged": ("sancho_rubio", _sr_wrong_surface),
    "sr_stopped_early": ("sancho_rubio", _sr_one_step),
    "sigma_left_wrong_order": ("self_energies", _self_energies_swapped),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(ro, attr, fn)
    with np.errstate(all="ignore"):
        try:
            ok = _battery()
        except (np.linalg.LinAlgError, ValueError):
            ok = False
    assert not ok, f"mutation {name} slipped through the pins"
