"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test checks the oracle against a closed form, an invariant, a brute
force or an independent algorithm, so that a dropped term, a wrong sign or
index, or a transposed operand in the oracle fails at least one of them
(``test_oracle_mutations`` plants such mistakes and checks that they are
caught).
"""
import numpy as np
import pytest

import oracle
import synth

ETA = 1e-6


# ---------------------------------------------------------------------------
# 1D chains: closed forms (textbook tight-binding scattering)
# ---------------------------------------------------------------------------

def test_chain_orthogonal_unit_transmission_in_band():
    """eps0 = 0, t = -1, s = 0: T = 1 for |E| < 2 and T = 0 for |E| > 2."""
    dev = synth.chain_device(12, 0.0, -1.0, 0.0)
    e_in = np.array([-1.9, -1.3, -0.7, -0.05, 0.05, 0.8, 1.5, 1.95])
    e_out = np.array([-3.5, -2.2, 2.1, 2.8])
    t_in = oracle.transmission(dev, e_in, ETA)
    t_out = oracle.transmission(dev, e_out, ETA)
    assert np.all(np.abs(t_in - 1.0) < 1e-3)
    assert np.all(np.abs(t_out) < 1e-6)


def test_chain_nonorthogonal_band_edges():
    """s = 0.1: band = [(eps0 + 2t)/(1 + 2s), (eps0 - 2t)/(1 - 2s)] = [-5/3, 5/2]."""
    eps0, t, s = 0.0, -1.0, 0.1
    lo, hi = (eps0 + 2 * t) / (1 + 2 * s), (eps0 - 2 * t) / (1 - 2 * s)
    dev = synth.chain_device(12, eps0, t, s)
    e_in = np.linspace(lo + 0.05, hi - 0.05, 9)
    e_in = e_in[np.abs(e_in - eps0) > 1e-2]
    e_out = np.array([lo - 0.3, lo - 0.05, hi + 0.05, hi + 0.5])
    assert np.all(np.abs(oracle.transmission(dev, e_in, ETA) - 1.0) < 1e-3)
    assert np.all(np.abs(oracle.transmission(dev, e_out, ETA)) < 1e-6)


def _scalar_surface_gf(eps0, t, s, z):
    """Scalar lead: g = 1/(w - b^2 g), w = z - eps0, b = z s - t; the decaying root |b g| < 1."""
    w = z - eps0
    b = z * s - t
    disc = np.sqrt(w * w - 4 * b * b + 0j)
    roots = [(w + disc) / (2 * b * b), (w - disc) / (2 * b * b)]
    good = [g for g in roots if abs(b * g) < 1.0]
    assert len(good) == 1
    return good[0]


@pytest.mark.parametrize("s", [0.0, 0.1, -0.15])
@pytest.mark.parametrize("E", [-2.6, -1.4, -0.3, 0.45, 1.2, 2.3, 3.1])
def test_sancho_rubio_scalar_closed_form(s, E):
    """M = 1: decimation reproduces the root of the scalar surface Dyson equation (both sides)."""
    eps0, t = 0.2, -1.0
    lead = synth.chain_lead(eps0, t, s)
    z = complex(E, ETA)
    gl, gr, it, ok = oracle.sancho_rubio(lead, z)
    g = _scalar_surface_gf(eps0, t, s, z)
    assert ok
    assert abs(gr[0, 0] - g) <= 1e-9 * max(1.0, abs(g))
    assert abs(gl[0, 0] - g) <= 1e-9 * max(1.0, abs(g))
    assert gr[0, 0].imag <= 0.0


@pytest.mark.parametrize("U", [0.4, 1.3])
def test_chain_single_impurity(U):
    """On-site impurity U in an orthogonal chain: T = 1 / (1 + (U / (2|t| sin k))^2), E = 2t cos k."""
    t = -1.0
    dev = synth.chain_device(11, 0.0, t, 0.0, impurity=(5, U))
    E = np.array([-1.7, -1.1, -0.4, 0.3, 0.9, 1.6])
    k = np.arccos(E / (2 * t))
    expect = 1.0 / (1.0 + (U / (2 * abs(t) * np.sin(k))) ** 2)
    got = oracle.transmission(dev, E, 1e-7)
    assert np.all(np.abs(got - expect) < 1e-4)


def test_decoupled_chains_with_basis_change_give_integer_transmission():
    """M decoupled chains, then one random congruence V^+ X V of every block.

    T(E) = #{m : E inside band m}, the band of chain m being [eps_m - 2|t_m|, eps_m + 2|t_m|].
    The congruence makes S nonorthogonal and all blocks dense and complex.
    """
    eps = np.array([-1.0, 0.0, 0.7, 1.5, -0.4])
    t = np.array([-1.0, -0.6, -0.8, -1.2, -0.3])
    dev = synth.decoupled_chains(eps, t, 6)
    V = synth.random_basis(len(eps), seed=11)
    devb = dev.with_basis_change(V)
    lo, hi = eps - 2 * np.abs(t), eps + 2 * np.abs(t)
    E = np.linspace(-3.2, 3.6, 41)
    edges = np.concatenate([lo, hi, eps])
    E = E[np.min(np.abs(E[:, None] - edges[None, :]), axis=1) > 2e-2]
    expect = np.sum((E[:, None] > lo[None, :]) & (E[:, None] < hi[None, :]), axis=1)
    got = oracle.transmission(devb, E, ETA)
    assert np.max(np.abs(got - expect)) < 1e-3


# ---------------------------------------------------------------------------
# Device solve: dense inversion versus block-Thomas (two formulations)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N,M", [(1, 3), (2, 4), (5, 3), (9, 5)])
def test_block_thomas_equals_dense_inversion(N, M):
    dev = synth.random_small_device(N, M, seed=40 + N, distinct_leads=True)
    E = np.array([-2.0, -0.6, 0.35, 1.7])
    for direction in ("LR", "RL"):
        d = oracle.transmission(dev, E, ETA, method="dense", direction=direction)
        b = oracle.transmission(dev, E, ETA, method="thomas", direction=direction)
        assert np.max(np.abs(d - b)) <= 1e-10 * max(1.0, np.max(np.abs(d)))


def test_mirrored_device_reverses_transmission():
    """T_LR of the mirrored device equals T_RL of the original (exact, same eta)."""
    dev = synth.random_small_device(6, 4, seed=7, distinct_leads=True)
    E = np.array([-1.5, -0.2, 0.9, 2.1])
    t_rl = oracle.transmission(dev, E, ETA, direction="RL")
    t_mir = oracle.transmission(dev.mirrored(), E, ETA, direction="LR")
    assert np.max(np.abs(t_rl - t_mir)) <= 1e-10 * max(1.0, np.max(np.abs(t_rl)))


def test_reciprocity_real_hamiltonian_exact():
    """Real H and S: z S - H is complex symmetric, so T_LR = T_RL to rounding."""
    dev = synth.random_small_device(7, 4, seed=21, real=True, distinct_leads=True)
    E = np.linspace(-2.5, 2.5, 11)
    a = oracle.transmission(dev, E, ETA, direction="LR")
    b = oracle.transmission(dev, E, ETA, direction="RL")
    assert np.all(np.abs(a - b) <= 1e-10 * np.maximum(1.0, np.abs(a)))


def test_reciprocity_complex_hamiltonian_up_to_absorption():
    """Complex couplings: T_LR - T_RL comes only from the device absorption 2 eta S; it shrinks with eta."""
    dev = synth.random_small_device(6, 4, seed=5, distinct_leads=True)
    E = np.array([-1.2, -0.3, 0.6, 1.4])
    d6 = np.abs(oracle.transmission(dev, E, 1e-6, direction="LR") - oracle.transmission(dev, E, 1e-6, direction="RL"))
    d7 = np.abs(oracle.transmission(dev, E, 1e-7, direction="LR") - oracle.transmission(dev, E, 1e-7, direction="RL"))
    assert np.all(d6 <= 1e-3)
    big = d6 > 1e-11
    assert np.all(d7[big] <= 0.3 * d6[big])


# ---------------------------------------------------------------------------
# Lead surface Green's functions: decimation versus Bloch modes, Dyson, Gamma >= 0
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("M", [2, 4, 8])
def test_sancho_rubio_matches_bloch_modes(M):
    lead = synth.random_small_device(1, M, seed=60 + M).left
    for E in [-2.7, -1.1, 0.23, 1.9, 3.3]:
        z = complex(E, ETA)
        gl, gr, it, ok = oracle.sancho_rubio(lead, z)
        bl, br = oracle.surface_gf_bloch(lead, z)
        assert ok
        assert np.linalg.norm(gl - bl) <= 1e-8 * max(1.0, np.linalg.norm(bl))
        assert np.linalg.norm(gr - br) <= 1e-8 * max(1.0, np.linalg.norm(br))


def test_dyson_residual_and_gamma_psd_c1_lead():
    cfg = synth.config_c1()
    lead = cfg.device.left
    D_norm = None
    for E in cfg.energies[::7]:
        z = complex(E, cfg.eta)
        gl, gr, it, ok = oracle.sancho_rubio(lead, z)
        assert ok and it <= 60
        D = z * lead.S00 - lead.H00
        D_norm = np.linalg.norm(D)
        for g, side in ((gl, "left"), (gr, "right")):
            r = oracle.dyson_residual(lead, z, g, side)
            assert r <= 1e-9 * (1.0 + np.linalg.norm(g) * D_norm)
        sl, sr, _ = oracle.self_energies(lead, lead, z)
        for s in (sl, sr):
            gam = oracle.broadening(s)
            w = np.linalg.eigvalsh(gam)
            assert w.min() >= -1e-12 * max(1.0, np.abs(w).max())


# ---------------------------------------------------------------------------
# Pristine devices: integer channel counts; bounds; zero coupling
# ---------------------------------------------------------------------------

def _away_from_edges(lead, energies, delta=1e-2):
    ext = oracle.band_extrema(lead)
    return np.array([np.min(np.abs(ext - e)) > delta for e in energies])


def test_c1_pristine_integer_channels_dense():
    """C1 (20 layers, M = 4, pristine): T(E) = N_ch(E) away from band extrema."""
    cfg = synth.config_c1()
    T = oracle.transmission(cfg.device, cfg.energies, cfg.eta, method="dense")
    nch = oracle.channel_count(cfg.device.left, cfg.energies)
    keep = _away_from_edges(cfg.device.left, cfg.energies)
    assert keep.sum() > 150
    assert np.max(np.abs(T - nch)[keep]) <= 1e-3
    assert np.all(T >= -1e-12)
    assert nch.max() >= 2


def test_transmission_bounds_random_device():
    """0 <= T <= min(N_ch,L, N_ch,R) for a disordered device between pristine C1 leads."""
    lead = synth.layer_c1()
    rnd = synth.random_small_device(5, 4, seed=3)
    dev = synth.device_from_blocks([rnd.Hd(i) for i in range(5)], [rnd.Hu(i) for i in range(4)],
                                   [rnd.Sd(i) for i in range(5)], [rnd.Su(i) for i in range(4)],
                                   lead, lead)
    E = np.linspace(-3.5, 3.5, 29)
    T = oracle.transmission(dev, E, ETA)
    nch = oracle.channel_count(lead, E)
    assert np.all(T >= -1e-12)
    assert np.all(T <= nch + 1e-8)


def test_zero_coupling_block_gives_zero_transmission():
    dev = synth.random_small_device(5, 3, seed=9)
    hd, hu, sd, su = dev.stacked()
    hu[2] = 0.0
    su[2] = 0.0
    cut = synth.device_from_blocks(hd, hu, sd, su, dev.left, dev.right)
    T = oracle.transmission(cut, np.array([-1.0, 0.2, 1.3]), ETA, method="thomas")
    assert np.all(T == 0.0)


def test_channel_count_brute_force_chain():
    """Channel count of the M = 1 chain is 1 inside the band and 0 outside."""
    lead = synth.chain_lead(0.0, -1.0, 0.0)
    E = np.array([-2.5, -1.5, 0.3, 1.99, 2.01])
    assert list(oracle.channel_count(lead, E, nk=512)) == [0, 1, 1, 1, 0]
