"""Pins of the finite-bias oracle and of the Landauer current (CPU).

The bias path shifts each electrode rigidly by its electrochemical
potential while the device keeps its zero-bias blocks; the current is the
trapezoid integral of (f_L - f_R) T times G0 = 2e^2/h.  Each pin below is
fixed by algebra or physics, not by the oracle itself, and the planted
mistakes at the end show that the pins constrain it.
"""
import numpy as np
import pytest

import oracle
import oracle.bias as ob
import synth

ETA = 1e-6


def shifted_device(dev, mu):
    """Every device block shifted by mu (H -> H + mu S); the electrodes are left as they are."""
    N = dev.N
    return synth.device_from_blocks([dev.Hd(i) + mu * dev.Sd(i) for i in range(N)],
                                    [dev.Hu(i) + mu * dev.Su(i) for i in range(N - 1)],
                                    [dev.Sd(i) for i in range(N)], [dev.Su(i) for i in range(N - 1)],
                                    dev.left, dev.right)


def test_conductance_quantum_value():
    # 2 e^2 / h with the exact SI constants: 7.748091729... e-5 S
    assert abs(ob.G0 - 7.748091729863649e-05) < 1e-18


def test_zero_bias_is_the_zero_bias_transmission():
    dev = synth.random_small_device(4, 3, seed=8, distinct_leads=True)
    E = np.array([-1.2, 0.1, 0.9])
    assert np.allclose(ob.transmission_bias(dev, E, ETA, 0.0, 0.0), oracle.transmission(dev, E, ETA),
                       rtol=0, atol=0)


def test_shifted_electrode_equals_energy_shift():
    """A lead shifted by mu has exactly the zero-bias self-energy at z - mu."""
    lead = synth.random_small_device(1, 4, seed=81).left
    for mu, en in ((0.3, -0.7), (-0.45, 1.1)):
        z = complex(en, ETA)
        a = oracle.self_energies(ob.shifted_lead(lead, mu), ob.shifted_lead(lead, mu), z)
        b = oracle.self_energies(lead, lead, z - mu)
        for x, y in zip(a[:2], b[:2]):
            assert np.linalg.norm(x - y) <= 1e-10 * np.linalg.norm(y)


def test_rigid_shift_of_everything_is_a_gauge():
    """Device shifted by mu and both electrodes at mu: T(E; mu, mu) = T0(E - mu)."""
    dev = synth.random_small_device(5, 3, seed=19, distinct_leads=True)
    mu = 0.37
    E = np.array([-1.0, -0.2, 0.6, 1.4])
    a = ob.transmission_bias(shifted_device(dev, mu), E, ETA, mu, mu)
    b = oracle.transmission(dev, E - mu, ETA)
    assert np.max(np.abs(a - b)) <= 1e-9 * max(1.0, np.abs(b).max())


def test_unit_transmission_gives_g0_times_the_window():
    """T = 1 on a grid covering the window: I = G0 (mu_L - mu_R), at finite and zero temperature."""
    E = np.linspace(-1.0, 1.0, 40001)
    T = np.ones_like(E)
    h = E[1] - E[0]
    for (ml, mr, kT) in ((0.1, -0.1, 0.0259), (0.05, -0.15, 0.01)):
        I = ob.landauer_current(E, T, ml, mr, kT)
        assert abs(I - ob.G0 * (ml - mr)) <= 1e-9 * ob.G0 * abs(ml - mr)
    # at zero temperature the trapezoid rule misses up to h/4 at each step of the window
    I = ob.landauer_current(E, T, 0.2, 0.0, 0.0)
    assert abs(I / ob.G0 - 0.2) <= h / 2 + 1e-15
    assert ob.landauer_current(E, T, 0.1, 0.1, 0.02) == 0.0


def test_fermi_function_limits():
    assert ob.fermi(0.0, 0.0, 0.02) == 0.5
    assert ob.fermi(-50.0, 0.0, 0.02) == 1.0 and ob.fermi(50.0, 0.0, 0.02) == 0.0
    x = np.linspace(-0.3, 0.3, 7)
    assert np.allclose(ob.fermi(x, 0.0, 0.05) + ob.fermi(-x, 0.0, 0.05), 1.0)


def test_current_reverses_for_the_mirrored_reciprocal_device():
    """Real H, S (time-reversal symmetric): I_mirror(V) = -I(-V) under symmetric bias."""
    dev = synth.random_small_device(4, 2, seed=27, real=True, distinct_leads=True)
    E = np.linspace(-3.0, 3.0, 241)
    V, kT = 0.3, 0.02
    T_fw = ob.transmission_bias(dev, E, ETA, -V / 2, V / 2)          # bias -V on dev
    T_mr = ob.transmission_bias(dev.mirrored(), E, ETA, V / 2, -V / 2)  # bias +V on the mirror
    I_fw = ob.landauer_current(E, T_fw, -V / 2, V / 2, kT)
    I_mr = ob.landauer_current(E, T_mr, V / 2, -V / 2, kT)
    assert abs(I_fw) > 1e-8
    assert abs(I_mr + I_fw) <= 1e-8 * abs(I_fw)


def test_linear_response_conductance():
    """Small bias at low temperature: I / V -> G0 T(E_F)."""
    dev = synth.chain_device(8, 0.0, -1.0, 0.0, impurity=(4, 0.6))
    EF, V, kT = 0.3, 2e-4, 2e-5
    E = np.linspace(EF - 2e-3, EF + 2e-3, 801)
    T, I = ob.current(dev, E, 1e-7, EF, V, kT)
    T0 = oracle.transmission(dev, [EF], 1e-7)[0]
    assert abs(I / V - ob.G0 * T0) <= 1e-3 * ob.G0 * T0


# ---- planted mistakes: each must break at least one pin ----

def _pins_hold() -> bool:
    try:
        test_shifted_electrode_equals_energy_shift()
        test_rigid_shift_of_everything_is_a_gauge()
        test_unit_transmission_gives_g0_times_the_window()
        test_fermi_function_limits()
        test_current_reverses_for_the_mirrored_reciprocal_device()
    except AssertionError:
        return False
    return True


def test_pins_hold_for_the_oracle():
    assert _pins_hold()


@pytest.mark.parametrize("name,fn", [
    ("shift sign", lambda lead, mu: type(lead)(lead.H00 - mu * lead.S00, lead.H01 - mu * lead.S01,
                                               lead.S00, lead.S01)),
    ("coupling not shifted", lambda lead, mu: type(lead)(lead.H00 + mu * lead.S00, lead.H01, lead.S00, lead.S01)),
    ("shift without S", lambda lead, mu: type(lead)(lead.H00 + mu * np.eye(lead.M), lead.H01 + mu * lead.S01,
                                                    lead.S00, lead.S01)),
])
def test_planted_shift_mistakes_are_caught(monkeypatch, name, fn):
    monkeypatch.setattr(ob, "shifted_lead", fn)
    assert not _pins_hold(), name


def test_planted_fermi_mistake_is_caught(monkeypatch):
    orig = ob.fermi
    monkeypatch.setattr(ob, "fermi", lambda E, mu, kT: orig(E, mu, 2 * kT) if kT else orig(E, mu, kT))
    assert not _pins_hold()
    monkeypatch.setattr(ob, "fermi", lambda E, mu, kT: 1.0 - orig(E, mu, kT))
    assert not _pins_hold()
