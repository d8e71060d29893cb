"""Pins of the two-temperature reading (Eq 19 for each phase, the suspension
temperature by Eq 33) in the oracle: reduction to one thermal lattice
without particles, the conduction limit, and the diffusion rate of each
thermal lattice against its relaxation time."""
import math

import numpy as np

import oracle


def test_without_particles_it_is_the_single_thermal_lattice():
    """phi0 = 0: the particle thermal lattice has no weight in Eq 33 and the
    fluid's relaxes like the single lattice (same velocity, same tau), so
    f, p and g evolve exactly as with one thermal lattice."""
    kw = dict(nx=20, ny=16, Ra=3e4, phi0=0.0, Pr=0.71, phi_perturb_amp=0.0)
    one = oracle.Oracle(**kw)
    two = oracle.Oracle(thermal_lattices=2, **kw)
    one.step(300)
    two.step(300)
    p1, p2 = one.populations(), two.populations()
    assert p2.shape[0] == 4
    np.testing.assert_allclose(p2[:3], p1, rtol=1e-12, atol=1e-15)
    m2 = two.moments()
    np.testing.assert_allclose(m2["theta"], m2["theta_f"], rtol=0, atol=0)
    assert abs(one.nusselt()[0] - two.nusselt()[0]) < 1e-12


def test_conduction_limit_with_two_thermal_lattices():
    """Ra = 0, no slip forces: both phases conduct to the linear profile
    between the isothermal walls, so theta_f = theta_p = theta_ns is linear
    and Nu = 1."""
    nx, ny = 12, 10
    o = oracle.Oracle(nx=nx, ny=ny, Ra=0.0, phi0=0.03, Pr=0.71, force_mask=0, phi_perturb_amp=0.0,
                      thermal_lattices=2)
    o.step(8000)
    m = o.moments()
    lin = 0.5 - (np.arange(nx) + 0.5) / nx
    for k in ("theta", "theta_f", "theta_p"):
        assert np.abs(m[k] - lin[None, :]).max() < 1e-12, k
    nu_h, nu_c, _ = o.nusselt()
    assert abs(nu_h - 1.0) < 1e-12 and abs(nu_c - 1.0) < 1e-12


def _mode_amplitude(th, nx):
    """Projection of theta - linear profile onto the slowest mode between
    the walls, sin(2 pi (x + 1/2) / nx) (the deviation is odd about the
    centre)."""
    x = np.arange(nx) + 0.5
    dev = th.mean(axis=0) - (0.5 - x / nx)
    s = np.sin(2.0 * np.pi * x / nx)
    return float(dev @ s / (s @ s))


def test_each_thermal_lattice_diffuses_at_its_own_rate():
    """Without flow each thermal lattice is a diffusion equation with
    alpha = (tau - 1/2)/3: the fluid's with the base-fluid diffusivity, the
    particles' with tau_p from Eq 24 (mass-weighted sum of the two
    relaxation times equal to that of the suspension, alpha_ns = alpha_f
    (k/k_f)/((rho c_p)/(rho c_p)_f), Eqs 8 and 10).  The slowest mode of
    the approach to the linear profile decays as exp(-alpha k^2 t),
    k = 2 pi / nx."""
    nx, ny, phi0 = 64, 4, 0.04
    o = oracle.Oracle(nx=nx, ny=ny, Ra=0.0, phi0=phi0, Pr=0.71, force_mask=0, phi_perturb_amp=0.0,
                      thermal_lattices=2)
    d = o.derived()
    t1, t2 = 1500, 3000
    o.step(t1)
    m1 = o.moments(("theta_f", "theta_p"))
    o.step(t2 - t1)
    m2 = o.moments(("theta_f", "theta_p"))
    k2 = (2.0 * np.pi / nx) ** 2
    rate = {f: math.log(_mode_amplitude(m1[f], nx) / _mode_amplitude(m2[f], nx)) / (t2 - t1) / k2
            for f in ("theta_f", "theta_p")}
    alpha_f = d["alpha_L"]
    R = d["R"]
    rbar_p = R * phi0 / (1.0 - phi0 + R * phi0)
    k_ratio = 1.0 + d["Ck"] * phi0 ** 0.764
    rc_ratio = 1.0 + phi0 * (d["rhoc_ratio"] - 1.0)
    alpha_ns = alpha_f * k_ratio / rc_ratio
    tau_f = 3.0 * alpha_f + 0.5
    tau_p = (3.0 * alpha_ns + 0.5 - (1.0 - rbar_p) * tau_f) / rbar_p
    alpha_p = (tau_p - 0.5) / 3.0
    assert alpha_p > 1.05 * alpha_f  # the two rates are distinguishable here
    assert abs(rate["theta_f"] / alpha_f - 1.0) < 0.01, rate
    assert abs(rate["theta_p"] / alpha_p - 1.0) < 0.01, rate
