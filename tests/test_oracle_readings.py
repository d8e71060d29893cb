"""Pins of the alternative readings (reading_flags) in the oracle: each is
checked against a closed form of its own."""
import math

import numpy as np
import pytest

import oracle

LIT_K, LIT_G, COMMON_U = 1, 2, 4


def test_literal_conductivity_ratio_in_the_conduction_limit():
    """Eq 10a as printed, (k_f/k_p)^0.7476: in the conduction limit the
    conductivity-weighted Nu is k_ns/k_f of that form (an enhancement ~3e-5,
    against ~1e-2 with the default reading)."""
    N, phi0 = 12, 0.02
    o = oracle.Oracle(nx=N, ny=N, Ra=0.0, phi0=phi0, Pr=0.71, force_mask=0, phi_perturb_amp=0.0,
                      reading_flags=LIT_K)
    o.step(6000)
    nu_h, _, nu_k = o.nusselt()
    kB, T0, rho_f, mu_f, d_f, k_f, k_p, dp = 1.380649e-23, 300.0, 997.1, 8.9e-4, 0.384e-9, 0.613, 40.0, 100e-9
    Re = rho_f * kB * T0 / (3 * math.pi * mu_f ** 2 * d_f)
    kratio = 1.0 + 64.7 * phi0 ** 0.764 * (d_f / dp) ** 0.369 * (k_f / k_p) ** 0.7476 * 0.71 ** 0.995 * Re ** 1.2321
    assert abs(nu_h - 1.0) < 1e-12
    assert abs(nu_k - kratio) < 1e-12
    assert 1.0 < kratio < 1.0 + 1e-3


def _periodic_momentum(flags, steps):
    o = oracle.Oracle(nx=6, ny=5, Ra=0.0, phi0=0.03, dp_nm=40.0, force_mask=oracle.F_DRAG | oracle.F_GRAV,
                      force_scale=[1, 1, 1, 1, 1, 1e-6], phi_perturb_amp=0.0, boundary=2, reading_flags=flags)
    o.step(steps)
    m = o.moments(("rho_f", "phi", "uy_f", "uy_p"))
    d = o.derived()
    jy = (m["rho_f"] * m["uy_f"] + d["R"] * m["phi"] * m["uy_p"]).sum()
    return jy, d, m


def test_literal_gravity_leaves_the_particle_weight_unbalanced():
    """Periodic box, uniform suspension at rest, gravity and drag on.  With
    the default reading the fluid carries the weight of the uniform
    suspension and the mixture momentum stays zero; with gravity on the
    particles only it grows by -(1 - 1/R) g_L sum(rho_p) per step (simple
    forcing adds exactly F per step, R-6)."""
    steps = 7
    jy_def, _, _ = _periodic_momentum(0, steps)
    jy_lit, d, m = _periodic_momentum(LIT_G, steps)
    rho_p_sum = d["R"] * m["phi"].sum()
    expect = -steps * 1e-6 * (1.0 - 1.0 / d["R"]) * d["grav_L"] * rho_p_sum
    assert abs(jy_def) <= 1e-12 * abs(expect)
    assert abs(jy_lit - expect) <= 1e-9 * abs(expect)


def test_common_velocity_relaxes_the_slip_geometrically():
    """Periodic uniform box, forces off, u_f != u_p: with one common
    equilibrium velocity u_c = (a u_f + b u_p)/(a + b), a = rho_f/tau_f,
    b = rho_p/tau_p, each step multiplies the slip by 1 - (b/tau_f +
    a/tau_p)/(a + b) and keeps the mixture momentum."""
    uf, up = (0.01, -0.004), (-0.002, 0.006)
    o = oracle.Oracle(nx=5, ny=4, Ra=0.0, phi0=0.03, dp_nm=40.0, force_mask=0, phi_perturb_amp=0.0,
                      boundary=2, u_f_init=uf, u_p_init=up, reading_flags=COMMON_U)
    d = o.derived()
    rho_f, rho_p = d["rho_f0"], d["R"] * 0.03
    tau_f = d["tau_f"]
    tau_p = o.node_forces(rho_f=rho_f, rho_p=rho_p)["tau_p"]
    a, b = rho_f / tau_f, rho_p / tau_p
    q = 1.0 - (b / tau_f + a / tau_p) / (a + b)
    j0 = np.array([rho_f * uf[0] + rho_p * up[0], rho_f * uf[1] + rho_p * up[1]])
    w0 = np.array(uf) - np.array(up)
    for n in (1, 4, 9):
        o.step(n - o.time)
        m = o.moments(("ux_f", "uy_f", "ux_p", "uy_p"))
        w = np.array([m["ux_f"].mean() - m["ux_p"].mean(), m["uy_f"].mean() - m["uy_p"].mean()])
        np.testing.assert_allclose(w, w0 * q ** n, rtol=1e-10)
        j = np.array([rho_f * m["ux_f"].mean() + rho_p * m["ux_p"].mean(),
                      rho_f * m["uy_f"].mean() + rho_p * m["uy_p"].mean()])
        np.testing.assert_allclose(j, j0, rtol=1e-12)


def test_unknown_reading_flags_are_refused():
    with pytest.raises(ValueError):
        oracle.Oracle(nx=8, ny=8, reading_flags=8)
