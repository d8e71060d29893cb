"""Pins of the oracle's slip-force terms that direction and scaling checks
alone leave open.

- Magnus and particle rotation (Table 1, merged into one force under the
  reading that takes the Magnus mass rate from Table 2's time scale
  tau_M = d_p / v_M): the Magnus part is split from the rotation part by
  projecting on the slip and on the slip rotated by +90 degrees.
- Drag (Table 1): the Schiller-Naumann drag coefficient
  C_d = 24 (1 + 0.15 Re_d^0.687) / Re_d, i.e. beta / beta_Stokes - 1 =
  0.15 Re_d^0.687, fixed by its value at Re_d = 1 and its log-log slope.
- Thermophoresis (Table 1): the coefficient's dependence on k* = k_ns / k_p
  in the continuum limit (Kn -> 0), where it is proportional to
  k* / (1 + 2 k*), and on Kn in the free-molecular limit (Kn -> infinity),
  where it falls as 1/Kn independently of k*.

Every check is a property of the printed expressions (a limit, a ratio, a
slope, a time scale of Table 2), evaluated on single nodes through
``node_forces``, so a dropped term, a wrong sign, a doubled rate or a
changed exponent in the oracle fails one of them.
"""
import math

import numpy as np

import oracle

MU_F, RHO_F_SI, RHO_P_SI = 8.9e-4, 997.1, 3970.0


def _cavity(dp_nm=50.0, **kw):
    return oracle.Oracle(nx=32, ny=32, Ra=1e5, phi0=0.03, dp_nm=dp_nm, **kw)


def _slip_state(o, uf, up, rho_f=0.97, rho_p=None, **extra):
    d = o.derived()
    if rho_p is None:
        rho_p = d["R"] * 0.03
    return o.node_forces(rho_f=rho_f, rho_p=rho_p,
                         jx_f=rho_f * uf[0], jy_f=rho_f * uf[1],
                         jx_p=rho_p * up[0], jy_p=rho_p * up[1], **extra)


def _split_magnus_rotation(r, uf, up):
    """Return (component along the slip w = u_f - u_p, component along w
    rotated by +90 degrees) of the Magnus/rotation acceleration."""
    w = np.asarray(uf, float) - np.asarray(up, float)
    wh = w / np.linalg.norm(w)
    wp = np.array([-wh[1], wh[0]])
    a = np.array([r["aMRx"], r["aMRy"]])
    return float(a @ wh), float(a @ wp)


def _si(o):
    d = o.derived()
    return d["dx"] / d["dt"], d["dx"] / d["dt"] ** 2, d  # velocity, acceleration


# ----------------------------------------------------------------- Magnus ---

def test_magnus_opposes_slip_at_table2_rate():
    """Magnus row of Table 1, F_M = mdot_p (v_p - v_M) with v_M the mean of
    the two phase velocities: v_p - v_M = -(v_f - v_p)/2, so the force is
    antiparallel to the slip.  Its rate per particle mass is 1/tau_M =
    v_M / d_p, the Magnus time scale of Table 2."""
    o = _cavity()
    vel, acc, d = _si(o)
    dp = 50e-9
    for uf, up in (((3e-3, 1e-3), (2.9e-3, 1.05e-3)),
                   ((-1e-2, 4e-3), (-1.02e-2, 4.1e-3)),
                   ((2e-4, -7e-4), (2.2e-4, -6.9e-4))):
        r = _slip_state(o, uf, up)
        a_m, _ = _split_magnus_rotation(r, uf, up)
        assert a_m < 0.0, (uf, up, a_m)
        vm = 0.5 * (np.asarray(uf) + np.asarray(up)) * vel          # m/s
        rel = np.linalg.norm(np.asarray(up) * vel - vm)             # |v_p - v_M|
        rate = abs(a_m) * acc / rel                                 # 1/s
        tau_m = dp / np.linalg.norm(vm)                             # Table 2
        assert abs(rate * tau_m - 1.0) < 1e-10, (rate, 1 / tau_m)


def test_magnus_scaling_laws():
    """|a_M| is linear in |v_M| at fixed slip, linear in the slip at fixed
    v_M, and falls as 1/d_p at fixed SI velocities."""
    o = _cavity()

    def am(vm, w, oo=o):
        vm, w = np.asarray(vm), np.asarray(w)
        uf, up = vm + w / 2, vm - w / 2
        return _split_magnus_rotation(_slip_state(oo, uf, up), uf, up)[0]

    vm, w = np.array([2e-3, -1e-3]), np.array([1e-5, 3e-5])
    base = am(vm, w)
    assert abs(am(2 * vm, w) / base - 2.0) < 1e-9
    assert abs(am(vm, 3 * w) / base - 3.0) < 1e-9
    o2 = _cavity(dp_nm=100.0)
    assert abs(o2.derived()["dx"] - o.derived()["dx"]) == 0.0  # lattice set by Ra only
    assert abs(am(vm, w, o2) / base - 0.5) < 1e-9


# --------------------------------------------------------------- rotation ---

def test_rotation_term_direction_scaling_and_table2_scale():
    """Rotation row of Table 1 times the particle area: along the slip
    rotated by +90 degrees, linear in the shear rate 8 |v_p| / H,
    independent of the slip magnitude, 1/d_p at fixed SI velocities, and
    with a_R tau_R = 6 gdot d_p, tau_R = rho_ns d_p^2 / mu_ns of Table 2
    (6 = A_p d_p / V_p for a sphere)."""
    o = _cavity()
    vel, acc, d = _si(o)
    R = d["R"]
    rho_p = R * 0.03

    def ar(up, w, oo=o):
        up, w = np.asarray(up), np.asarray(w)
        uf = up + w
        r = _slip_state(oo, uf, up, rho_p=rho_p)
        return _split_magnus_rotation(r, uf, up), r

    up, w = np.array([4e-3, 1e-3]), np.array([-2e-5, 1e-5])
    (a_m, a_r), r = ar(up, w)
    assert a_r > 0.0
    assert abs(ar(2 * up, w)[0][1] / a_r - 2.0) < 1e-9
    assert abs(ar(up, 5 * w)[0][1] / a_r - 1.0) < 1e-9
    assert abs(ar(up, _rot90(w))[0][1] / a_r - 1.0) < 1e-9
    assert abs(ar(up, w, _cavity(dp_nm=25.0))[0][1] / a_r - 2.0) < 1e-9
    # absolute scale against Table 2's rotation time
    phi = rho_p / R
    mu_ns = MU_F * r["r_mu"]
    rho_ns = RHO_F_SI * (1.0 + phi * (R - 1.0))                    # Eq 7
    gdot = 8.0 * np.linalg.norm(up) * vel / d["H"]
    dp = 50e-9
    tau_r = rho_ns * dp ** 2 / mu_ns
    assert abs(a_r * acc * tau_r / (gdot * dp) - 6.0) < 1e-9


def _rot90(v):
    return np.array([-v[1], v[0]])


# ------------------------------------------------------------------- drag ---

def _drag_ratio(o, re_d, direction=(0.6, -0.8)):
    """beta / beta_Stokes at particle Reynolds number re_d."""
    vel, _, d = _si(o)
    r0 = o.node_forces(rho_f=0.97, rho_p=d["R"] * 0.03)
    mu_ns = MU_F * r0["r_mu"]
    dp = 50e-9
    w_si = re_d * mu_ns / (RHO_P_SI * dp)
    uf = np.asarray(direction) * w_si / vel
    r = _slip_state(o, uf, (0.0, 0.0))
    beta_stokes = 18.0 * mu_ns / (RHO_P_SI * dp ** 2)
    return r["beta_L"] / d["dt"] / beta_stokes


def test_schiller_naumann_correction_value_and_slope():
    """Drag row of Table 1: beta = 18 mu C_d Re_d / (24 rho_p d_p^2) with
    C_d = 24 (1 + 0.15 Re_d^0.687) / Re_d.  At Re_d = 1 the correction over
    Stokes drag is exactly 0.15; between Re_d = 1/4 and 4 the correction
    grows with log-log slope 0.687; it is independent of the slip's
    direction."""
    o = _cavity()
    assert abs(_drag_ratio(o, 1.0) - 1.15) < 1e-10
    c_lo = _drag_ratio(o, 0.25) - 1.0
    c_hi = _drag_ratio(o, 4.0) - 1.0
    slope = math.log(c_hi / c_lo) / math.log(16.0)
    assert abs(slope - 0.687) < 1e-9, slope
    assert abs(_drag_ratio(o, 2.0, direction=(-1.0, 0.0)) / _drag_ratio(o, 2.0) - 1.0) < 1e-12


# --------------------------------------------------------- thermophoresis ---

def _a_t(o, rho_p=1e-9):
    r = o.node_forces(rho_f=0.97, rho_p=rho_p, theta=0.1, dth_dx=-0.02, dth_dy=0.005)
    return np.array([r["aTx"], r["aTy"]]), r


def _k_star(r, k_p, k_f=0.613):
    return k_f * r["r_k"] / k_p


def test_thermophoresis_continuum_limit_k_star_dependence():
    """Thermophoresis row of Table 1 at Kn -> 0 (mean free path 1e-18 m, so
    Kn = 2e-11): the coefficient reduces to 6 pi C_S k* / (1 + 2 k*), so the
    ratio of the accelerations for two particle conductivities is
    [k1*/(1 + 2 k1*)] / [k2*/(1 + 2 k2*)], with k* = k_ns / k_p.  A nearly
    empty particle phase keeps k_ns close to k_f; k_ns is read per node."""
    fluid = {"d_mol": 1e-18}
    ratios = []
    for k_p1, k_p2 in ((40.0, 0.4), (40.0, 4.0), (2.0, 0.2)):
        o1 = _cavity(fluid=fluid, particle={"k": k_p1})
        o2 = _cavity(fluid=fluid, particle={"k": k_p2})
        a1, r1 = _a_t(o1)
        a2, r2 = _a_t(o2)
        k1, k2 = _k_star(r1, k_p1), _k_star(r2, k_p2)
        expect = (k1 / (1 + 2 * k1)) / (k2 / (1 + 2 * k2))
        got = a1[0] / a2[0]
        assert abs(a1[1] / a2[1] - got) < 1e-12 * abs(got)
        assert abs(got / expect - 1.0) < 1e-8, (k_p1, k_p2, got, expect)
        ratios.append(got)
    assert ratios[0] < 0.2  # the k* dependence is strong, not a constant


def test_thermophoresis_free_molecular_limit():
    """At Kn -> infinity the coefficient of Table 1 falls as
    6 pi C_S / (6 C_m Kn), independent of k*: Kn times the acceleration
    converges, is the same for two particle conductivities, and relates to
    the continuum value (same k_p) by (1 + 2 k0*) / (6 C_m k0*), with
    C_m = 1.14 as printed."""
    dp = 50e-9
    k_p = 4.0
    lam_hi = [1e4 * dp, 1e6 * dp]
    kn_a = []
    for lam in lam_hi:
        o = _cavity(fluid={"d_mol": lam}, particle={"k": k_p})
        kn_a.append(_a_t(o)[0][0] * lam / dp)
    assert abs(kn_a[0] / kn_a[1] - 1.0) < 1e-3
    o_other = _cavity(fluid={"d_mol": lam_hi[1]}, particle={"k": 400.0})
    assert abs(_a_t(o_other)[0][0] * lam_hi[1] / dp / kn_a[1] - 1.0) < 1e-5
    o0 = _cavity(fluid={"d_mol": 1e-18}, particle={"k": k_p})
    a0, r0 = _a_t(o0)
    k0 = _k_star(r0, k_p)
    expect = (1 + 2 * k0) / (6 * 1.14 * k0)
    assert abs(kn_a[1] / a0[0] / expect - 1.0) < 1e-5, (kn_a[1] / a0[0], expect)
