"""Pins of the warm-start oracles (field mapping, equilibrium loader, FP64
network) against closed forms, library routines and brute force."""
import math

import numpy as np
import pytest

import oracle
from oracle import warmstart
from paper_1511_04552_amd import inputs

torch = pytest.importorskip("torch")
from oracle import fno_oracle  # noqa: E402


# ---------------------------------------------------------- field mapping ---

def test_resample_identity_on_equal_grids():
    rng = np.random.default_rng(1)
    F = rng.normal(size=(9, 13, 4)).astype(np.float32)
    out = warmstart.resample(F, 13, 9)
    np.testing.assert_array_equal(out, np.moveaxis(F.astype(np.float64), 2, 0))


def test_resample_reproduces_linear_fields_and_constants():
    """Bilinear interpolation is exact for a + b x + c y away from the
    clamped edge band; constants are exact everywhere."""
    sx, sy, nx, ny = 8, 6, 37, 29
    xs = (np.arange(sx) + 0.5) / sx
    ys = (np.arange(sy) + 0.5) / sy
    F = np.zeros((sy, sx, 4))
    F[:, :, 0] = 0.25 + 2.0 * xs[None, :] - 3.0 * ys[:, None]
    F[:, :, 1] = 1.5
    out = warmstart.resample(F, nx, ny, scale=(1, 2, 1, 1), offset=(0, -1, 0, 0))
    X = (np.arange(nx) + 0.5) / nx
    Y = (np.arange(ny) + 0.5) / ny
    inside = ((X[None, :] >= xs[0]) & (X[None, :] <= xs[-1]) & (Y[:, None] >= ys[0]) & (Y[:, None] <= ys[-1]))
    exact = 0.25 + 2.0 * X[None, :] - 3.0 * Y[:, None]
    assert inside.sum() > 0.5 * nx * ny
    np.testing.assert_allclose(out[0][inside], exact[inside], atol=1e-13)
    np.testing.assert_allclose(out[1], 2.0, atol=1e-15)


def test_renormalize_conserves_inventory_and_handles_empty_fields():
    phi = np.array([[0.02, -0.01], [0.03, 0.0]])
    r = warmstart.renormalize(phi, 0.1)
    assert abs(r.sum() - 0.1) < 1e-16 and (r >= 0).all() and r[0, 1] == 0.0
    np.testing.assert_allclose(r[0, 0] / r[1, 0], 2.0 / 3.0, rtol=1e-15)
    u = warmstart.renormalize(np.full((2, 2), -1.0), 0.2)
    np.testing.assert_allclose(u, 0.05, rtol=1e-15)
    xi = inputs.phi_perturbation(3, 5, 4)
    inv = warmstart.cold_inventory(0.02, 0.5, xi, 20)
    assert abs(inv - np.maximum(0.02 + 0.5 * xi, 0).sum()) < 1e-15


# ---------------------------------------------------- equilibrium loader ---

def test_load_fields_of_cold_state_is_the_cold_start():
    """Loading the cold start's own fields (rest, theta = 0, phi = phi0 + A xi)
    gives back its populations exactly."""
    kw = dict(nx=12, ny=10, Ra=1e4, phi0=0.02, dp_nm=50.0, phi_perturb_amp=0.01)
    xi = inputs.phi_perturbation(5, 12, 10)
    cold = oracle.Oracle(xi=xi, **kw)
    warm = oracle.Oracle(xi=xi, **kw)
    z = np.zeros((10, 12))
    warm.step(3)
    warm.load_fields(z, z, z, np.maximum(0.02 + 0.01 * xi.reshape(10, 12), 0))
    assert warm.time == 0
    np.testing.assert_allclose(warm.populations(), cold.populations(), rtol=1e-15, atol=1e-18)
    cold.step(20)
    warm.step(20)
    np.testing.assert_allclose(warm.populations(), cold.populations(), rtol=1e-13, atol=1e-17)


def test_load_fields_moments_are_the_fields():
    """Eqs 26-27: the moments of the equilibrium state are the loaded fields
    (rho_f~ = 1 - phi0, phi, both phase velocities u, theta)."""
    nx, ny = 9, 7
    rng = np.random.default_rng(2)
    ux, uy = 0.02 * rng.normal(size=(2, ny, nx))
    th = rng.uniform(-0.5, 0.5, (ny, nx))
    phi = rng.uniform(0.0, 0.05, (ny, nx))
    o = oracle.Oracle(nx=nx, ny=ny, Ra=1e4, phi0=0.03, dp_nm=40.0)
    o.load_fields(ux, uy, th, phi)
    m = o.moments()
    np.testing.assert_allclose(m["rho_f"], 1.0 - 0.03, rtol=1e-14)
    np.testing.assert_allclose(m["phi"], phi, rtol=1e-13, atol=1e-18)
    np.testing.assert_allclose(m["theta"], th, rtol=1e-13, atol=1e-16)
    for k in ("ux_f", "ux_p", "ux_ns"):
        np.testing.assert_allclose(m[k], ux, rtol=1e-12, atol=1e-18)
    for k in ("uy_f", "uy_p", "uy_ns"):
        np.testing.assert_allclose(m[k], uy, rtol=1e-12, atol=1e-18)
    rf = 0.97 + 1e-3 * rng.normal(size=(ny, nx))
    o.load_fields(ux, uy, th, phi, rf)
    np.testing.assert_allclose(o.moments("rho_f")["rho_f"], rf, rtol=1e-14)


def test_load_fields_non_equilibrium_parts_are_stress_and_heat_flux():
    """Chapman-Enskog closed forms: with u_x = a y and theta = b x, the
    second moment of f - f_eq at interior nodes is -(tau_f rho_f / 3) a in
    xy (zero on the diagonal), and the first moment of g - g_eq is
    -(tau_theta / 3) b along x, with tau_theta = 3 alpha (k/k_f) / (rho c_p
    ratio) + 1/2 (Eqs 10, 8, 24)."""
    nx, ny = 12, 10
    a, b = 2e-4, 3e-3
    Y, X = np.mgrid[0:ny, 0:nx].astype(float)
    ux, uy = a * Y, np.zeros((ny, nx))
    th = b * X - 0.01
    phi = np.full((ny, nx), 0.02)
    o = oracle.Oracle(nx=nx, ny=ny, Ra=1e5, phi0=0.02, dp_nm=40.0)
    o.load_fields(ux, uy, th, phi)
    d = o.derived()
    e, _ = _d2q9_ew()
    pops = o.populations().reshape(3, 9, ny, nx)
    rf = d["rho_f0"]
    k_ratio = 1.0 + d["Ck"] * 0.02 ** 0.764
    rc_ratio = 1.0 + 0.02 * (d["rhoc_ratio"] - 1.0)
    tau_th = 3.0 * d["alpha_L"] * k_ratio / rc_ratio + 0.5
    for (y, x) in ((3, 4), (5, 7), (8, 1 + 1)):
        feq = oracle.equilibrium(rf, ux[y, x], uy[y, x])
        fneq = pops[0, :, y, x] - feq
        Pi = np.einsum("i,ij,ik->jk", fneq, e, e)
        np.testing.assert_allclose(Pi[0, 1], -d["tau_f"] * rf * a / 3.0, rtol=1e-9)
        assert abs(Pi[0, 0]) < 1e-12 * abs(Pi[0, 1]) + 1e-20 and abs(Pi[1, 1]) < 1e-12 * abs(Pi[0, 1]) + 1e-20
        geq = oracle.equilibrium(th[y, x], ux[y, x], uy[y, x])
        gneq = pops[2, :, y, x] - geq
        q = gneq @ e
        np.testing.assert_allclose(q[0], -tau_th * b / 3.0, rtol=1e-9)
        assert abs(q[1]) < 1e-15
        assert abs(gneq.sum()) < 1e-15 and abs(fneq.sum()) < 1e-15
        np.testing.assert_allclose(pops[1, :, y, x], oracle.equilibrium(d["R"] * 0.02, ux[y, x], uy[y, x]), rtol=1e-14)


def test_fluid_density_conserves_the_fluid_mass():
    dev = np.array([[0.1, -0.3], [0.5, 0.2]])
    r = warmstart.fluid_density(dev, 0.02)
    assert abs(r.sum() - 4 * 0.98) < 1e-15
    np.testing.assert_allclose(np.diff(r.ravel()), np.diff(dev.ravel()), atol=1e-15)


def _d2q9_ew():
    import os
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "d2q9.txt"))
    return rows[:, 1:3], rows[:, 3] / rows[:, 4]


# ------------------------------------------------------- network oracle ---

def _irfft_reference(h, r_full, m):
    """spectral layer with per-mode diagonal complex weights, via numpy's FFT:
    truncate the half spectrum to K_y x {0..m-1}, multiply, invert."""
    S = h.shape[1]
    H = np.fft.rfft2(h, axes=(1, 2))                          # (B, S, S/2+1, C)
    mask = np.zeros(H.shape[1:3], dtype=bool)
    mask[fno_oracle.ky_modes(S, m), :m] = True
    Z = np.where(mask[None, :, :, None], H * r_full[None, :, :, None], 0.0)
    return np.fft.irfft2(Z, s=(S, S), axes=(1, 2))


@pytest.mark.parametrize("S,m", [(8, 2), (12, 3), (16, 8)])
def test_spectral_layer_is_truncated_fft_filter(S, m):
    """With R[ky, kx] = r(ky, kx) times the identity, the spectral layer is the
    real 2-D FFT filter of numpy (closed form of the truncated transform,
    including the mode ordering, the sign of the exponents and the kx > 0
    doubling)."""
    rng = np.random.default_rng(S)
    B, C = 2, 3
    h = rng.normal(size=(B, S, S, C))
    r = rng.normal(size=(2 * m, m)) + 1j * rng.normal(size=(2 * m, m))
    R_re = np.einsum("ab,co->abco", r.real, np.eye(C))
    R_im = np.einsum("ab,co->abco", r.imag, np.eye(C))
    got = fno_oracle.spectral(torch.tensor(h), torch.tensor(R_re), torch.tensor(R_im), m).numpy()
    r_full = np.zeros((S, S // 2 + 1), dtype=complex)
    for a, ky in enumerate(fno_oracle.ky_modes(S, m)):
        r_full[ky, :m] = r[a]
    ref = _irfft_reference(h, r_full, m)
    np.testing.assert_allclose(got, ref, atol=1e-12)


def test_spectral_layer_mixes_channels_per_mode():
    """A real channel permutation R (same for all modes) permutes the
    filtered channels."""
    rng = np.random.default_rng(4)
    S, m, B, C = 8, 3, 1, 4
    h = rng.normal(size=(B, S, S, C))
    perm = np.array([2, 0, 3, 1])
    P = np.eye(C)[perm].T                       # h @ P moves channel perm[o] to o
    R_re = np.broadcast_to(P, (2 * m, m, C, C)).copy()
    got = fno_oracle.spectral(torch.tensor(h), torch.tensor(R_re), torch.zeros(2 * m, m, C, C, dtype=torch.float64), m).numpy()
    r_full = np.zeros((S, S // 2 + 1), dtype=complex)
    r_full[fno_oracle.ky_modes(S, m), :m] = 1.0
    ref = _irfft_reference(h, r_full, m)[..., perm]
    np.testing.assert_allclose(got, ref, atol=1e-12)


def _tiny_params(rng, C=3, m=2, L=2, Q=5):
    p = {"W_lift": rng.normal(size=(5, C)), "b_lift": rng.normal(size=C)}
    for l in range(L):
        p[f"R_re_{l}"] = 0.3 * rng.normal(size=(2 * m, m, C, C))
        p[f"R_im_{l}"] = 0.3 * rng.normal(size=(2 * m, m, C, C))
        p[f"W_{l}"] = rng.normal(size=(C, C))
        p[f"b_{l}"] = rng.normal(size=C)
    p["P1"] = rng.normal(size=(C, Q))
    p["c1"] = rng.normal(size=Q)
    p["P2"] = rng.normal(size=(Q, 4))
    p["c2"] = rng.normal(size=4)
    return {k: torch.tensor(v) for k, v in p.items()}


def test_network_gradients_match_finite_differences():
    """Brute force: central differences of the loss in every parameter of a
    tiny network."""
    rng = np.random.default_rng(7)
    S, m = 6, 2
    params = _tiny_params(rng)
    a = torch.tensor(rng.normal(size=(2, S, S, 5)))
    t = torch.tensor(rng.normal(size=(2, S, S, 4)))
    _, loss, grads = fno_oracle.loss_and_grads(params, a, t, m)
    eps = 1e-6
    for k, v in params.items():
        flat = v.reshape(-1)
        for idx in rng.choice(flat.numel(), size=min(4, flat.numel()), replace=False):
            old = float(flat[idx])
            flat[idx] = old + eps
            lp = float(((fno_oracle.forward(params, a, m) - t) ** 2).mean())
            flat[idx] = old - eps
            lm = float(((fno_oracle.forward(params, a, m) - t) ** 2).mean())
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            g = float(grads[k].reshape(-1)[idx])
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)), (k, idx, fd, g)


def test_gelu_definition_points():
    x = torch.tensor([0.0, 1.0, -1.0, 8.0, -8.0], dtype=torch.float64)
    g = fno_oracle.gelu(x)
    # Phi(1) = 0.841344746068543 (standard normal CDF)
    np.testing.assert_allclose(g.numpy(), [0.0, 0.841344746068543, -0.158655253931457, 8.0, 0.0], atol=1e-12)
