"""FP64 CPU oracle of the three-lattice MCLBM step (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The HIP product path
never imports, loads or calls it, and the two share no code: the oracle is a
plain C file (``mclbm_oracle.c``) written from the paper's Section 2.d, Table 1
and Eqs 7-36 with its own constants and setup derivation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mclbm_oracle.c")
_SO = os.path.join(_HERE, "libmclbm_oracle.so")

FIELDS = ("rho_f", "ux_f", "uy_f", "phi", "ux_p", "uy_p", "theta", "ux_ns", "uy_ns", "theta_f", "theta_p")
FIELD_BIT = {name: 1 << i for i, name in enumerate(FIELDS)}

F_DRAG, F_BROWN, F_THERMO, F_SAFF, F_MAGROT, F_GRAV = 1, 2, 4, 8, 16, 32
F_ALL = 63
CAVITY, CHANNEL, PERIODIC = 0, 1, 2

DERIVED = ("nu_L", "alpha_L", "H", "dx", "dt", "G_L", "grav_L", "Ck", "R", "tau_f",
           "rhoc_ratio", "beta_ratio", "rho_f0", "rho_p0", "nu_f", "alpha_f")
NODE_IN = ("rho_f", "jx_f", "jy_f", "rho_p", "jx_p", "jy_p", "theta",
           "dphi_dx", "dphi_dy", "dth_dx", "dth_dy")
NODE_OUT = ("Ffx", "Ffy", "Fpx", "Fpy", "tau_p", "tau_th", "aBx", "aBy", "aTx", "aTy",
            "aSx", "aSy", "aMRx", "aMRy", "aGx", "aGy", "Dx", "Dy", "beta_L", "kappa",
            "r_k", "r_mu")


def build() -> str:
    """Compile the oracle with gcc (plain IEEE FP64: no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", _SO + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


class Material(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("rho", "cp", "k", "beta", "mu", "d_mol")]


class Config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("Ra", ctypes.c_double), ("Pr", ctypes.c_double),
        ("phi0", ctypes.c_double), ("dp", ctypes.c_double),
        ("tau_f", ctypes.c_double),
        ("dT", ctypes.c_double), ("T0", ctypes.c_double),
        ("force_mask", ctypes.c_uint32),
        ("force_scale", ctypes.c_double * 6),
        ("phi_perturb_amp", ctypes.c_double),
        ("fluid", Material), ("particle", Material),
        ("boundary", ctypes.c_int32),
        ("body_force", ctypes.c_double * 2),
        ("u_f_init", ctypes.c_double * 2), ("u_p_init", ctypes.c_double * 2),
        ("thermal_lattices", ctypes.c_int32),
        ("reading_flags", ctypes.c_uint32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        D = ctypes.POINTER(ctypes.c_double)
        L.mclbm_oracle_config_defaults.argtypes = [ctypes.POINTER(Config)]
        L.mclbm_oracle_config_defaults.restype = None
        L.mclbm_oracle_create.argtypes = [ctypes.POINTER(Config), D, ctypes.POINTER(P)]
        L.mclbm_oracle_step.argtypes = [P, ctypes.c_int64]
        L.mclbm_oracle_time.argtypes = [P]
        L.mclbm_oracle_time.restype = ctypes.c_int64
        L.mclbm_oracle_read_moments.argtypes = [P, ctypes.c_uint32, D, ctypes.c_size_t]
        L.mclbm_oracle_read_populations.argtypes = [P, D, ctypes.c_size_t]
        L.mclbm_oracle_write_populations.argtypes = [P, D, ctypes.c_size_t]
        L.mclbm_oracle_checkpoint.argtypes = [P, ctypes.c_char_p]
        L.mclbm_oracle_restore.argtypes = [P, ctypes.c_char_p]
        L.mclbm_oracle_nusselt.argtypes = [P, D, D, D]
        L.mclbm_oracle_residual.argtypes = [P, D, D]
        L.mclbm_oracle_derived.argtypes = [P, D, ctypes.c_int]
        L.mclbm_oracle_equilibrium.argtypes = [ctypes.c_double] * 3 + [D]
        L.mclbm_oracle_equilibrium.restype = None
        L.mclbm_oracle_forcing.argtypes = [ctypes.c_double] * 2 + [D]
        L.mclbm_oracle_forcing.restype = None
        L.mclbm_oracle_node_forces.argtypes = [P, D, D]
        L.mclbm_oracle_load_fields.argtypes = [P, D, D, D, D, D]
        L.mclbm_oracle_destroy.argtypes = [P]
        L.mclbm_oracle_destroy.restype = None
        L.mclbm_oracle_set_threads.argtypes = [ctypes.c_int]
        L.mclbm_oracle_set_threads.restype = None
        L.mclbm_oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def equilibrium(a: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().mclbm_oracle_equilibrium(a, ux, uy, _dptr(out))
    return out


def forcing(Fx: float, Fy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().mclbm_oracle_forcing(Fx, Fy, _dptr(out))
    return out


def set_threads(n: int) -> None:
    lib().mclbm_oracle_set_threads(int(n))


def max_threads() -> int:
    return int(lib().mclbm_oracle_max_threads())


def make_config(**kw) -> Config:
    c = Config()
    lib().mclbm_oracle_config_defaults(ctypes.byref(c))
    for key, val in kw.items():
        if key in ("force_scale", "body_force", "u_f_init", "u_p_init"):
            arr = getattr(c, key)
            for i, v in enumerate(val):
                arr[i] = float(v)
        elif key in ("fluid", "particle"):
            m = getattr(c, key)
            for mk, mv in val.items():
                setattr(m, mk, float(mv))
        elif key == "dp_nm":
            c.dp = float(val) * 1e-9
        else:
            if not hasattr(c, key):
                raise KeyError(key)
            setattr(c, key, val)
    return c


class Oracle:
    """One cavity (or test channel / periodic box) on the FP64 oracle."""

    def __init__(self, xi: np.ndarray | None = None, **kw):
        self.cfg = make_config(**kw)
        self.nx, self.ny = int(self.cfg.nx), int(self.cfg.ny)
        self._h = ctypes.c_void_p()
        xp = None
        if xi is not None:
            self._xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(-1)
            if self._xi.size != self.nx * self.ny:
                raise ValueError("xi must hold nx*ny values")
            xp = _dptr(self._xi)
        rc = lib().mclbm_oracle_create(ctypes.byref(self.cfg), xp, ctypes.byref(self._h))
        if rc != 0:
            raise ValueError(f"mclbm_oracle_create failed: {rc}")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            try:
                _lib.mclbm_oracle_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def time(self) -> int:
        return int(lib().mclbm_oracle_time(self._h))

    def step(self, n: int) -> None:
        rc = lib().mclbm_oracle_step(self._h, int(n))
        if rc != 0:
            raise RuntimeError(f"oracle step failed: {rc}")

    def load_fields(self, ux, uy, theta, phi, rho_f=None) -> None:
        """Warm start: equilibrium populations of the given (ny, nx) fields
        (mixture velocity, temperature, particle volume fraction and,
        optionally, the fluid partial density); t = 0."""
        arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in (ux, uy, theta, phi)]
        if rho_f is not None:
            arrs.append(np.ascontiguousarray(rho_f, dtype=np.float64).reshape(-1))
        if any(a.size != self.nx * self.ny for a in arrs):
            raise ValueError("fields must hold nx*ny values")
        ptrs = [_dptr(a) for a in arrs] + ([None] if rho_f is None else [])
        rc = lib().mclbm_oracle_load_fields(self._h, *ptrs)
        if rc != 0:
            raise RuntimeError(f"load_fields failed: {rc}")

    def moments(self, names=FIELDS) -> dict:
        if isinstance(names, str):
            names = (names,)
        mask = 0
        for n in names:
            mask |= FIELD_BIT[n]
        order = [n for n in FIELDS if mask & FIELD_BIT[n]]
        out = np.zeros(len(order) * self.nx * self.ny)
        rc = lib().mclbm_oracle_read_moments(self._h, mask, _dptr(out), out.size)
        if rc != 0:
            raise RuntimeError(f"read_moments failed: {rc}")
        out = out.reshape(len(order), self.ny, self.nx)
        return {n: out[k] for k, n in enumerate(order)}

    def checkpoint(self, path) -> None:
        rc = lib().mclbm_oracle_checkpoint(self._h, str(path).encode())
        if rc != 0:
            raise RuntimeError(f"checkpoint failed: {rc}")

    def restore(self, path) -> None:
        rc = lib().mclbm_oracle_restore(self._h, str(path).encode())
        if rc != 0:
            raise ValueError(f"restore failed: {rc}")

    def write_populations(self, pops: np.ndarray) -> None:
        a = np.ascontiguousarray(pops, dtype=np.float64).reshape(-1)
        rc = lib().mclbm_oracle_write_populations(self._h, _dptr(a), a.size)
        if rc != 0:
            raise RuntimeError(f"write_populations failed: {rc}")

    def populations(self) -> np.ndarray:
        nl = 4 if self.cfg.thermal_lattices == 2 else 3
        out = np.zeros(9 * nl * self.nx * self.ny)
        rc = lib().mclbm_oracle_read_populations(self._h, _dptr(out), out.size)
        if rc != 0:
            raise RuntimeError(f"read_populations failed: {rc}")
        return out.reshape(nl, 9, self.ny, self.nx)

    def nusselt(self) -> tuple:
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        rc = lib().mclbm_oracle_nusselt(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        if rc not in (0, -4):
            raise RuntimeError(f"nusselt failed: {rc}")
        return a.value, b.value, c.value

    def residual(self) -> tuple:
        a, b = ctypes.c_double(), ctypes.c_double()
        lib().mclbm_oracle_residual(self._h, ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value

    def derived(self) -> dict:
        out = np.zeros(len(DERIVED))
        rc = lib().mclbm_oracle_derived(self._h, _dptr(out), out.size)
        if rc != 0:
            raise RuntimeError("derived failed")
        return dict(zip(DERIVED, out.tolist()))

    def node_forces(self, **inputs) -> dict:
        vin = np.array([float(inputs.get(k, 0.0)) for k in NODE_IN])
        for k in inputs:
            if k not in NODE_IN:
                raise KeyError(k)
        vout = np.zeros(len(NODE_OUT))
        lib().mclbm_oracle_node_forces(self._h, _dptr(vin), _dptr(vout))
        return dict(zip(NODE_OUT, vout.tolist()))
