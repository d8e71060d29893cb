"""MI355X-native multi-component lattice Boltzmann (MCLBM) cavity solver.

Thin ctypes binding of ``libmclbm.so`` (C ABI in ``include/mclbm.h``): three
coupled D2Q9 lattices (base fluid, nanoparticle phase, temperature) for
buoyancy-driven flow of a nanosuspension in a differentially heated cavity
(Section 2.d of arXiv:1511.04552).  Every step of the method runs in the HIP
kernels of the library; this module only marshals arguments.  PyTorch provides
the device memory and the stream.  There is no CPU fallback: without the
built library (``python -m paper_1511_04552_amd.build``) every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MCLBM_LIBRARY may point at another build of the same C ABI.
LIB_PATH = os.environ.get("MCLBM_LIBRARY") or os.path.join(_HERE, "libmclbm.so")

# Interface constants of include/mclbm.h.
OK, EINVAL, ENOMEM, EHIP, EDIVERGED, ESTATE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
FP32S, FP16S, BF16S = 0, 1, 2
F_DRAG, F_BROWN, F_THERMO, F_SAFF, F_MAGROT, F_GRAV = 1, 2, 4, 8, 16, 32
F_ALL = 63
R_LITERAL_K_RATIO, R_LITERAL_GRAVITY, R_COMMON_VELOCITY, R_GUO_FORCING, R_LITERAL_REACTIONS = 1, 2, 4, 8, 16
FIELDS = ("rho_f", "ux_f", "uy_f", "phi", "ux_p", "uy_p", "theta", "ux_ns", "uy_ns", "theta_f", "theta_p")
FIELD_BIT = {name: 1 << i for i, name in enumerate(FIELDS)}
DERIVED = ("nu_L", "alpha_L", "H", "dx", "dt", "G_L", "grav_L", "Ck", "R", "tau_f",
           "rhoc_ratio", "beta_ratio", "rho_f0", "rho_p0", "nu_f", "alpha_f")
EXPORTED = ("mclbm_config_defaults", "mclbm_device_bytes", "mclbm_derive_constants", "mclbm_create",
            "mclbm_set_properties", "mclbm_reset", "mclbm_load_fields", "mclbm_copy_state", "mclbm_step",
            "mclbm_time", "mclbm_record_nusselt", "mclbm_nusselt_records",
            "mclbm_export_moments", "mclbm_read_moments", "mclbm_read_populations",
            "mclbm_export_populations", "mclbm_nusselt", "mclbm_residual", "mclbm_residual_noalloc",
            "mclbm_derived", "mclbm_checkpoint", "mclbm_restore", "mclbm_checkpoint_info", "mclbm_destroy", "mclbm_last_error",
            "mclbm_copy_kernel",
            "mclbm_version", "mclbm_abi_version",
            "mclbm_batch_device_bytes", "mclbm_batch_create", "mclbm_batch_step",
            "mclbm_batch_set_graph_steps", "mclbm_batch_set_active", "mclbm_batch_residual",
            "mclbm_batch_nusselt", "mclbm_batch_autotune", "mclbm_batch_tile_shape",
            "mclbm_batch_set_per_cavity", "mclbm_batch_per_cavity",
            "mclbm_batch_reset", "mclbm_batch_size", "mclbm_batch_time", "mclbm_batch_cavity",
            "mclbm_batch_destroy",
            "mclbm_nn_gemm", "mclbm_nn_bias_act", "mclbm_nn_act_backward", "mclbm_nn_colsum_scratch",
            "mclbm_nn_colsum", "mclbm_nn_mse_scratch", "mclbm_nn_mse", "mclbm_nn_adamw")


class MclbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mclbm error {code}: {msg}")
        self.code = code


class Material(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("rho", "cp", "k", "beta", "mu", "d_mol")]


class Config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("Ra", ctypes.c_double), ("Pr", ctypes.c_double),
        ("phi0", ctypes.c_double), ("dp_m", ctypes.c_double),
        ("tau_f", ctypes.c_double),
        ("dT_K", ctypes.c_double), ("T0_K", ctypes.c_double),
        ("force_mask", ctypes.c_uint32),
        ("force_scale", ctypes.c_double * 6),
        ("phi_perturb_amp", ctypes.c_double),
        ("fluid", Material), ("particle", Material),
        ("storage", ctypes.c_int32),
        ("block_x", ctypes.c_int32), ("block_y", ctypes.c_int32),
        ("reading_flags", ctypes.c_uint32),
        ("thermal_lattices", ctypes.c_int32),
        ("steps_per_launch", ctypes.c_int32),
    ]


_lib = None


def lib(load_torch: bool = True):
    """Load ``libmclbm.so`` (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if load_torch:
        import torch  # noqa: F401  (shares libamdhip64 with the library)
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_1511_04552_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, D, I = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    CP = ctypes.POINTER(Config)
    L.mclbm_config_defaults.argtypes = [CP]
    L.mclbm_config_defaults.restype = None
    L.mclbm_device_bytes.argtypes = [CP]
    L.mclbm_device_bytes.restype = ctypes.c_size_t
    L.mclbm_derive_constants.argtypes = [CP, D, I]
    L.mclbm_create.argtypes = [CP, D, P, ctypes.c_size_t, P, ctypes.POINTER(P)]
    L.mclbm_set_properties.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    L.mclbm_reset.argtypes = [P]
    L.mclbm_checkpoint.argtypes = [P, ctypes.c_char_p]
    L.mclbm_restore.argtypes = [P, ctypes.c_char_p]
    L.mclbm_checkpoint_info.argtypes = [ctypes.c_char_p, CP, ctypes.POINTER(ctypes.c_int64), D,
                                        ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    L.mclbm_load_fields.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, D]
    L.mclbm_step.argtypes = [P, ctypes.c_int64]
    L.mclbm_copy_state.argtypes = [P, P]
    L.mclbm_record_nusselt.argtypes = [P, ctypes.c_int32, P, ctypes.c_int32]
    L.mclbm_nusselt_records.argtypes = [P]
    L.mclbm_nusselt_records.restype = ctypes.c_int64
    L.mclbm_time.argtypes = [P]
    L.mclbm_time.restype = ctypes.c_int64
    L.mclbm_export_moments.argtypes = [P, ctypes.c_uint32, P, ctypes.c_size_t]
    L.mclbm_read_moments.argtypes = [P, ctypes.c_uint32, D, ctypes.c_size_t]
    L.mclbm_read_populations.argtypes = [P, D, ctypes.c_size_t]
    L.mclbm_export_populations.argtypes = [P, P, ctypes.c_size_t]
    L.mclbm_nusselt.argtypes = [P, D, D, D]
    L.mclbm_residual.argtypes = [P, D, D]
    L.mclbm_residual_noalloc.argtypes = [P, P]
    L.mclbm_derived.argtypes = [P, D, I]
    L.mclbm_destroy.argtypes = [P]
    L.mclbm_last_error.restype = ctypes.c_char_p
    L.mclbm_copy_kernel.argtypes = [P, P, ctypes.c_size_t, P]
    L.mclbm_version.restype = ctypes.c_char_p
    L.mclbm_abi_version.restype = I
    I32P = ctypes.POINTER(ctypes.c_int32)
    L.mclbm_batch_device_bytes.argtypes = [CP, ctypes.c_int32]
    L.mclbm_batch_device_bytes.restype = ctypes.c_size_t
    L.mclbm_batch_create.argtypes = [CP, ctypes.c_int32, ctypes.POINTER(D), P, ctypes.c_size_t, P,
                                     ctypes.POINTER(P)]
    L.mclbm_batch_step.argtypes = [P, ctypes.c_int64]
    L.mclbm_batch_set_graph_steps.argtypes = [P, ctypes.c_int32]
    L.mclbm_batch_set_active.argtypes = [P, I32P]
    L.mclbm_batch_residual.argtypes = [P, ctypes.c_double, D, I32P]
    L.mclbm_batch_nusselt.argtypes = [P, D]
    L.mclbm_batch_autotune.argtypes = [P, ctypes.c_int32]
    L.mclbm_batch_tile_shape.argtypes = [P, ctypes.c_int32, I32P, I32P]
    L.mclbm_batch_set_per_cavity.argtypes = [P, ctypes.c_int32]
    L.mclbm_batch_per_cavity.argtypes = [P]
    L.mclbm_batch_per_cavity.restype = ctypes.c_int32
    L.mclbm_batch_reset.argtypes = [P]
    L.mclbm_batch_size.argtypes = [P]
    L.mclbm_batch_size.restype = ctypes.c_int32
    L.mclbm_batch_time.argtypes = [P, ctypes.c_int32]
    L.mclbm_batch_time.restype = ctypes.c_int64
    L.mclbm_batch_cavity.argtypes = [P, ctypes.c_int32]
    L.mclbm_batch_cavity.restype = P
    L.mclbm_batch_destroy.argtypes = [P]
    i64, i32, f32 = ctypes.c_int64, ctypes.c_int32, ctypes.c_float
    L.mclbm_nn_gemm.argtypes = [i32, i32, i32, i32, i32, f32, P, i64, i64, i64, P, i64, i64, i64,
                                f32, P, i64, i64, i64, i32, i32, P]
    L.mclbm_nn_bias_act.argtypes = [P, P, i64, i32, i32, P, P]
    L.mclbm_nn_act_backward.argtypes = [P, P, i64, i32, P]
    L.mclbm_nn_colsum_scratch.argtypes = [i64, i32]
    L.mclbm_nn_colsum_scratch.restype = i64
    L.mclbm_nn_colsum.argtypes = [P, P, i64, i32, f32, P, P]
    L.mclbm_nn_mse_scratch.argtypes = [i64]
    L.mclbm_nn_mse_scratch.restype = i64
    L.mclbm_nn_mse.argtypes = [P, P, P, i64, P, P, P]
    L.mclbm_nn_adamw.argtypes = [P, P, P, P, i64, f32, f32, f32, f32, f32, i32, P]
    _lib = L
    return L


def _check(rc: int) -> int:
    if rc != 0:
        raise MclbmError(rc, lib().mclbm_last_error().decode())
    return rc


def make_config(**kw) -> Config:
    """Config with the library defaults, overridden by keyword arguments
    (``dp_nm`` is accepted for the particle diameter in nanometres)."""
    c = Config()
    lib().mclbm_config_defaults(ctypes.byref(c))
    for key, val in kw.items():
        if key == "force_scale":
            for i, v in enumerate(val):
                c.force_scale[i] = float(v)
        elif key in ("fluid", "particle"):
            m = getattr(c, key)
            for mk, mv in val.items():
                setattr(m, mk, float(mv))
        elif key == "dp_nm":
            c.dp_m = float(val) * 1e-9
        elif key == "seed":
            continue
        else:
            if not hasattr(c, key):
                raise KeyError(key)
            setattr(c, key, val)
    return c


def device_bytes(**kw) -> int:
    n = lib().mclbm_device_bytes(ctypes.byref(make_config(**kw)))
    if n == 0:
        raise MclbmError(EINVAL, lib().mclbm_last_error().decode())
    return int(n)


def derive_constants(**kw) -> dict:
    """Derived lattice constants of a configuration (host-side, no GPU)."""
    out = np.zeros(len(DERIVED))
    _check(lib().mclbm_derive_constants(ctypes.byref(make_config(**kw)),
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size))
    return dict(zip(DERIVED, out.tolist()))


def checkpoint_info(path) -> tuple:
    """(configuration fields, step count, initial perturbation field or None)
    of a checkpoint file, read on the host (mclbm_checkpoint_info)."""
    L = lib()
    cfg = Config()
    t = ctypes.c_int64()
    n = ctypes.c_size_t()
    _check(L.mclbm_checkpoint_info(str(path).encode(), ctypes.byref(cfg), ctypes.byref(t), None, 0,
                                   ctypes.byref(n)))
    xi = None
    if n.value:
        xi = np.zeros(n.value)
        _check(L.mclbm_checkpoint_info(str(path).encode(), None, None,
                                       xi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), xi.size, None))
        xi = xi.reshape(cfg.ny, cfg.nx)
    fields = {name: getattr(cfg, name) for name, _ in Config._fields_
              if name not in ("force_scale", "fluid", "particle")}
    fields["force_scale"] = list(cfg.force_scale)
    return fields, int(t.value), xi


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Cavity:
    """One cavity resident on the current GPU.

    ``xi``: optional (ny, nx) field in [-1, 1] scaling the initial phi
    perturbation (see ``paper_1511_04552_amd.inputs.phi_perturbation``).
    Work is enqueued on ``stream`` (default: torch's current stream).
    """

    def __init__(self, xi=None, stream=None, device=None, **cfg):
        import torch
        L = lib()
        self.cfg = make_config(**cfg)
        self.nx, self.ny = int(self.cfg.nx), int(self.cfg.ny)
        nbytes = L.mclbm_device_bytes(ctypes.byref(self.cfg))
        if nbytes == 0:
            msg = L.mclbm_last_error().decode()
            # the validation's own code (EINVAL or EUNSUPPORTED)
            rc = L.mclbm_derive_constants(ctypes.byref(self.cfg), None, 0)
            raise MclbmError(rc if rc not in (OK, EINVAL) else EINVAL, msg)
        dev = torch.device("cuda" if device is None else device)
        self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self._buf.data_ptr()
        self._base = (base + 255) // 256 * 256
        self.nbytes = int(nbytes)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self._h = ctypes.c_void_p()
        xp = None
        if xi is not None:
            self._xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(-1)
            if self._xi.size != self.nx * self.ny:
                raise ValueError("xi must hold nx*ny values")
            xp = _dptr(self._xi)
        _check(L.mclbm_create(ctypes.byref(self.cfg), xp, ctypes.c_void_p(self._base),
                              ctypes.c_size_t(self.nbytes),
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._h)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mclbm_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- stepping -----------------------------------------------------------
    def step(self, n: int) -> None:
        _check(lib().mclbm_step(self._h, int(n)))

    @property
    def time(self) -> int:
        return int(lib().mclbm_time(self._h))

    def reset(self) -> None:
        _check(lib().mclbm_reset(self._h))

    def set_properties(self, Ra: float, phi0: float, dp_m: float) -> None:
        _check(lib().mclbm_set_properties(self._h, float(Ra), float(phi0), float(dp_m)))

    def checkpoint(self, path) -> None:
        """Write the complete state to ``path`` (JSON header line + raw sections)."""
        _check(lib().mclbm_checkpoint(self._h, str(path).encode()))

    def restore(self, path) -> None:
        """Read a checkpoint of a cavity with the identical configuration."""
        _check(lib().mclbm_restore(self._h, str(path).encode()))

    def load_fields(self, fields, affine=None) -> None:
        """Warm start from fields: a float32 device tensor (sy, sx, nc), nc = 4
        (u_x, u_y, theta, phi) or 5 (plus the deviation of rho_f~ from
        1 - phi0); affine: None or 2 nc floats mapping channel c to
        affine[c] * v + affine[nc + c].  Restarts at t = 0."""
        import torch
        if (fields.dtype != torch.float32 or not fields.is_cuda or fields.dim() != 3
                or fields.shape[2] not in (4, 5)):
            raise ValueError("fields must be a float32 device tensor of shape (sy, sx, 4 or 5)")
        f = fields.contiguous()
        nc = int(f.shape[2])
        aff = None
        if affine is not None:
            self._affine = np.ascontiguousarray(affine, dtype=np.float64)
            if self._affine.size != 2 * nc:
                raise ValueError(f"affine must hold {2 * nc} values")
            aff = _dptr(self._affine)
        _check(lib().mclbm_load_fields(self._h, ctypes.c_void_p(f.data_ptr()), int(f.shape[1]),
                                       int(f.shape[0]), nc, aff))

    def record_nusselt(self, every: int, ring=None) -> None:
        """mclbm_record_nusselt: every ``every`` steps the Nusselt numbers go
        to ``ring`` (a float64 device tensor of 4 * capacity values), with
        no host synchronisation; every = 0 switches recording off."""
        import torch
        if every > 0:
            if ring is None or ring.dtype != torch.float64 or not ring.is_cuda or not ring.is_contiguous() \
                    or ring.numel() < 4:
                raise ValueError("ring must be a contiguous float64 device tensor of 4 * capacity values")
            self._nu_ring = ring
            _check(lib().mclbm_record_nusselt(self._h, int(every), ctypes.c_void_p(ring.data_ptr()),
                                              int(ring.numel() // 4)))
        else:
            _check(lib().mclbm_record_nusselt(self._h, 0, None, 0))
            self._nu_ring = None

    def nusselt_records(self) -> int:
        return int(lib().mclbm_nusselt_records(self._h))

    def copy_state_from(self, src: "Cavity") -> None:
        """mclbm_copy_state: continue ``src``'s run here, converting the
        populations to this cavity's storage type (same configuration
        otherwise; ``src`` at an even step count)."""
        _check(lib().mclbm_copy_state(self._h, src._h))

    # ---- outputs ------------------------------------------------------------
    @staticmethod
    def _mask(names):
        if isinstance(names, str):
            names = (names,)
        mask = 0
        for n in names:
            mask |= FIELD_BIT[n]
        return mask, [n for n in FIELDS if mask & FIELD_BIT[n]]

    def moments(self, names=FIELDS) -> dict:
        mask, order = self._mask(names)
        out = np.zeros(len(order) * self.nx * self.ny)
        _check(lib().mclbm_read_moments(self._h, mask, _dptr(out), out.size))
        out = out.reshape(len(order), self.ny, self.nx)
        return {n: out[k] for k, n in enumerate(order)}

    def moments_device(self, names=FIELDS):
        """Moments as a float64 torch tensor on the device, (nf, ny, nx)."""
        import torch
        mask, order = self._mask(names)
        out = torch.empty((len(order), self.ny, self.nx), dtype=torch.float64, device=self._buf.device)
        _check(lib().mclbm_export_moments(self._h, mask, ctypes.c_void_p(out.data_ptr()), out.numel()))
        return order, out

    def populations(self) -> np.ndarray:
        nl = 4 if self.cfg.thermal_lattices == 2 else 3
        out = np.zeros(9 * nl * self.nx * self.ny)
        _check(lib().mclbm_read_populations(self._h, _dptr(out), out.size))
        return out.reshape(nl, 9, self.ny, self.nx)

    def nusselt(self, check: bool = True) -> tuple:
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        rc = lib().mclbm_nusselt(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        if check:
            _check(rc)
        return a.value, b.value, c.value

    def residual(self, check: bool = True) -> tuple:
        a, b = ctypes.c_double(), ctypes.c_double()
        rc = lib().mclbm_residual(self._h, ctypes.byref(a), ctypes.byref(b))
        if check:
            _check(rc)
        return a.value, b.value

    def residual_noalloc(self, dev_out) -> None:
        """mclbm_residual_noalloc: the residual into ``dev_out`` (a float64
        device tensor of at least 3 values: res_u, res_theta, non-finite
        flag) on the cavity's stream, without allocation or synchronisation."""
        import torch
        if dev_out.dtype != torch.float64 or not dev_out.is_cuda or dev_out.numel() < 3 \
                or not dev_out.is_contiguous():
            raise ValueError("dev_out must be a contiguous float64 device tensor of >= 3 values")
        _check(lib().mclbm_residual_noalloc(self._h, ctypes.c_void_p(dev_out.data_ptr())))

    def derived(self) -> dict:
        out = np.zeros(len(DERIVED))
        _check(lib().mclbm_derived(self._h, _dptr(out), out.size))
        return dict(zip(DERIVED, out.tolist()))


class _BatchMember(Cavity):
    """A cavity owned by a batch (outputs only; stepping goes through the batch)."""

    def __init__(self, batch, idx, handle, cfg):
        self._batch, self._idx = batch, idx
        self._h = ctypes.c_void_p(handle)
        self.cfg = cfg
        self.nx, self.ny = int(cfg.nx), int(cfg.ny)
        self.stream = batch.stream
        self._buf = batch._buf

    def close(self):
        self._h = None

    def step(self, n):
        raise MclbmError(ESTATE, "step the batch, not its members")


class Batch:
    """Uneven cavities stepped together: one launch per step (or per pair of
    steps) updates every active cavity, one workgroup per tile of every
    cavity, replayed from a captured graph.  ``cfgs``: list of keyword dicts as for ``Cavity``;
    ``xis``: optional list of perturbation fields (or None entries)."""

    def __init__(self, cfgs, xis=None, stream=None, device=None, graph_steps=None):
        import torch
        L = lib()
        n = len(cfgs)
        self._cfgs = (Config * n)(*[make_config(**c) for c in cfgs])
        nbytes = L.mclbm_batch_device_bytes(self._cfgs, n)
        if nbytes == 0:
            raise MclbmError(EINVAL, L.mclbm_last_error().decode())
        dev = torch.device("cuda" if device is None else device)
        self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = (self._buf.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.n = n
        xp = None
        if xis is not None:
            self._xis = [None if x is None else np.ascontiguousarray(x, dtype=np.float64).reshape(-1) for x in xis]
            arr = (ctypes.POINTER(ctypes.c_double) * n)()
            for k, x in enumerate(self._xis):
                if x is not None:
                    if x.size != self._cfgs[k].nx * self._cfgs[k].ny:
                        raise ValueError(f"xi {k} must hold nx*ny values")
                    arr[k] = _dptr(x)
            xp = arr
        self._h = ctypes.c_void_p()
        _check(L.mclbm_batch_create(self._cfgs, n, xp, ctypes.c_void_p(base), ctypes.c_size_t(nbytes),
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._h)))
        if graph_steps is not None:
            self.set_graph_steps(graph_steps)
        self.members = [_BatchMember(self, k, L.mclbm_batch_cavity(self._h, k), self._cfgs[k]) for k in range(n)]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mclbm_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int) -> None:
        _check(lib().mclbm_batch_step(self._h, int(n)))

    def set_graph_steps(self, steps: int) -> None:
        _check(lib().mclbm_batch_set_graph_steps(self._h, int(steps)))

    @property
    def per_cavity(self) -> bool:
        """True when the batch steps one workgroup per cavity, many steps per
        launch (``mclbm_batch_set_per_cavity``); False over tiles."""
        return lib().mclbm_batch_per_cavity(self._h) == 1

    @per_cavity.setter
    def per_cavity(self, on: bool) -> None:
        _check(lib().mclbm_batch_set_per_cavity(self._h, 1 if on else 0))

    def set_active(self, active) -> None:
        a = (ctypes.c_int32 * self.n)(*[1 if v else 0 for v in active])
        _check(lib().mclbm_batch_set_active(self._h, a))

    def residual(self, tol: float = 0.0):
        out = np.zeros(2 * self.n)
        st = (ctypes.c_int32 * self.n)()
        _check(lib().mclbm_batch_residual(self._h, float(tol), _dptr(out), st))
        return out.reshape(self.n, 2), np.array(st[:], dtype=np.int32)

    def nusselt(self) -> np.ndarray:
        out = np.zeros(3 * self.n)
        _check(lib().mclbm_batch_nusselt(self._h, _dptr(out)))
        return out.reshape(self.n, 3)

    def autotune(self, steps: int = 20) -> list:
        _check(lib().mclbm_batch_autotune(self._h, int(steps)))
        return [self.tile_shape(k) for k in range(self.n)]

    def tile_shape(self, idx: int) -> tuple:
        bx, by = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().mclbm_batch_tile_shape(self._h, int(idx), ctypes.byref(bx), ctypes.byref(by)))
        return bx.value, by.value

    def reset(self) -> None:
        _check(lib().mclbm_batch_reset(self._h))

    def time(self, idx: int) -> int:
        return int(lib().mclbm_batch_time(self._h, int(idx)))


def copy_kernel(dst, src, stream=None) -> None:
    """Plain device-to-device streaming copy (bandwidth calibration)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    nbytes = src.numel() * src.element_size()
    _check(lib().mclbm_copy_kernel(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                   ctypes.c_size_t(nbytes), ctypes.c_void_p(s.cuda_stream)))
