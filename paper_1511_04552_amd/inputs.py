"""Seeded synthetic inputs for the MCLBM cavity workloads.

This module holds no arithmetic of the method.  It only draws random numbers
and names workload parameter sets, so that the HIP path and the FP64 oracle
(used by the tests) receive identical inputs without sharing any code.

* ``phi_perturbation`` draws the +-1 field xi that scales the initial
  particle-volume-fraction perturbation (the cavity starts at rest with a
  uniform suspension, Section 2.d; the tiny seeded perturbation only breaks
  exact symmetry).  SplitMix64 (Steele, Lea and Flood, 2014), one draw per
  node in row-major order (x fastest).
* ``sweep_parameters`` draws a batch of uneven cavities for parameter sweeps.
* ``WORKLOADS`` names the cavity configurations used by tests and the bench.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int) -> np.ndarray:
    """First ``n`` outputs of SplitMix64 started at ``seed`` (uint64)."""
    with np.errstate(over="ignore"):
        k = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, n: int) -> np.ndarray:
    """``n`` doubles in [0, 1) from the top 53 bits of SplitMix64."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def phi_perturbation(seed: int, nx: int, ny: int) -> np.ndarray:
    """xi in [-1, 1), shape (ny, nx), row-major draw order."""
    return (2.0 * uniform(seed, nx * ny) - 1.0).reshape(ny, nx)


# Cavity workloads: 64^2 FP64 reference run; 512^2 run to steady state;
# 2048^2 reduced-precision storage case (properties of water / alumina).
WORKLOADS = {
    "cavity64_ra1e3": dict(nx=64, ny=64, Ra=1e3, Pr=6.2, phi0=0.01, dp_nm=100.0,
                           tau_f=0.8, seed=1),
    "cavity512_ra1e5": dict(nx=512, ny=512, Ra=1e5, Pr=6.2, phi0=0.03, dp_nm=50.0,
                            tau_f=0.8, seed=2),
    "cavity2048_ra1e6": dict(nx=2048, ny=2048, Ra=1e6, Pr=6.2, phi0=0.04, dp_nm=30.0,
                             tau_f=0.8, seed=4),
    "cavity160_paper": dict(nx=160, ny=160, Ra=1e6, Pr=8.923, phi0=0.04, dp_nm=33.0,
                            tau_f=0.8, seed=6),
    # 1.8 GB of populations: seven times the 256 MB last-level cache, so
    # every step streams from HBM (2048^2, 450 MB, is still partly cached)
    "cavity4096_ra1e6": dict(nx=4096, ny=4096, Ra=1e6, Pr=6.2, phi0=0.04, dp_nm=30.0,
                             tau_f=0.8, seed=7),
    # 2.29 GB of populations (above 2 GiB: 64-bit element offsets); the
    # stored 2000-step oracle samples of this cavity use seed 4
    "cavity4608_ra1e6": dict(nx=4608, ny=4608, Ra=1e6, Pr=6.2, phi0=0.04, dp_nm=30.0,
                             tau_f=0.8, seed=4),
}


def sweep_parameters(seed: int, count: int,
                     sides=(64, 128, 256, 384, 512)) -> list:
    """Uneven cavity batch: side uniform over ``sides``, Ra log-uniform in
    [1e3, 1e6], phi uniform in [0, 0.05], d_p uniform in [10, 100] nm."""
    u = uniform(seed, 4 * count).reshape(count, 4)
    out = []
    for k in range(count):
        side = int(sides[min(int(u[k, 0] * len(sides)), len(sides) - 1)])
        out.append(dict(nx=side, ny=side, Ra=float(10.0 ** (3.0 + 3.0 * u[k, 1])),
                        phi0=float(0.05 * u[k, 2]), dp_nm=float(10.0 + 90.0 * u[k, 3]),
                        seed=seed * 1000003 + k))
    return out


# Section 3.e: aspect ratio = height / width of the cavity (ny / nx); Ra and
# Nu are based on the width between the isothermal walls.
def aspect_ratio_configs(base: dict, width: int, ratios=(0.5, 1.0, 2.0)) -> list:
    """One cavity per aspect ratio: width nx = ``width``, height ny =
    round(ratio * width), the rest of ``base`` unchanged."""
    return [dict(base, nx=int(width), ny=max(4, int(round(r * width)))) for r in ratios]


# Slip-force ablation (Sections 3.a-3.b): every force on, each slip force
# off in turn, and all slip forces off (buoyancy only).  Force bits as in
# include/mclbm.h.
FORCE_BITS = {"drag": 1, "brownian": 2, "thermophoresis": 4, "saffman": 8, "magnus_rotation": 16, "gravity": 32}


def ablation_configs(base: dict) -> list:
    """(label, config) pairs of the ablation study."""
    full = sum(FORCE_BITS.values())
    out = [("all", dict(base, force_mask=full))]
    for name, bit in FORCE_BITS.items():
        out.append((f"no_{name}", dict(base, force_mask=full & ~bit)))
    out.append(("none", dict(base, force_mask=0)))
    return out
