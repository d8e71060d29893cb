"""Grid convergence of the pure-fluid cavity on the GPU: the hot-wall Nu at
64^2, 128^2 and 256^2 (air, Ra = 1e4, steady state) converges at about
second order, and its Richardson extrapolation lands on the benchmark
value of the golden file (de Vahl Davis 1983)."""
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1511_04552_amd as mc  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cavity_air_nu.txt")


def _benchmark(Ra):
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            r, nu = line.split()[:2]
            if float(r) == Ra:
                return float(nu)
    raise KeyError(Ra)


def test_pure_fluid_nusselt_converges_to_benchmark():
    Ra = 1e4
    sides = (64, 128, 256)
    cfgs = [dict(nx=n, ny=n, Ra=Ra, Pr=0.71, phi0=0.0, tau_f=0.8, phi_perturb_amp=0.0) for n in sides]
    b = mc.Batch(cfgs)
    b.residual(tol=0.0)
    t = 0
    done = np.zeros(len(sides), bool)
    while t < 3_000_000 and not done.all():
        b.step(5000)
        t += 5000
        _, st = b.residual(tol=2e-7)  # 1: converged now (dropped), 3: dropped before
        assert not (st == 2).any(), st
        done |= (st == 1) | (st == 3)
    assert done.all(), t
    nu = b.nusselt()[:, 0]
    ref = _benchmark(Ra)
    p = math.log2((nu[0] - nu[1]) / (nu[1] - nu[2]))
    extrap = nu[2] + (nu[2] - nu[1]) / (2.0 ** p - 1.0)
    print("Nu", nu.tolist(), "order", p, "extrapolated", extrap, "benchmark", ref, "steps", t)
    # monotone convergence (the benchmark is printed to four digits, so the
    # distance to it does not resolve the finer grids)
    assert abs(nu[0] - nu[1]) > abs(nu[1] - nu[2]) > 0
    assert 1.3 < p < 2.7
    assert abs(extrap - ref) <= 5e-3 * ref
