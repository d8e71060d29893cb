"""The C ABI used from C: a plain C program (tests/c_abi/cavity_driver.c,
built by build()) allocates the device buffer with the HIP runtime, creates
a cavity, steps it with one and with two steps per launch, and reads Nu and
moments back.  Its output is compared with the FP64 oracle."""
import json
import os
import subprocess

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "c_abi", "cavity_driver")


@pytest.mark.parametrize("spl", [1, 2])
def test_c_program_on_the_abi_matches_oracle(spl):
    assert os.path.exists(DRIVER), "the C program is built by __graft_entry__.build()"
    nx, ny, Ra, phi0, dp_nm, steps = 48, 40, 1e4, 0.02, 50.0, 301
    print(f"driver {nx}x{ny} Ra {Ra} steps {steps} steps_per_launch {spl}", flush=True)
    r = subprocess.run([DRIVER, str(nx), str(ny), str(Ra), str(phi0), str(dp_nm), str(steps), str(spl)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["time"] == steps
    o = oracle.Oracle(nx=nx, ny=ny, Ra=Ra, phi0=phi0, dp_nm=dp_nm)
    o.step(steps)
    nu = o.nusselt()
    for key, ref in zip(("nu_hot", "nu_cold", "nu_hot_k"), nu):
        assert abs(out[key] - ref) <= 1e-4 * abs(ref), (key, out[key], ref)
    m = o.moments(("phi", "theta", "ux_ns"))
    assert abs(out["phi_sum"] - m["phi"].sum()) <= 1e-6 * m["phi"].sum()
    assert abs(out["theta_abs_sum"] - np.abs(m["theta"]).sum()) <= 1e-5 * np.abs(m["theta"]).sum()
    assert abs(out["ux_ns_max"] - np.abs(m["ux_ns"]).max()) <= 1e-5 * np.abs(m["ux_ns"]).max()
