"""Checkpoint / resume of the oracle: a run checkpointed at step k,
restored into a fresh state and continued is bitwise the uninterrupted run;
foreign or damaged files are refused."""
import numpy as np
import pytest

import oracle
from paper_1511_04552_amd import inputs


@pytest.mark.parametrize("kw", [dict(nx=20, ny=14, Ra=3e4, phi0=0.03, dp_nm=40.0),
                                dict(nx=16, ny=12, Ra=2e4, phi0=0.02, dp_nm=60.0, thermal_lattices=2)])
def test_resume_is_bitwise(tmp_path, kw):
    xi = inputs.phi_perturbation(12, kw["nx"], kw["ny"])
    full = oracle.Oracle(xi=xi, **kw)
    full.step(157)
    part = oracle.Oracle(xi=xi, **kw)
    part.step(63)
    path = tmp_path / "o.ckpt"
    part.checkpoint(path)
    part.step(5)  # diverge from the checkpoint, then come back
    fresh = oracle.Oracle(xi=xi, **kw)
    fresh.restore(path)
    assert fresh.time == 63
    fresh.step(94)
    assert np.array_equal(fresh.populations(), full.populations())
    assert fresh.nusselt() == full.nusselt()
    header = open(path, "rb").readline().decode()
    assert '"format": "mclbm-checkpoint"' in header and '"t": 63' in header and '"parity": 1' in header


def test_restore_refuses_other_configs_and_damaged_files(tmp_path):
    a = oracle.Oracle(nx=12, ny=10, Ra=1e4)
    a.step(3)
    path = tmp_path / "a.ckpt"
    a.checkpoint(path)
    b = oracle.Oracle(nx=12, ny=10, Ra=2e4)
    with pytest.raises(ValueError):
        b.restore(path)
    data = open(path, "rb").read()
    short = tmp_path / "short.ckpt"
    short.write_bytes(data[:-8])
    c = oracle.Oracle(nx=12, ny=10, Ra=1e4)
    before = c.populations().copy()
    with pytest.raises(ValueError):
        c.restore(short)
    assert np.array_equal(c.populations(), before) and c.time == 0
    junk = tmp_path / "junk.ckpt"
    junk.write_bytes(b"not a checkpoint\n" + data)
    with pytest.raises(ValueError):
        c.restore(junk)


def test_killed_run_resumes_from_its_last_checkpoint(tmp_path):
    """A process that checkpoints and is then killed (SIGKILL, mid-step)
    leaves a complete checkpoint; a new process restores it and continues
    bitwise like the uninterrupted run."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    path = tmp_path / "k.ckpt"
    kw = dict(nx=20, ny=14, Ra=3e4, phi0=0.03, dp_nm=40.0)
    code = (
        "import oracle\n"
        "from paper_1511_04552_amd import inputs\n"
        f"kw = {kw!r}\n"
        "o = oracle.Oracle(xi=inputs.phi_perturbation(12, 20, 14), **kw)\n"
        "o.step(63)\n"
        f"o.checkpoint({str(path)!r})\n"
        "print('checkpointed', flush=True)\n"
        "while True:\n"
        "    o.step(50)\n")
    p = subprocess.Popen([sys.executable, "-c", code], cwd=root, stdout=subprocess.PIPE, text=True)
    try:
        assert p.stdout.readline().strip() == "checkpointed"
        p.kill()
        p.wait(timeout=60)
    finally:
        if p.poll() is None:
            p.kill()
            p.wait(timeout=60)
    assert p.returncode != 0
    xi = inputs.phi_perturbation(12, 20, 14)
    full = oracle.Oracle(xi=xi, **kw)
    full.step(150)
    fresh = oracle.Oracle(xi=xi, **kw)
    fresh.restore(path)
    assert fresh.time == 63
    fresh.step(87)
    assert np.array_equal(fresh.populations(), full.populations())


def test_injected_nan_is_reported_as_divergence():
    """A NaN written into one interior population spreads and the residual
    reports MCLBM_EDIVERGED (-4); the wall Nusselt numbers become non-finite
    once it reaches the walls."""
    import ctypes
    o = oracle.Oracle(nx=16, ny=12, Ra=1e4, phi0=0.02, dp_nm=50.0)
    o.step(10)
    a, b = ctypes.c_double(), ctypes.c_double()
    assert oracle.lib().mclbm_oracle_residual(o._h, ctypes.byref(a), ctypes.byref(b)) == 0
    pops = o.populations()
    pops[0, 5, 6, 8] = np.nan
    o.write_populations(pops)
    o.step(30)
    assert oracle.lib().mclbm_oracle_residual(o._h, ctypes.byref(a), ctypes.byref(b)) == -4
    assert not np.isfinite(o.nusselt()[0])
