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
