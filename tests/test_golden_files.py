"""The stored oracle references are complete and self-consistent: every
sampled field and its scale present, finite values, the records in step
order.  (Host only; the values themselves come from the oracle scripts
beside them.)"""
import os

import numpy as np
import pytest

from parity import load_records, load_sampled

HERE = os.path.join(os.path.dirname(__file__), "golden")
FIELDS = ("rho_f", "ux_f", "uy_f", "phi", "ux_p", "uy_p", "theta", "ux_ns", "uy_ns")


@pytest.mark.parametrize("name,steps,side", [("cavity2048_ra1e6_sampled.txt", 2000, 2048),
                                             ("cavity4608_ra1e6_sampled.txt", 2000, 4608)])
def test_sampled_references(name, steps, side):
    g = load_sampled(os.path.join(HERE, name))
    assert g["steps"] == steps
    assert len(g["nu"]) == 3 and all(np.isfinite(g["nu"])) and g["nu"][0] > 1.0
    assert set(g["scales"]) == set(FIELDS) == set(g["samples"])
    for f in FIELDS:
        mean, dev, mag = g["scales"][f]
        assert np.isfinite([mean, dev, mag]).all() and mag > 0.0
        pts = g["samples"][f]
        assert len(pts) == 256
        assert all(0 <= x < side and 0 <= y < side and np.isfinite(v) and abs(v) <= mag * (1 + 1e-12)
                   for x, y, v in pts)


@pytest.mark.parametrize("name,side,last", [("cavity256_ra1e6_steady.txt", 256, 1000000),
                                            ("cavity160_paper_steady.txt", 160, None)])
def test_record_references(name, side, last):
    path = os.path.join(HERE, name)
    if not os.path.exists(path):
        pytest.skip("not written yet")
    rows, g = load_records(path, FIELDS)
    assert rows.shape[1] == 6 and len(rows) >= 2
    assert (np.diff(rows[:, 0]) > 0).all()
    if last is not None:
        assert rows[-1, 0] == last
    assert np.isfinite(rows).all() and (rows[:, 1:4] > 1.0).all()
    assert set(g["scales"]) == set(FIELDS) == set(g["samples"])
    assert all(len(g["samples"][f]) == 100 for f in FIELDS)
    assert all(0 <= x < side and 0 <= y < side for f in FIELDS for x, y, _ in g["samples"][f])
