"""The GPU ablation cases resolve every slip force they switch on.

For each case of the force-ablation parity test, and each force on in it
other than drag, the oracle run with that force removed differs from the
case itself by at least 100 times the parity bar in some field.  A GPU path
that dropped or mis-scaled any one force would therefore fail that case.
"""
import numpy as np
import pytest

import oracle
from paper_1511_04552_amd import inputs
from parity import (ABLATION_MASKS, ABLATION_SEED, ABLATION_STEPS, MOMENT_TOL,
                    ablation_config, field_errors)

_NAMES = ("drag", "brownian", "thermophoresis", "saffman", "magnus/rotation", "gravity")


def _run(mask, scales_from):
    cfg = ablation_config(scales_from)
    cfg["force_mask"] = mask
    xi = inputs.phi_perturbation(ABLATION_SEED, cfg["nx"], cfg["ny"])
    o = oracle.Oracle(xi=xi, **cfg)
    o.step(ABLATION_STEPS)
    return o.moments(oracle.FIELDS[:9])


@pytest.mark.parametrize("mask", ABLATION_MASKS)
def test_each_force_changes_the_fields_beyond_the_bar(mask):
    ref = _run(mask, mask)
    assert all(np.isfinite(v).all() for v in ref.values())
    for k in range(1, 6):
        if not (mask >> k) & 1:
            continue
        eff = max(field_errors(_run(mask & ~(1 << k), mask), ref).values())
        print(_NAMES[k], f"{eff:.1e}")
        assert eff >= 100 * MOMENT_TOL, (_NAMES[k], eff)
