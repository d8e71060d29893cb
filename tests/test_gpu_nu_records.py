"""Periodic Nusselt numbers recorded on the device while stepping
(mclbm_record_nusselt): equal, bitwise, to synchronous mclbm_nusselt calls
on a twin cavity stepped to the same step counts, with one and with two
steps per launch (where a record falls on the odd step of a pair, the pair
runs as two single steps, which the twin's stepping to that count does
too), through the ring's wrap-around."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1511_04552_amd as mc  # noqa: E402
from paper_1511_04552_amd import inputs  # noqa: E402

CFG = dict(nx=300, ny=41, Ra=1e5, phi0=0.03, dp_nm=50.0)


@pytest.mark.parametrize("spl", [1, 2])
def test_recorded_nusselt_equals_synchronous_calls(spl):
    xi = inputs.phi_perturbation(14, CFG["nx"], CFG["ny"])
    rec = mc.Cavity(xi=xi, steps_per_launch=spl, **CFG)
    twin = mc.Cavity(xi=xi, steps_per_launch=spl, **CFG)
    ring = torch.full((4 * 4,), float("nan"), dtype=torch.float64, device="cuda")
    every = 75
    rec.record_nusselt(every, ring)
    rec.step(1000)
    assert rec.nusselt_records() == 1000 // every
    expect = {}
    for m in range(every, 1001, every):
        twin.step(m - twin.time)
        expect[m] = twin.nusselt()
    got = ring.cpu().numpy().reshape(4, 4)
    n = rec.nusselt_records()
    for k in range(n - 4, n):
        m = (k + 1) * every
        slot = got[k % 4]
        assert slot[3] == 0.0
        assert tuple(slot[:3]) == expect[m], (m, slot, expect[m])
    # the state itself is the twin's: the recording steps are the same steps
    twin.step(1000 - twin.time)
    assert np.array_equal(rec.populations(), twin.populations())
    rec.record_nusselt(0)
    rec.step(150)
    assert rec.nusselt_records() == 0


def test_record_nusselt_rejects_bad_arguments():
    c = mc.Cavity(nx=16, ny=16, Ra=1e4)
    with pytest.raises(ValueError):
        c.record_nusselt(10, torch.zeros(2, dtype=torch.float64, device="cuda"))
    L = mc.lib()
    assert L.mclbm_record_nusselt(c._h, -1, None, 0) == mc.EINVAL
    assert L.mclbm_record_nusselt(c._h, 5, None, 4) == mc.EINVAL
    b = mc.Batch([dict(nx=16, ny=16, Ra=1e4)])
    assert L.mclbm_record_nusselt(b.members[0]._h, 0, None, 0) == mc.ESTATE
