"""Batches of many small cavities stepped one workgroup per cavity, up to 256
steps per launch: bitwise the results of the tile schedule, with drop-out,
odd step counts and the default choice of schedule; one member against the
oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_1511_04552_amd as mc  # noqa: E402
from paper_1511_04552_amd import inputs  # noqa: E402
from parity import MOMENT_TOL, NU_TOL, assert_fields, assert_nusselt  # noqa: E402


def _small(n, seed=31, sides=((32, 32), (48, 40), (64, 64), (17, 23))):
    rng = np.random.default_rng(seed)
    cfgs = []
    for k in range(n):
        nx, ny = sides[k % len(sides)]
        cfgs.append(dict(nx=nx, ny=ny, Ra=float(10 ** rng.uniform(3, 5)), phi0=float(rng.uniform(0, 0.05)),
                         dp_nm=float(rng.uniform(20, 100)), tau_f=-1.0))
    xis = [inputs.phi_perturbation(seed + k, c["nx"], c["ny"]) for k, c in enumerate(cfgs)]
    return cfgs, xis


def _pair(n, seed=31):
    cfgs, xis = _small(n, seed)
    a = mc.Batch(cfgs, xis=xis)
    b = mc.Batch(cfgs, xis=xis)
    a.per_cavity = True
    b.per_cavity = False
    return cfgs, xis, a, b


def _equal(a, b, idx):
    for k in idx:
        assert np.array_equal(a.members[k].populations(), b.members[k].populations()), k


def test_per_cavity_equals_tiles_bitwise_with_odd_counts():
    cfgs, _, a, b = _pair(12)
    assert a.per_cavity and not b.per_cavity
    # 300 = one launch of 256 steps and one of 44; then an odd count, after
    # which the batch restarts from an odd step (one tile step first)
    for n in (300, 7, 101):
        a.step(n)
        b.step(n)
        _equal(a, b, range(len(cfgs)))
    assert a.time(0) == 408
    assert np.array_equal(np.asarray(a.nusselt()), np.asarray(b.nusselt()))


def test_per_cavity_with_dropped_cavities():
    cfgs, _, a, b = _pair(10, seed=7)
    a.step(64)
    b.step(64)
    active = [k % 3 != 1 for k in range(len(cfgs))]
    a.set_active(active)
    b.set_active(active)
    frozen = {k: a.members[k].populations() for k in range(len(cfgs)) if not active[k]}
    a.step(130)
    b.step(130)
    _equal(a, b, range(len(cfgs)))
    for k, p in frozen.items():
        assert np.array_equal(a.members[k].populations(), p), k
        assert a.time(k) == 64
    # every cavity back (dropped ones rejoin at an even step count of theirs)
    a.set_active([True] * len(cfgs))
    b.set_active([True] * len(cfgs))
    a.step(40)
    b.step(40)
    _equal(a, b, range(len(cfgs)))


def test_per_cavity_member_against_oracle():
    cfgs, xis = _small(3, seed=5)
    b = mc.Batch(cfgs, xis=xis)
    b.per_cavity = True
    b.step(400)
    for k in (1, 2):
        o = oracle.Oracle(xi=xis[k], **cfgs[k])
        o.step(400)
        assert_fields(b.members[k].moments(), o.moments(), MOMENT_TOL, f"member {k}")
        assert_nusselt(b.members[k].nusselt(), o.nusselt(), NU_TOL, f"member {k}")


def test_default_schedule_and_eligibility():
    def batch(n, side):
        return mc.Batch([dict(nx=side, ny=side, Ra=1e4, phi0=0.02, dp_nm=50.0)] * n)
    assert batch(128, 32).per_cavity           # many cavities of 32^2
    assert not batch(16, 32).per_cavity        # too few to fill the compute units
    assert not batch(64, 64).per_cavity
    assert batch(256, 64).per_cavity
    assert not batch(300, 96).per_cavity       # above 64^2: by choice or autotuning only
    big = mc.Batch([dict(nx=32, ny=32, Ra=1e4), dict(nx=200, ny=120, Ra=1e4)])
    assert not big.per_cavity
    with pytest.raises(mc.MclbmError) as e:
        big.per_cavity = True                  # a cavity above 128^2 nodes
    assert e.value.code == mc.EINVAL


def test_autotune_chooses_a_schedule_and_keeps_results():
    cfgs, xis = _small(128, seed=11, sides=((32, 32),))
    b = mc.Batch(cfgs, xis=xis)
    b.autotune(16)
    chosen = b.per_cavity
    ref = mc.Batch(cfgs, xis=xis)
    ref.per_cavity = not chosen
    b.step(70)
    ref.step(70)
    _equal(b, ref, range(0, 128, 9))
    print("autotuned schedule for 128 x 32^2: one workgroup per cavity" if chosen else "tiles", flush=True)


@pytest.mark.parametrize("storage", [mc.FP16S, mc.BF16S])
def test_per_cavity_16bit_storage_equals_tiles(storage):
    cfgs, xis = _small(9, seed=13)
    cfgs = [dict(c, storage=storage) for c in cfgs]
    a = mc.Batch(cfgs, xis=xis)
    b = mc.Batch(cfgs, xis=xis)
    a.per_cavity = True
    b.per_cavity = False
    for n in (260, 5):
        a.step(n)
        b.step(n)
        _equal(a, b, range(len(cfgs)))


def test_per_cavity_largest_cavities_equal_tiles():
    """Cavities up to the 128^2-node limit (16 nodes per thread, ragged
    last pass) give the tile schedule's bits."""
    cfgs, xis = _small(4, seed=23, sides=((128, 128), (100, 72), (127, 129), (33, 31)))
    a = mc.Batch(cfgs, xis=xis)
    b = mc.Batch(cfgs, xis=xis)
    a.per_cavity = True
    b.per_cavity = False
    for n in (130, 33):
        a.step(n)
        b.step(n)
        _equal(a, b, range(len(cfgs)))
