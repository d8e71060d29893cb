"""Two time steps per launch (k_step2): an even step and the following odd
step in one pass, from one population copy into the other.  Parity with the
oracle (every wall rule, both parities, ragged strips and bands), closeness
to the one-step path, the race check, checkpoints across the two schedules,
and full-size cavities."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_1511_04552_amd as mc  # noqa: E402
from paper_1511_04552_amd import inputs  # noqa: E402
from parity import field_errors, worst_error  # noqa: E402


class _env:
    def __init__(self, **kv):
        self.env = {k: str(v) for k, v in kv.items()}

    def __enter__(self):
        self.old = {k: os.environ.get(k) for k in self.env}
        os.environ.update(self.env)

    def __exit__(self, *a):
        for k, v in self.old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _make(cfg, xi, band=None, poison=False):
    env = {"MCLBM_POISON": "1" if poison else "0"}
    if band is not None:
        env["MCLBM_BAND2"] = band
    with _env(**env):
        return mc.Cavity(xi=xi, **cfg)


def _worst(mg, mo):
    return worst_error(mg, mo)


def _oracle_cfg(cfg):
    return {k: v for k, v in cfg.items() if k not in ("storage", "steps_per_launch")}


# strips are 62 columns wide: 37 (one ragged strip), 130 (three, the last
# with 6 columns), 62 and 63 (exact and one over); bands of 1, 3 and the
# automatic height (8 rows for these sizes)
CASES = [
    (dict(nx=37, ny=29, Ra=5e4, phi0=0.03, dp_nm=40.0), None),
    (dict(nx=37, ny=29, Ra=5e4, phi0=0.03, dp_nm=40.0), 1),
    (dict(nx=130, ny=21, Ra=1e5, phi0=0.02, dp_nm=30.0), 3),
    (dict(nx=62, ny=40, Ra=2e4, phi0=0.01, dp_nm=80.0, force_mask=mc.F_ALL & ~mc.F_MAGROT), None),
    (dict(nx=63, ny=5, Ra=1e4, phi0=0.04, dp_nm=60.0), 2),
    (dict(nx=5, ny=4, Ra=1e3, phi0=0.02, dp_nm=50.0), None),
    (dict(nx=48, ny=40, Ra=2e4, phi0=0.03, dp_nm=50.0, reading_flags=mc.R_COMMON_VELOCITY), 5),
]


@pytest.mark.parametrize("cfg,band", CASES)
def test_two_steps_per_launch_match_oracle(cfg, band):
    """1001 steps (500 launches of two and one single step at the end), and
    a start at an odd step (a single step first), against the oracle at the
    parity bar (1e-5 of each field's scale; Nu to 1e-4)."""
    cfg = dict(cfg, steps_per_launch=2)
    xi = inputs.phi_perturbation(141, cfg["nx"], cfg["ny"])
    o = oracle.Oracle(xi=xi, **_oracle_cfg(cfg))
    g = _make(cfg, xi, band)
    for n in (1, 2, 998):  # t = 1 (odd start), 3, 1001
        g.step(n)
        o.step(n)
        w = _worst(g.moments(), o.moments())
        print(cfg["nx"], cfg["ny"], band, g.time, f"vs oracle {w:.2e}")
        assert w <= 1e-5, (g.time, w)
    nu_g, nu_o = g.nusselt(), o.nusselt()
    for a, b in zip(nu_g, nu_o):
        assert abs(a - b) <= 1e-4 * max(abs(b), 1.0)


@pytest.mark.parametrize("shape", [(130, 67), (300, 200), (62, 9)])
def test_two_steps_per_launch_bitwise_equal_to_single_steps(shape):
    """Both schedules run the same node arithmetic on the same values: FP32
    storage holds the intermediate state exactly, and multiply-adds are
    fused per source expression, so the kernels give the same bits after
    every launch (odd counts end with a one-step launch)."""
    nx, ny = shape
    cfg = dict(nx=nx, ny=ny, Ra=1e5, phi0=0.03, dp_nm=40.0)
    xi = inputs.phi_perturbation(142, nx, ny)
    one = mc.Cavity(xi=xi, steps_per_launch=1, **cfg)
    two = mc.Cavity(xi=xi, steps_per_launch=2, **cfg)
    for n in (2, 3, 40, 600):
        one.step(n - one.time)
        two.step(n - two.time)
        assert np.array_equal(two.populations(), one.populations()), (shape, n)
    assert one.nusselt() == two.nusselt()
    assert np.isfinite(two.populations()).all()


@pytest.mark.parametrize("nx,ny,knobs,steps", [
    (300, 200, dict(MCLBM_BAND2=3, MCLBM_BANDMIX=3), 40),   # one whole window of 48 bands and a tail
    (300, 200, dict(MCLBM_BAND2=1, MCLBM_BANDMIX=5), 41),   # two windows of 80 bands and a tail, odd end
    (1536, 1400, dict(), 20),                               # the default interleave (6) at 2^21 nodes
])
def test_band_interleave_is_bitwise_neutral(nx, ny, knobs, steps):
    """The order in which the bands of a two-step launch are dispatched
    (MCLBM_BANDMIX, by default about 150 / strips from 2^21 nodes on) is a
    permutation of independent tiles: the results equal those of bands in
    order bit for bit."""
    cfg = dict(nx=nx, ny=ny, Ra=1e5, phi0=0.03, dp_nm=40.0, steps_per_launch=2)
    xi = inputs.phi_perturbation(143, nx, ny)
    with _env(**{**knobs, "MCLBM_BANDMIX": 1}):
        ref = mc.Cavity(xi=xi, **cfg)
    with _env(**knobs):
        mix = mc.Cavity(xi=xi, **cfg)
    ref.step(steps)
    mix.step(steps)
    names = ("rho_f", "ux_f", "uy_f", "phi", "ux_p", "theta")
    mr, mm = ref.moments(names), mix.moments(names)
    assert all(np.array_equal(mm[k], mr[k]) for k in names)
    assert mix.nusselt() == ref.nusselt()
    if nx * ny < 1 << 20:
        assert np.array_equal(mix.populations(), ref.populations())


@pytest.mark.parametrize("storage,tol", [(mc.FP16S, 6e-3), (mc.BF16S, 1.2e-1)])
def test_two_steps_per_launch_16bit_storage(storage, tol):
    """16-bit storage: the odd step starts from the even step's FP32 result
    (one rounding to storage per two steps); the bar is the 16-bit one, and
    the error is not above the one-step path's."""
    cfg = dict(nx=40, ny=33, Ra=1e5, phi0=0.02, dp_nm=30.0, storage=storage)
    xi = inputs.phi_perturbation(143, cfg["nx"], cfg["ny"])
    o = oracle.Oracle(xi=xi, **_oracle_cfg(cfg))
    o.step(1001)
    one = mc.Cavity(xi=xi, steps_per_launch=1, **cfg)
    two = mc.Cavity(xi=xi, steps_per_launch=2, **cfg)
    one.step(1001)
    two.step(1001)
    w1, w2 = _worst(one.moments(), o.moments()), _worst(two.moments(), o.moments())
    print(storage, f"one-step {w1:.2e}, two-step {w2:.2e}")
    assert w2 <= tol
    assert w2 <= 1.5 * w1 + 1e-4


@pytest.mark.parametrize("cfg,band", [CASES[0], CASES[2], CASES[5]])
def test_two_step_target_is_fully_written(cfg, band):
    """Race check: before every launch the target population copy and the
    lag field it writes are filled with NaN; the run must equal the plain
    run bitwise (every slot written once, nothing read before it is
    written)."""
    cfg = dict(cfg, steps_per_launch=2)
    xi = inputs.phi_perturbation(144, cfg["nx"], cfg["ny"])
    ref = _make(cfg, xi, band)
    ref.step(201)
    got = _make(cfg, xi, band, poison=True)
    got.step(201)
    p = got.populations()
    assert np.isfinite(p).all()
    assert np.array_equal(p, ref.populations())
    assert got.nusselt() == ref.nusselt()
    got.step(1)  # an even state: both lag fields in use
    ref.step(1)
    assert np.array_equal(got.populations(), ref.populations())


def test_checkpoints_cross_schedules(tmp_path):
    """A checkpoint holds the state, not the schedule: written by a two-step
    cavity (at an odd and at an even step) it resumes bitwise like the run
    that was not interrupted, in either schedule."""
    cfg = dict(nx=37, ny=29, Ra=5e4, phi0=0.03, dp_nm=40.0)
    xi = inputs.phi_perturbation(145, cfg["nx"], cfg["ny"])
    for at in (333, 334):
        full = mc.Cavity(xi=xi, steps_per_launch=2, **cfg)
        full.step(at)
        full.step(700 - at)
        part = mc.Cavity(xi=xi, steps_per_launch=2, **cfg)
        part.step(at)
        path = tmp_path / f"c{at}.ckpt"
        part.checkpoint(path)
        del part
        again = mc.Cavity(xi=xi, steps_per_launch=2, **cfg)
        again.restore(path)
        again.step(700 - at)
        assert np.array_equal(again.populations(), full.populations())
        single = mc.Cavity(xi=xi, steps_per_launch=1, **cfg)
        single.restore(path)
        single.step(700 - at)
        assert np.array_equal(single.populations(), full.populations())


def test_two_steps_per_launch_rejected_where_unsupported():
    with pytest.raises(mc.MclbmError) as e:
        mc.Cavity(nx=16, ny=16, thermal_lattices=2, steps_per_launch=2)
    assert e.value.code == mc.EUNSUPPORTED
    with pytest.raises(mc.MclbmError, match="one step per launch"):
        mc.Batch([dict(nx=16, ny=16), dict(nx=16, ny=16, steps_per_launch=2)])


@pytest.mark.parametrize("n", [2048, pytest.param(4096, marks=pytest.mark.slow)])
def test_full_size_two_steps_per_launch_match_oracle(n):
    """The full-size cavities (2048^2 Ra 1e6, 4096^2) with two steps per
    launch, their default schedule, in the launch shape the timing uses.  Four steps (two launches)
    and five (one more single step) against the oracle: densities and theta
    to 1e-5 of their variation (the velocities after a few steps are ~1e-9,
    below what FP32 deviations resolve), and the particle mass.  Host memory
    for the FP64 oracle: ~2 GB (2048^2), ~8 GB (4096^2)."""
    cfg = dict(nx=n, ny=n, Ra=1e6, phi0=0.04, dp_nm=30.0)
    xi = inputs.phi_perturbation(4, n, n)
    g = mc.Cavity(xi=xi, steps_per_launch=2, **cfg)
    # the default schedule at these sizes
    assert mc.device_bytes(**cfg) == mc.device_bytes(steps_per_launch=1, **cfg) + 27 * 4 * (n * n + 4160)
    phi0 = g.moments("phi")["phi"].sum()
    o = oracle.Oracle(xi=xi, **cfg)
    names = ("rho_f", "theta", "phi")
    for k in (4, 1):
        g.step(k)
        o.step(k)
        mg, mo = g.moments(names), o.moments(names)
        for f, v in field_errors(mg, mo).items():
            print(n, g.time, f, f"{v:.2e}")
            assert v <= 1e-5, (g.time, f)
        assert abs(mg["phi"].sum() - phi0) <= 1e-6 * phi0
    del o


def test_reset_set_properties_and_load_fields_with_two_steps():
    """The calls that rewrite the state work on whichever population copy is
    current: reset and set_properties restart bitwise like a fresh cavity,
    and a warm start from fields continues within rounding of the one-step
    run."""
    cfg = dict(nx=37, ny=29, Ra=5e4, phi0=0.03, dp_nm=40.0)
    xi = inputs.phi_perturbation(146, cfg["nx"], cfg["ny"])
    c = mc.Cavity(xi=xi, steps_per_launch=2, **cfg)
    c.step(101)  # odd: the second copy is current after the pairs
    c.reset()
    assert c.time == 0
    c.step(64)
    fresh = mc.Cavity(xi=xi, steps_per_launch=2, **cfg)
    fresh.step(64)
    assert np.array_equal(c.populations(), fresh.populations())
    c.step(3)
    c.set_properties(2e4, 0.02, 60e-9)
    c.step(50)
    other = mc.Cavity(xi=xi, steps_per_launch=2, **dict(cfg, Ra=2e4, phi0=0.02, dp_nm=60.0))
    other.step(50)
    assert np.array_equal(c.populations(), other.populations())
    # warm start: the same fields loaded into both schedules
    rng = np.random.default_rng(0)
    F = torch.tensor(rng.normal(size=(12, 16, 4)).astype(np.float32), device="cuda")
    aff = [0.01, 0.01, 0.5, 0.005, 0.0, 0.0, 0.0, cfg["phi0"]]
    runs = []
    for spl in (1, 2):
        d = mc.Cavity(xi=xi, steps_per_launch=spl, **cfg)
        d.step(7)
        d.load_fields(F, affine=aff)
        d.step(300)
        runs.append(d.populations())
    assert np.array_equal(runs[1], runs[0])
