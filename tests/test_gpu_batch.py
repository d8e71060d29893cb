"""Batched sweeps of uneven cavities (one launch per step over the tiles of
every cavity, replayed from a captured HIP graph) against single-cavity runs and the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_1511_04552_amd as mc  # noqa: E402
from paper_1511_04552_amd import inputs  # noqa: E402
from parity import field_errors  # noqa: E402

CFGS = [dict(nx=16, ny=16, Ra=1e4, phi0=0.01, dp_nm=100.0),
        dict(nx=37, ny=29, Ra=3e4, phi0=0.02, dp_nm=40.0),
        dict(nx=64, ny=64, Ra=1e3, phi0=0.01, dp_nm=100.0),
        dict(nx=100, ny=70, Ra=2e5, phi0=0.04, dp_nm=30.0, tau_f=-1.0),
        dict(nx=300, ny=40, Ra=5e4, phi0=0.0, dp_nm=60.0)]


def _xis(cfgs, seed=21):
    return [inputs.phi_perturbation(seed + k, c["nx"], c["ny"]) for k, c in enumerate(cfgs)]


def test_batch_bitwise_equals_single_cavities_and_matches_oracle():
    xis = _xis(CFGS)
    b = mc.Batch(CFGS, xis=xis)
    b.step(301)  # graph replays (32 steps) plus direct steps, odd total
    for k, (c, xi) in enumerate(zip(CFGS, xis)):
        single = mc.Cavity(xi=xi, **c)
        single.step(301)
        assert b.time(k) == 301
        assert np.array_equal(b.members[k].populations(), single.populations()), k
    # two members against the oracle (the others are equal to single runs,
    # which the single-cavity parity tests cover)
    for k in (1, 3):
        o = oracle.Oracle(xi=xis[k], **CFGS[k])
        o.step(301)
        err = field_errors(b.members[k].moments(), o.moments())
        for f, v in err.items():
            assert v <= 1e-5, (k, f, v)


def test_graph_replay_equals_direct_launches():
    """Replays of the captured step graph, with eager work and
    synchronisations between them, give bitwise the result of direct
    launches after every replay."""
    xis = _xis(CFGS)
    g = mc.Batch(CFGS, xis=xis, graph_steps=8)
    d = mc.Batch(CFGS, xis=xis, graph_steps=0)
    for rep in range(4):
        g.step(8)
        d.step(8)
        torch.cuda.synchronize()
        scratch = torch.zeros(1 << 20, device="cuda")  # unrelated eager work in between
        scratch += 1.0
        torch.cuda.synchronize()
        for k in range(len(CFGS)):
            assert np.array_equal(g.members[k].populations(), d.members[k].populations()), (rep, k)


def test_dropout_freezes_converged_cavities():
    xis = _xis(CFGS)
    b = mc.Batch(CFGS, xis=xis)
    b.step(200)
    res, st = b.residual(tol=0.0)  # report only
    assert (st == 0).all() and np.isfinite(res).all()
    b.set_active([1, 0, 1, 0, 1])
    frozen = {k: b.members[k].populations() for k in (1, 3)}
    b.step(50)
    for k in (1, 3):
        assert b.time(k) == 200
        assert np.array_equal(b.members[k].populations(), frozen[k])
    assert b.time(0) == 250
    # a dropped cavity at odd distance cannot rejoin
    b.step(1)
    with pytest.raises(mc.MclbmError):
        b.set_active([1, 1, 1, 1, 1])
    # converge-and-drop: a huge tolerance drops every active cavity
    res, st = b.residual(tol=1e30)
    assert list(st) == [1, 3, 1, 3, 1]
    t0 = [b.time(k) for k in range(5)]
    b.step(10)
    assert [b.time(k) for k in range(5)] == t0


def test_divergent_cavity_is_isolated():
    cfgs = CFGS[:2] + [dict(nx=16, ny=16, Ra=1e12, tau_f=0.51, phi0=0.0, force_mask=0)]
    b = mc.Batch(cfgs, xis=_xis(cfgs))
    b.step(3000)
    res, st = b.residual(tol=1e-30)
    assert st[2] == 2 and st[0] == 0 and st[1] == 0
    nu = b.nusselt()
    assert np.isfinite(nu[:2]).all()
    ref = mc.Cavity(xi=_xis(cfgs)[1], **cfgs[1])
    ref.step(3000)
    assert np.array_equal(b.members[1].populations(), ref.populations())


def test_autotune_picks_candidate_shapes_without_changing_results():
    xis = _xis(CFGS)
    b = mc.Batch(CFGS, xis=xis)
    shapes = b.autotune(steps=4)
    assert all(bx * by == 256 and bx in (256, 128, 64, 32) for bx, by in shapes)
    assert all(b.time(k) == 0 for k in range(len(CFGS)))
    b.step(64)
    ref = mc.Batch(CFGS, xis=xis)
    ref.step(64)
    for k in range(len(CFGS)):
        assert np.array_equal(b.members[k].populations(), ref.members[k].populations()), k


def test_members_cannot_be_stepped_directly():
    b = mc.Batch(CFGS[:2], xis=_xis(CFGS[:2]))
    with pytest.raises(mc.MclbmError):
        b.members[0].step(1)
    L = mc.lib()
    assert L.mclbm_step(b.members[0]._h, 1) == mc.ESTATE


def test_batch_nusselt_of_dropped_cavities_follows_their_state():
    """A dropped cavity's Nusselt numbers are reduced once and reused while
    its state is unchanged; a change of that state (a copied state, or
    rejoining and stepping) shows in the next batch call, which always
    equals the cavity's own call."""
    xis = _xis(CFGS)
    b = mc.Batch(CFGS, xis=xis)
    b.step(100)
    b.set_active([1, 0, 1, 1, 1])
    first = b.nusselt()
    b.step(50)
    second = b.nusselt()
    assert np.array_equal(first[1], second[1])
    assert np.array_equal(second[1], np.array(b.members[1].nusselt()))
    assert not np.array_equal(first[0], second[0])
    # a new state for the dropped member
    other = mc.Cavity(xi=xis[1], **CFGS[1])
    other.step(40)
    b.members[1].copy_state_from(other)
    third = b.nusselt()
    assert np.array_equal(third[1], np.array(other.nusselt()))
    assert not np.array_equal(third[1], second[1])
    # rejoin (even step counts on both sides), step, drop again
    b.set_active([1, 1, 1, 1, 1])
    b.step(10)
    b.set_active([1, 0, 1, 1, 1])
    fourth = b.nusselt()
    assert np.array_equal(fourth[1], np.array(b.members[1].nusselt()))
    assert not np.array_equal(fourth[1], third[1])
