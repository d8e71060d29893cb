"""Learned warm start end to end: training data from the solver itself,
training through the library's kernels, and the gain over a cold start in
the time until the hot-wall Nu stays within 1e-3 of its steady value, with
both runs still converging to the same steady state."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1511_04552_amd import inputs, surrogate as sg  # noqa: E402


def _cases(seed, n, side):
    return [dict(c, tau_f=-1.0) for c in inputs.sweep_parameters(seed, n, sides=(side,))]


def test_warm_start_settles_sooner_and_converges_to_the_same_state():
    S = 32
    train = _cases(11, 96, S)
    F, steps, ok = sg.generate_dataset(train, chunk=2000, tol=1e-6, max_steps=600_000)
    assert ok.sum() >= 80
    ws = sg.WarmStart(S=S, C=32, m=8, L=4, Q=64, B=16, seed=0)
    hist = ws.fit([c for c, o in zip(train, ok) if o], F[ok], epochs=120, lr=3e-3, weights=(1, 1, 4, 1, 1))
    assert hist[-1] < 0.02 * hist[0]
    test = _cases(12, 8, S)
    cold = sg.run_to_steady(test, None, chunk=500, tol=1e-6, max_steps=800_000)
    warm = sg.run_to_steady(test, ws, chunk=500, tol=1e-6, max_steps=800_000)
    done = cold["converged"] & warm["converged"]
    assert done.sum() >= 6, (cold["converged"], warm["converged"])
    # the solver's own criterion reaches the same steady state either way
    nu_c, nu_w = cold["nu"][done], warm["nu"][done]
    assert np.all(np.abs(nu_w - nu_c) <= 1e-4 * np.abs(nu_c)), (nu_c, nu_w)
    # held-out prediction accuracy (standardised units, temperature channel)
    pred = ws.predict(test).cpu().numpy() * ws.std + ws.mean
    th_err = np.sqrt(((pred[..., 2] - cold["fields"][..., 2]) ** 2).mean()) / cold["fields"][..., 2].std()
    assert th_err < 0.03, th_err
    # time until Nu stays within 1e-3 of the cold run's converged value
    sc = sg.settle_steps(cold["times"], cold["nu_hist"], cold["nu"])[done]
    sw = sg.settle_steps(warm["times"], warm["nu_hist"], cold["nu"])[done]
    print("settle steps cold", sc.tolist(), "warm", sw.tolist())
    assert sw.sum() * 2.5 <= sc.sum(), (sc, sw)
