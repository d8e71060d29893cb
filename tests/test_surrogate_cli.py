"""The warm-start evaluation split over processes: runs saved by
``--eval cold`` / ``--eval warm --save-run`` combine into the same report
as one process would make (host-side, synthetic runs)."""
import json

import numpy as np

from paper_1511_04552_amd import surrogate as sg


def _run(nu_inf, tau, seconds, t_load):
    times = np.arange(1, 401) * 500
    nu_hist = nu_inf[None, :] * (1.0 + 0.2 * np.exp(-times[:, None] / tau[None, :]))
    return dict(steps=np.array([20000, 30000, 0]), converged=np.array([True, True, False]),
                nu=nu_hist[-1], times=times, nu_hist=nu_hist, seconds=np.float64(seconds),
                t_load=np.float64(t_load), fields=np.zeros((3, 4, 4, sg.NCH), np.float32))


def test_combine_saved_runs(tmp_path):
    nu_inf = np.array([1.3, 2.5, 6.0])
    cold = _run(nu_inf, np.array([8000.0, 12000.0, 5000.0]), 12.0, 0.0)
    warm = _run(nu_inf * (1 + 1e-5), np.array([1000.0, 3000.0, 500.0]), 12.0, 0.004)
    np.savez(tmp_path / "c.npz", **cold)
    np.savez(tmp_path / "w.npz", **warm)
    out = tmp_path / "r.json"
    assert sg.main(["--combine", str(tmp_path / "c.npz"), str(tmp_path / "w.npz"), "--train-side", "8",
                    "--eval-side", "16", "--horizon", "200000", "--out", str(out)]) == 0
    ev = json.load(open(out))["eval"]
    sc = sg.settle_steps(cold["times"], cold["nu_hist"], cold["nu"])
    sw = sg.settle_steps(warm["times"], warm["nu_hist"], cold["nu"])
    assert ev["cold_settle_steps"] == sc.tolist() and ev["warm_settle_steps"] == sw.tolist()
    assert abs(ev["settle_ratio_total"] - sc.sum() / sw.sum()) < 1e-12
    # a decay 8x faster settles about 8x sooner
    assert 5 < ev["settle_ratio_total"] < 12
    assert ev["count"] == 3 and ev["met_both"] == 2
    assert abs(ev["final_nu_rel_diff_max"] - 1e-5) < 1e-9
    assert abs(ev["seconds_load"] - 0.004) < 1e-12
