"""The seeded input generators both sides consume (host-side): SplitMix64
against a scalar, arbitrary-precision rendering of its published definition
(Steele, Lea and Flood 2014: add the golden-ratio increment, then two
xor-shift-multiply rounds and a final xor-shift), and the ranges and
determinism of the fields and parameter sweeps drawn from it."""
import numpy as np

from paper_1511_04552_amd import inputs

MASK = (1 << 64) - 1


def _splitmix64_scalar(seed, n):
    state, out = seed & MASK, []
    for _ in range(n):
        state = (state + 0x9E3779B97F4A7C15) & MASK
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        out.append(z ^ (z >> 31))
    return out


def test_splitmix64_matches_its_definition():
    for seed in (0, 1, 42, 2**63 + 12345, MASK):
        got = inputs.splitmix64(seed, 257)
        assert [int(v) for v in got] == _splitmix64_scalar(seed, 257), seed


def test_uniform_and_perturbation_ranges():
    u = inputs.uniform(7, 100000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01 and abs(u.var() - 1 / 12) < 0.005
    # the top 53 bits of each draw, exactly
    raw = inputs.splitmix64(7, 10)
    assert np.array_equal(u[:10], (raw >> np.uint64(11)).astype(np.float64) / 2.0**53)
    xi = inputs.phi_perturbation(3, 37, 29)
    assert xi.shape == (29, 37) and xi.min() >= -1.0 and xi.max() < 1.0
    # row-major draw order, x fastest
    assert np.array_equal(xi.reshape(-1), 2.0 * inputs.uniform(3, 37 * 29) - 1.0)
    assert np.array_equal(xi, inputs.phi_perturbation(3, 37, 29))
    assert not np.array_equal(xi, inputs.phi_perturbation(4, 37, 29))


def test_sweep_parameters_ranges_and_determinism():
    a = inputs.sweep_parameters(3, 500)
    assert a == inputs.sweep_parameters(3, 500)
    assert {c["nx"] for c in a} == {64, 128, 256, 384, 512}
    assert all(c["nx"] == c["ny"] for c in a)
    ra = np.log10([c["Ra"] for c in a])
    assert ra.min() >= 3.0 and ra.max() < 6.0 and ra.max() - ra.min() > 2.8
    phi = np.array([c["phi0"] for c in a])
    dp = np.array([c["dp_nm"] for c in a])
    assert phi.min() >= 0.0 and phi.max() < 0.05 and dp.min() >= 10.0 and dp.max() < 100.0
    assert len({c["seed"] for c in a}) == len(a)
    assert {c["nx"] for c in inputs.sweep_parameters(5, 20, sides=(128,))} == {128}


def test_variant_builders():
    base = dict(nx=64, ny=64, Ra=1e4, phi0=0.02, dp_nm=40.0)
    ar = inputs.aspect_ratio_configs(base, 40)
    assert [(c["nx"], c["ny"]) for c in ar] == [(40, 20), (40, 40), (40, 80)]
    ab = dict(inputs.ablation_configs(base))
    full = sum(inputs.FORCE_BITS.values())
    assert ab["all"]["force_mask"] == full and ab["none"]["force_mask"] == 0
    for name, bit in inputs.FORCE_BITS.items():
        assert ab[f"no_{name}"]["force_mask"] == full & ~bit
