"""Seeded input generators: lattice sites, momentum, temperature, determinism."""
import numpy as np
import pytest

from paper_2003_14061_amd import inputs


def test_fcc_full_lattice_counts_and_spacing():
    L = inputs.box_length(4000, 0.8)
    p = inputs.fcc_positions(4000, L)
    assert p.shape == (4000, 3)
    assert np.all(p >= 0) and np.all(p < L)
    a = L / 10
    # nearest-neighbour distance of FCC is a / sqrt(2)
    d = p[1:] - p[0]
    d -= L * np.round(d / L)
    assert np.sqrt((d * d).sum(1)).min() == pytest.approx(a / np.sqrt(2), rel=1e-12)
    assert len(np.unique(np.round(p, 9), axis=0)) == 4000


def test_fcc_subset_is_seeded_and_without_replacement():
    L = inputs.box_length(1234, 0.7)
    a = inputs.fcc_positions(1234, L, np.random.default_rng(3))
    b = inputs.fcc_positions(1234, L, np.random.default_rng(3))
    assert np.array_equal(a, b)
    assert len(np.unique(np.round(a, 9), axis=0)) == 1234


def test_velocities_zero_momentum_and_temperature():
    v = inputs.thermal_velocities(5000, 0.72, np.random.default_rng(1))
    assert np.abs(v.sum(0)).max() < 1e-10
    T = (v * v).sum() / (3 * (5000 - 1))
    assert T == pytest.approx(0.72, rel=1e-12)


def test_presets_and_ensemble():
    w = inputs.preset("wca_4000").materialize()
    assert w.pos.shape == (4000, 3) and w.L == pytest.approx(17.0997594, rel=1e-7)
    w2 = inputs.preset("wca_4000").materialize()
    assert np.array_equal(w.vel, w2.vel)
    specs = inputs.ensemble_specs()
    assert len(specs) == 64
    ns = np.array([s[0] for s in specs])
    rhos = np.array([s[1] for s in specs])
    assert ns.min() >= 500 and ns.max() <= 32000
    assert rhos.min() >= 0.6 and rhos.max() <= 0.9
