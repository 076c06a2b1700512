"""Checks of the seeded input draws (composition, packing, velocities)."""

import numpy as np
import pytest
from scipy.spatial import cKDTree

import synth


@pytest.mark.parametrize("name", ["mol22", "cluster2500", "batch256"])
def test_min_separation_and_composition(make_system, name):
    s = make_system(name)
    for m in range(s.n_molecules):
        sl = s.molecule(m)
        p = s.pos[sl]
        d, _ = cKDTree(p).query(p, k=2)
        assert d[:, 1].min() >= 0.9
        counts = np.bincount(s.species[sl], minlength=4).tolist()
        n = p.shape[0]
        want = [12, 6, 2, 2] if name == "mol22" else synth.composition_counts(n)
        assert counts == want
        assert np.all(np.diff(s.species[sl]) >= 0)  # H block, then C, N, O
        mv = (s.masses[sl, None] * s.vel[sl]).sum(0)
        assert np.abs(mv).max() < 1e-12


def test_largest_remainder():
    assert synth.composition_counts(2500) == [1250, 750, 250, 250]
    assert synth.composition_counts(17) == [8, 5, 2, 2]
    for n in range(10, 301):
        c = synth.composition_counts(n)
        assert sum(c) == n
        assert all(abs(ci - n * r / 100) < 1 for ci, r in zip(c, (50, 30, 10, 10)))


def test_ball_density_and_radius(make_system):
    s = make_system("cluster2500")
    R = synth.ball_radius(2500)
    assert R == pytest.approx(18.14, abs=0.01)
    r = np.linalg.norm(s.pos, axis=1)
    assert r.max() < R
    inner = (r < 0.8 * R).sum() / (4 / 3 * np.pi * (0.8 * R) ** 3)
    assert inner == pytest.approx(0.1, rel=0.05)


def test_temperature_is_a_300K_draw(make_system):
    s = make_system("cluster2500")
    K = 0.5 * (s.masses[:, None] * s.vel ** 2).sum() / synth.generate.KAPPA
    dof = 3 * s.n_atoms - 3
    T = 2 * K / (dof * synth.generate.KB_EV)
    assert T == pytest.approx(300.0, rel=5 * np.sqrt(2.0 / dof))


def test_determinism_and_batch_sizes(make_system):
    a = synth.make_config("mol22")
    b = make_system("mol22")
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.weights, b.weights)
    s = make_system("batch256")
    sizes = np.diff(s.mol_offsets)
    assert s.n_molecules == 256 and sizes.min() >= 10 and sizes.max() <= 300
    w = synth.xavier_weights(0)
    assert w.dtype == np.float32 and w.shape == (synth.N_WEIGHTS,)
    W1 = w[:160 * 384]
    assert W1.std() == pytest.approx(np.sqrt(2.0 / 544), rel=0.02)


def test_golden_mol22_regression():
    """The stored 22-atom oracle values (written by tests/golden/make_golden.py
    from the oracle alone) are reproduced, so GPU tests may compare to them."""
    import json
    import os
    import oracle
    path = os.path.join(os.path.dirname(__file__), "golden", "mol22_oracle.json")
    ref = json.load(open(path))
    s = synth.make_config("mol22")
    E, Ei, F = oracle.energy_forces(s.pos, s.species, s.weights)
    assert E == pytest.approx(ref["energy"], rel=1e-13)
    np.testing.assert_allclose(F, np.array(ref["forces"]), atol=1e-13)
    x, v, U, K = oracle.vv(s.pos, s.vel, s.masses, s.species, s.weights, 0.5, 100)
    np.testing.assert_allclose(x, np.array(ref["final_positions"]), atol=1e-11)
    np.testing.assert_allclose(U, np.array(ref["U"]), atol=1e-11)


@pytest.mark.parametrize("name", ["box250", "box2500"])
def test_periodic_boxes(name):
    """Periodic cubes at 0.1 atoms/A^3: positions in [0, L), minimum distance
    between nearest images >= 0.9 A, the 50:30:10:10 composition, box edge at
    least twice the pair-list radius 6.2 A."""
    from scipy.spatial import cKDTree
    s = synth.make_config(name)
    L = s.box[0]
    assert L == pytest.approx((s.n_atoms / 0.1) ** (1 / 3))
    assert L >= 12.4
    assert s.pos.min() >= 0.0 and s.pos.max() < L
    d, _ = cKDTree(s.pos, boxsize=s.box).query(s.pos, k=2)
    assert d[:, 1].min() >= 0.9
    assert list(np.bincount(s.species, minlength=4)) == synth.composition_counts(s.n_atoms)
