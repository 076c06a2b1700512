"""Langevin dynamics (BAOAB, Philox4x64-10 noise) on the GPU against the
oracle's BAOAB with its own Philox (through the C ABI).

The noise of atom c in the step that starts at step count s depends only on
(seed, c, s), so the HIP trajectory and the oracle's follow the same random
path; they differ by the FP32 model arithmetic, as in velocity Verlet.
"""

import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

KB = 8.617333262e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ctx(system, **kw):
    import paper_2412_18271_amd as P
    return P.Context.from_system(system, **kw)


@pytest.mark.parametrize("friction", [0.1, 50.0])
def test_langevin_trajectory_matches_oracle(make_system, friction):
    """22 atoms, 100 BAOAB steps of 0.5 fs at 300 K, in two calls (60 + 40
    steps: the step count carries the noise sequence across calls), eager
    and graph-replayed: positions within 1e-3 A of the oracle's, energies
    within 1e-5 eV."""
    s = make_system("mol22")
    x, v, U, K = oracle.langevin(s.pos, s.vel, s.masses, s.species, s.weights, 0.5, 100, 300.0, friction, 7)
    _, _, Uv, _ = oracle.vv(s.pos, s.vel, s.masses, s.species, s.weights, 0.5, 100)
    for graph in (False, True):
        ctx = _ctx(s, path="fused", dtype="fp32")
        ctx.set_state(s.pos, s.vel)
        ctx.set_thermostat(300.0, friction, 7)
        ctx.step(0.5, 60, graph=graph)
        ctx.step(0.5, 40, graph=graph)
        st = ctx.get_state()
        Ug, Kg = ctx.energy_log(101)
        dx = np.abs(st["pos"] - x).max()
        dv = np.abs(st["vel"] - v).max()
        dU = np.abs(Ug[:, 0] - U).max()
        dK = np.abs(Kg[:, 0] - K).max()
        _say("friction %g graph %s: max|dx| %.2e max|dv| %.2e max|dU| %.2e max|dK| %.2e (|U - U_nve| %.2e)"
             % (friction, graph, dx, dv, dU, dK, np.abs(U - Uv).max()))
        assert dx <= 1e-3
        assert dU <= 1e-5 and dK <= 1e-5
        assert ctx.stats()["steps"] == 100
        ctx.close()
    # the thermostat changed the trajectory (it is not velocity Verlet)
    assert np.abs(U - Uv).max() > 1e-4


def test_langevin_off_restores_velocity_verlet(make_system):
    """friction 0 after a Langevin block gives the velocity-Verlet step again:
    the continuation equals the oracle's NVE run from the same state."""
    s = make_system("mol22")
    ctx = _ctx(s, path="fused", dtype="fp32")
    ctx.set_state(s.pos, s.vel)
    ctx.set_thermostat(300.0, 50.0, 3)
    ctx.step(0.5, 20)
    st = ctx.get_state()
    ctx.set_thermostat(300.0, 0.0, 3)
    ctx.step(0.5, 50)
    end = ctx.get_state()
    x, _, _, _ = oracle.vv(st["pos"], st["vel"], s.masses, s.species, s.weights, 0.5, 50)
    dx = np.abs(end["pos"] - x).max()
    _say("after thermostat off: max|dx| %.2e" % dx)
    assert dx <= 1e-3
    with pytest.raises(Exception):
        ctx.set_thermostat(-1.0, 0.1, 0)
    with pytest.raises(Exception):
        ctx.set_thermostat(300.0, float("nan"), 0)
    ctx.close()


def test_langevin_batch_noise_follows_caller_index(make_system):
    """256 molecules in one launch per step: molecules 0 and 37 follow the
    oracle's trajectories, each drawing its noise under its atoms' caller
    indices (the library's internal atom order does not enter)."""
    s = make_system("batch256")
    ctx = _ctx(s, path="fused", dtype="fp32")
    ctx.set_state(s.pos, s.vel)
    ctx.set_thermostat(300.0, 50.0, 11)
    ctx.step(0.5, 30)
    st = ctx.get_state()
    for m in (0, 37):
        sl = s.molecule(m)
        x, _, _, _ = oracle.langevin(s.pos[sl], s.vel[sl], s.masses[sl], s.species[sl], s.weights, 0.5, 30,
                                     300.0, 50.0, 11, first_index=sl.start)
        dx = np.abs(st["pos"][sl] - x).max()
        _say("molecule %d (%d atoms): max|dx| %.2e" % (m, sl.stop - sl.start, dx))
        assert dx <= 1e-3
    ctx.close()


def test_langevin_graph_replay_is_bitwise_equal_to_eager(make_system):
    s = make_system("cluster2500")
    out = []
    for graph in (False, True):
        ctx = _ctx(s, path="fused", dtype="bf16x3")
        ctx.set_state(s.pos, s.vel)
        ctx.set_thermostat(300.0, 0.1, 5)
        ctx.step(0.5, 120, graph=graph)
        ctx.step(0.5, 90, graph=graph)
        out.append(ctx.get_state())
        ctx.close()
    assert np.array_equal(out[0]["pos"], out[1]["pos"])
    assert np.array_equal(out[0]["vel"], out[1]["vel"])


def test_langevin_free_gas_is_exact_ornstein_uhlenbeck(make_system):
    """1,728 atoms on a lattice of 10 A spacing: no pair within the 5.2 A cutoff
    during 100 steps, so every force is exactly zero and BAOAB reduces to the
    Ornstein-Uhlenbeck velocity update plus free drift.  Positions and
    velocities equal the oracle's to FP64 rounding, and from v = 0 the scaled
    velocity variance after n steps is 1 - a^(2n), a = exp(-gamma dt) (tolerance:
    four standard errors of 5,184 values)."""
    import math
    import synth
    import paper_2412_18271_amd as P
    w = make_system("mol22").weights
    g = np.arange(12) * 10.0
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    n = pos.shape[0]
    rng = np.random.Generator(np.random.PCG64(17))
    species = rng.choice(4, size=n, p=[0.5, 0.3, 0.1, 0.1]).astype(np.int32)
    masses = np.array(synth.MASSES_AMU)[species]
    vel = np.zeros((n, 3))
    fric, T, dt = 50.0, 300.0, 0.5
    ctx = P.Context(species, masses, w, None, dtype="fp32", path="fused")
    ctx.set_state(pos, vel)
    ctx.set_thermostat(T, fric, 23)
    ctx.step(dt, 40)
    st = ctx.get_state()
    assert np.all(st["forces"] == 0.0)
    x, v, _, _ = oracle.langevin(pos, vel, masses, species, w, dt, 40, T, fric, 23, model=2)
    dx, dv = np.abs(st["pos"] - x).max(), np.abs(st["vel"] - v).max()
    a = math.exp(-fric * 1e-3 * dt)
    u = st["vel"] / np.sqrt(KB * T * 9.64853321e-3 / masses)[:, None]
    _say("free gas after 40 steps: max|dx| %.2e max|dv| %.2e; scaled variance %.4f (expected %.4f)"
         % (dx, dv, u.var(), 1 - a ** 80))
    assert dx <= 1e-12 and dv <= 1e-13
    assert abs(u.var() - (1 - a ** 80)) <= 4 * math.sqrt(2.0 / u.size) * (1 - a ** 80)
    ctx.step(dt, 60)
    st = ctx.get_state()
    assert np.all(st["forces"] == 0.0)
    u = st["vel"] / np.sqrt(KB * T * 9.64853321e-3 / masses)[:, None]
    _say("after 100 steps: scaled variance %.4f (expected %.4f)" % (u.var(), 1 - a ** 200))
    assert abs(u.var() - (1 - a ** 200)) <= 4 * math.sqrt(2.0 / u.size)
    ctx.close()
