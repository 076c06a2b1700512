"""Periodic boxes on the GPU (nearest-image pair search, periodic cell lists)
against the oracle's explicit-image periodic system (through the C ABI).

Whole-system parity at 250 and 2,500 atoms; at 23,000 atoms (cell list
tiling the box) sampled atoms against the gas-phase oracle on their nearest
images within 10.4 A, which the oracle pins show equal to the explicit-image
forces when the box is wider than 20.8 A.
"""

import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

TOL_F = {"fp32": 1e-4, "bf16x3": 1e-3}
TOL_E = {"fp32": 1e-6, "bf16x3": 1e-5}
# Per-atom energies, element-wise (derived with the parity tests' bars).
TOL_EI = {"fp32": 2e-6, "bf16x3": 1e-4}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ctx(system, **kw):
    import paper_2412_18271_amd as P
    return P.Context.from_system(system, **kw)


@pytest.fixture(scope="module")
def periodic_ref():
    cache = {}

    def get(s):
        if s.name not in cache:
            cache[s.name] = oracle.periodic_energy_forces(s.pos, s.species, s.weights, s.box)
        return cache[s.name]
    return get


@pytest.mark.parametrize("name,dtype,path,T", [
    ("box250", "fp32", "fused", 0), ("box250", "fp32", "plain", 0), ("box250", "bf16x3", "fused", 0),
    ("box2500", "fp32", "fused", 0), ("box2500", "bf16x3", "fused", 0),
    # 14-atom tiles: every atom a full shell, the smallest force-merge table
    ("box2500", "bf16x3", "fused", 14), ("box2500", "bf16x3", "fused", 16),
])
def test_periodic_energy_forces_match_oracle(make_system, periodic_ref, name, dtype, path, T):
    s = make_system(name)
    Eo, Eio, Fo = periodic_ref(s)
    ctx = _ctx(s, dtype=dtype, path=path, atoms_per_tile=T)
    E, F = ctx.compute(s.pos)
    Ei = ctx.atom_energies()
    S = np.abs(Eio).sum()
    dE = abs(E[0] - Eo) / S
    dF = np.abs(F - Fo).max()
    dEi = np.abs(Ei - Eio).max()
    _say("%s %s %s T=%d: |dE|/S %.2e max|dF| %.2e max|dEi| %.2e" % (name, dtype, path, T, dE, dF, dEi))
    assert dE <= TOL_E[dtype]
    assert dF <= TOL_F[dtype]
    assert dEi <= TOL_EI[dtype]
    # positions translated by whole box edges and shifted: same result
    shift = s.box * np.array([3.0, -2.0, 1.0]) + np.array([0.37, -1.1, 5.0])
    E2, F2 = ctx.compute(s.pos + shift)
    Eo2, _, Fo2 = oracle.periodic_energy_forces(s.pos + shift, s.species, s.weights, s.box) if name == "box250" \
        else (Eo, None, Fo)
    _say("  translated: |dE|/S %.2e max|dF| %.2e" % (abs(E2[0] - Eo2) / S, np.abs(F2 - Fo2).max()))
    assert abs(E2[0] - Eo2) / S <= TOL_E[dtype]
    assert np.abs(F2 - Fo2).max() <= TOL_F[dtype]
    ctx.close()


def test_periodic_box_via_compute_and_errors(make_system, periodic_ref):
    """The box passed to compute() becomes the context's box; NULL keeps it;
    set_box(None) returns to the gas phase; invalid boxes are rejected."""
    import paper_2412_18271_amd as P
    s = make_system("box250")
    Eo, _, Fo = periodic_ref(s)
    ctx = P.Context(s.species, s.masses, s.weights, None, dtype="fp32")
    E, F = ctx.compute(s.pos, box=s.box)
    assert np.abs(F - Fo).max() <= 1e-4
    E2, F2 = ctx.compute(s.pos)
    assert np.array_equal(F, F2)
    ctx.set_box(None)
    E3, F3 = ctx.compute(s.pos)
    Eg, _, Fg = oracle.energy_forces(s.pos, s.species, s.weights)
    _say("gas phase again: max|dF| %.2e" % np.abs(F3 - Fg).max())
    assert np.abs(F3 - Fg).max() <= 1e-4
    for bad in ([12.0, 20.0, 20.0], [20.0, float("inf"), 20.0], [20.0, 20.0, -30.0]):
        with pytest.raises(P.NNPError):
            ctx.set_box(bad)
    ctx.close()
    b = make_system("batch256")
    ctx = P.Context.from_system(b)
    with pytest.raises(P.NNPError):
        ctx.set_box([50.0, 50.0, 50.0])
    ctx.close()


def _check_sampled(ctx, s, pos, F, dtype, nsample, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    sel = np.sort(rng.choice(s.n_atoms, size=nsample, replace=False))
    Ei = ctx.atom_energies()
    dF, dEi = 0.0, 0.0
    for a in sel:
        idx, x = oracle.periodic_local_environment(pos, s.box, int(a), 10.4)
        loc = int(np.nonzero(idx == a)[0][0])
        Fa = oracle.forces_on(x, s.species[idx], s.weights, [loc])[0]
        idx5, x5 = oracle.periodic_local_environment(pos, s.box, int(a), 5.2)
        loc5 = int(np.nonzero(idx5 == a)[0][0])
        Ea = oracle.energy_forces(x5, s.species[idx5], s.weights, forces=False)[1][loc5]
        dF = max(dF, np.abs(F[a] - Fa).max())
        dEi = max(dEi, abs(Ei[a] - Ea))
    _say("  sampled %d atoms: max|dF| %.2e max|dEi| %.2e" % (nsample, dF, dEi))
    assert dF <= TOL_F[dtype]
    assert dEi <= TOL_EI[dtype]


@pytest.mark.parametrize("dtype", ["fp32", "bf16x3"])
def test_box23k_periodic_cell_lists(make_system, dtype):
    """23,000 atoms, L = 61.3 A: the cell list tiles the box (9 cells per
    edge); sampled atoms at the start and after 40 MD steps with rebuilds
    (atoms cross the faces: positions stay unwrapped)."""
    s = make_system("box23k")
    ctx = _ctx(s, dtype=dtype, path="fused")
    E, F = ctx.compute(s.pos)
    assert np.abs(F.sum(axis=0)).max() < 1e-3
    _check_sampled(ctx, s, s.pos, F, dtype, 48, 5)
    ctx.set_state(s.pos, s.vel)
    ctx.step(0.5, 40, graph=True)
    st = ctx.get_state()
    stats = ctx.stats()
    out = ((st["pos"] < 0) | (st["pos"] >= s.box)).any(axis=1).sum()
    _say("  after 40 steps: %s; %d atoms outside the box" % (stats, out))
    assert stats["rebuilds"] >= 2 and out > 0
    E2, F2 = ctx.compute(st["pos"])
    _check_sampled(ctx, s, st["pos"], F2, dtype, 24, 6)
    ctx.close()


def test_periodic_trajectory_matches_oracle(make_system):
    """250 atoms in the 13.6 A box, 20 velocity-Verlet steps of 0.5 fs: the
    positions follow the oracle's explicit-image periodic trajectory."""
    s = make_system("box250")
    x, v, U, K = oracle.periodic_vv(s.pos, s.vel, s.masses, s.species, s.weights, s.box, 0.5, 20)
    for graph in (False, True):
        ctx = _ctx(s, dtype="fp32", path="fused")
        ctx.set_state(s.pos, s.vel)
        ctx.step(0.5, 20, graph=graph)
        st = ctx.get_state()
        Ug, Kg = ctx.energy_log(21)
        dx = np.abs(st["pos"] - x).max()
        dU = np.abs(Ug[:, 0] - U).max()
        dK = np.abs(Kg[:, 0] - K).max()
        _say("graph %s: max|dx| %.2e max|dU| %.2e max|dK| %.2e" % (graph, dx, dU, dK))
        assert Ug.shape[0] == 21 and Kg.shape[0] == 21
        assert dx <= 1e-4
        assert dU <= 1e-4
        assert dK <= 1e-4
        ctx.close()


def test_periodic_autograd_matches_oracle(make_system, periodic_ref):
    """torch.autograd through the periodic box (recompute mode): the gradient
    of the energy is minus the explicit-image oracle forces."""
    import torch
    from paper_2412_18271_amd.autograd import NNPModel
    s = make_system("box250")
    Eo, _, Fo = periodic_ref(s)
    model = NNPModel.from_system(s, dtype="fp32", mode="recompute")
    pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda", requires_grad=True)
    E = model(pos)
    E.sum().backward()
    torch.cuda.synchronize()
    g = pos.grad.cpu().numpy()
    dF = np.abs(-g - Fo).max()
    _say("periodic autograd: |dE| %.2e max|grad + F| %.2e" % (abs(float(E.detach()[0]) - Eo), dF))
    assert dF <= TOL_F["fp32"]
