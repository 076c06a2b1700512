"""Extra force providers summed with the network (the paper's callback
mechanism: an energy-only model differentiated by autograd, and explicit
forces from host NumPy code), through the C ABI callbacks.

The extra model is the paper's Methods example, E = sum of x^2; the oracle's
model 3 is the network plus that term.
"""

import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _model42(x):
    return (x ** 2).sum()


def _model42_forces(x):
    return (x ** 2).sum(), -2.0 * x


def _model42_numpy(x):
    return float((x ** 2).sum()), -2.0 * x


def _centred(s):
    return s.pos - s.pos.mean(axis=0)


def _ctx(s, **kw):
    import paper_2412_18271_amd as P
    return P.Context.from_system(s, **kw)


def test_energy_provider_matches_oracle(make_system):
    s = make_system("mol22")
    x = _centred(s)
    ctx = _ctx(s, dtype="fp32", path="fused")
    ctx.add_force(_model42, kind="energy")
    E, F = ctx.compute(x)
    Eo, Eio, Fo = oracle.energy_forces(x, s.species, s.weights)
    Eo += (x ** 2).sum()
    Fo = Fo - 2.0 * x
    dE, dF = abs(E[0] - Eo), np.abs(F - Fo).max()
    _say("network + sum x^2: |dE| %.2e max|dF| %.2e" % (dE, dF))
    assert dE <= 1e-6 * (np.abs(Eio).sum() + (x ** 2).sum())
    assert dF <= 1e-4
    # per-atom energies stay the network's
    assert np.abs(ctx.atom_energies() - Eio).max() <= 1e-5
    ctx.close()


def test_provider_md_matches_oracle(make_system):
    """100 velocity-Verlet steps with the provider against the oracle's
    network-plus-harmonic trajectory."""
    s = make_system("mol22")
    x = _centred(s)
    xo, vo, Uo, Ko = oracle.vv(x, s.vel, s.masses, s.species, s.weights, 0.5, 100, model=3)
    ctx = _ctx(s, dtype="fp32", path="fused")
    ctx.add_force(_model42, kind="energy")
    ctx.set_state(x, s.vel)
    ctx.step(0.5, 100)
    st = ctx.get_state()
    U, K = ctx.energy_log(101)
    dx, dU = np.abs(st["pos"] - xo).max(), np.abs(U[:, 0] - Uo).max()
    _say("100 steps: max|dx| %.2e max|dU| %.2e" % (dx, dU))
    # |dU| follows from |dx| through forces of up to ~10 eV/A on 66 coordinates
    assert dx <= 1e-3
    assert dU <= 1e-3
    ctx.close()


def test_provider_kinds_agree_bitwise(make_system):
    """Energy-only (autograd), explicit torch forces and NumPy forces give
    the same forces (the gradient of x^2 is exactly 2x) and therefore the
    same trajectory, bit for bit; graph requests fall back to step-by-step
    launches with the same result."""
    s = make_system("mol22")
    x = _centred(s)
    out = []
    for kind, fn, graph in (("energy", _model42, False), ("forces", _model42_forces, False),
                            ("numpy", _model42_numpy, False), ("energy", _model42, True)):
        ctx = _ctx(s, dtype="bf16x3", path="fused")
        ctx.add_force(fn, kind=kind)
        ctx.set_state(x, s.vel)
        ctx.step(0.5, 30, graph=graph)
        out.append(ctx.get_state())
        ctx.close()
    for o in out[1:]:
        assert np.array_equal(o["pos"], out[0]["pos"])
        assert np.array_equal(o["forces"], out[0]["forces"])
        assert abs(o["pot"][0] - out[0]["pot"][0]) <= 1e-9


def test_provider_errors_propagate_and_clear(make_system):
    import paper_2412_18271_amd as P
    s = make_system("mol22")

    def broken(x):
        raise ValueError("model failed")

    ctx = _ctx(s, dtype="fp32", path="fused")
    ctx.add_force(broken, kind="energy")
    with pytest.raises(P.NNPError) as ei:
        ctx.compute(s.pos)
    assert isinstance(ei.value.__cause__, ValueError)
    ctx.set_state(s.pos, s.vel)
    with pytest.raises(P.NNPError):
        ctx.step(0.5, 5)
    ctx.clear_forces()
    E, F = ctx.compute(s.pos)
    _, _, Fo = oracle.energy_forces(s.pos, s.species, s.weights)
    assert np.abs(F - Fo).max() <= 1e-4
    with pytest.raises(ValueError):
        ctx.add_force(_model42, kind="bogus")
    ctx.close()


def test_provider_per_molecule_energies(make_system):
    """A batch of 256 molecules: a provider returning one energy per molecule
    (sum of x^2 over each molecule) adds to each molecule's energy."""
    import torch
    s = make_system("batch256")
    mol = torch.as_tensor(np.repeat(np.arange(s.n_molecules), np.diff(s.mol_offsets)), device="cuda")

    def per_mol(x):
        return torch.zeros(s.n_molecules, dtype=x.dtype, device=x.device).index_add(0, mol, (x ** 2).sum(dim=1))

    ctx = _ctx(s, dtype="fp32", path="fused")
    ctx.add_force(per_mol, kind="energy")
    E, F = ctx.compute(s.pos)
    Eo, Eio, Fo = oracle.system_energy_forces(s)
    extra = np.array([(s.pos[s.molecule(m)] ** 2).sum() for m in range(s.n_molecules)])
    dE = np.abs(E - (Eo + extra)).max()
    dF = np.abs(F - (Fo - 2.0 * s.pos)).max()
    _say("batch256 + per-molecule sum x^2: max|dE| %.2e max|dF| %.2e" % (dE, dF))
    assert dE <= 1e-6 * extra.max()
    assert dF <= 1e-4
    ctx.close()
