"""Differentiation path: torch.autograd over the HIP energy and adjoint.

Forces are checked against the FP64 oracle's analytic gradient, against
central finite differences of the oracle energy (h = 1e-4 A) and between
the recompute and stored-intermediate modes.
"""

import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _grad(model, pos_np, dtype=None):
    import torch
    dtype = dtype or torch.float64
    pos = torch.tensor(pos_np, dtype=dtype, device="cuda", requires_grad=True)
    E = model(pos)
    E.sum().backward()
    torch.cuda.synchronize()
    return E.detach().cpu().numpy(), pos.grad.detach().cpu().numpy()


@pytest.mark.parametrize("mode", ["recompute", "store"])
@pytest.mark.parametrize("dtype", ["fp32", "bf16x3"])
def test_autograd_forces_match_oracle(make_system, mode, dtype):
    import torch
    from paper_2412_18271_amd.autograd import NNPModel
    s = make_system("cluster2500")
    model = NNPModel.from_system(s, dtype=dtype, mode=mode)
    E, g = _grad(model, s.pos)
    Eo, Eio, Fo = oracle.energy_forces(s.pos, s.species, s.weights)
    dE = abs(E[0] - Eo) / np.abs(Eio).sum()
    dF = np.abs(-g - Fo).max()
    _say("autograd %s %s: |dE|/S %.2e  max|grad + F| %.2e" % (mode, dtype, dE, dF))
    assert dF <= (1e-4 if dtype == "fp32" else 1e-3)
    # float32 positions: the same path, positions rounded to float32
    E32, g32 = _grad(model, s.pos, torch.float32)
    Eo32, _, Fo32 = oracle.energy_forces(s.pos.astype(np.float32).astype(np.float64), s.species, s.weights)
    _say("  float32 positions: |dE|/S %.2e  max|grad + F| %.2e" % (
        abs(E32[0] - Eo32) / np.abs(Eio).sum(), np.abs(-g32 - Fo32).max()))
    assert np.abs(-g32 - Fo32).max() <= (1e-4 if dtype == "fp32" else 1e-3)


def test_autograd_modes_agree_and_scale(make_system):
    """Recompute and stored modes give the same gradient; a weighted sum of
    two molecules' energies scales each molecule's gradient.

    With 8-atom tiles both modes sum each atom's descriptors in the same
    order and agree to 1e-9.  The default tiles of a system this size (16
    atoms, angular work pooled over the workgroup) sum the angular
    descriptors in fixed point instead: rounding-level differences, bounded
    by twice the split-BF16 force error against the oracle (3e-5 eV/A)."""
    import torch
    from paper_2412_18271_amd.autograd import NNPModel
    s = make_system("batch256")
    grads = {}
    for mode, T in (("recompute", 8), ("store", 8), ("recompute", 0)):
        m = NNPModel.from_system(s, dtype="bf16x3", mode=mode, atoms_per_tile=T)
        pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda", requires_grad=True)
        E = m(pos)
        w = torch.zeros_like(E)
        w[0], w[5] = 2.0, -0.5
        (E * w).sum().backward()
        grads[mode, T] = pos.grad.cpu().numpy()
    np.testing.assert_allclose(grads["recompute", 8], grads["store", 8], rtol=0, atol=1e-9)
    d = np.abs(grads["recompute", 0] - grads["store", 8]).max()
    _say("default tiles against 8-atom tiles: max|d grad| %.2e" % d)
    assert d <= 1e-4
    _, _, F0 = oracle.energy_forces(s.pos[s.molecule(0)], s.species[s.molecule(0)], s.weights)
    for key in grads:
        np.testing.assert_allclose(grads[key][s.molecule(0)], -2.0 * F0, atol=2e-3)
        assert np.all(grads[key][s.molecule(1)] == 0.0)


def test_droplet100k_finite_differences_subcluster_and_memory(make_system):
    """100,000 atoms, split-BF16 network, descriptors recomputed in backward:
    forces on 64 random atoms against central differences of the oracle
    energy (h = 1e-4 A; only E_i with r_ia < 5.2 A change, evaluated on their
    exact local environments), the 500 atoms nearest the centroid as an
    isolated molecule against the oracle, and device memory of both modes."""
    import torch
    from paper_2412_18271_amd.autograd import NNPModel
    s = make_system("droplet100k")
    torch.cuda.reset_peak_memory_stats()
    model = NNPModel.from_system(s, dtype="bf16x3", mode="recompute")
    E, g = _grad(model, s.pos)
    bytes_recompute = model.device_bytes()
    rng = np.random.Generator(np.random.PCG64(43))
    sel = rng.choice(s.n_atoms, size=64, replace=False)
    h = 1e-4
    errs = []
    for a in sel:
        env = oracle.local_environment(s.pos, int(a), 10.4 + 0.5)
        loc = int(np.nonzero(env == a)[0][0])
        near = oracle.local_environment(s.pos[env], loc, 5.2 + 1e-3)  # E_i that depend on x_a
        fd = np.zeros(3)
        for c in range(3):
            e = []
            for sign in (1, -1):
                p = s.pos[env].copy()
                p[loc, c] += sign * h
                Ei = oracle.energy_forces(p, s.species[env], s.weights, forces=False)[1]
                e.append(Ei[near].sum())
            fd[c] = -(e[0] - e[1]) / (2 * h)
        errs.append(np.abs(-g[a] - fd).max())
    _say("droplet100k FD on 64 atoms: max|grad + F_fd| %.2e" % max(errs))
    assert max(errs) <= 1e-3
    # 500-atom sub-cluster
    c0 = s.pos.mean(axis=0)
    sub = np.sort(np.argsort(np.linalg.norm(s.pos - c0, axis=1))[:500])
    subsys = synth.System("sub500", s.pos[sub], s.species[sub], s.masses[sub], s.vel[sub],
                          np.array([0, 500], np.int32), s.weights, {})
    order = np.argsort(subsys.species, kind="stable")
    subsys = synth.System("sub500", subsys.pos[order], subsys.species[order], subsys.masses[order],
                          subsys.vel[order], subsys.mol_offsets, s.weights, {})
    msub = NNPModel.from_system(subsys, dtype="bf16x3", mode="recompute")
    Es, gs = _grad(msub, subsys.pos)
    Eo, Eio, Fo = oracle.energy_forces(subsys.pos, subsys.species, s.weights)
    _say("sub-cluster 500: |dE|/S %.2e max|grad + F| %.2e" % (abs(Es[0] - Eo) / np.abs(Eio).sum(),
                                                            np.abs(-gs - Fo).max()))
    assert np.abs(-gs - Fo).max() <= 1e-3
    # stored mode holds descriptors and dE/dG in addition
    mstore = NNPModel.from_system(s, dtype="bf16x3", mode="store")
    E2, g2 = _grad(mstore, s.pos)
    bytes_store = mstore.device_bytes()
    _say("device bytes: recompute %.1f MB, store %.1f MB" % (bytes_recompute / 1e6, bytes_store / 1e6))
    assert bytes_store - bytes_recompute >= 2 * 384 * 4 * s.n_atoms
    # the recompute mode's default tiles pool the angular descriptor sums
    # (fixed point) where the stored mode sums per atom: rounding-level
    # differences (see test_autograd_modes_agree_and_scale)
    d = np.abs(g2 - g).max()
    _say("stored against recompute: max|d grad| %.2e" % d)
    assert d <= 1e-4
