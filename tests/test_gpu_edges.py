"""Degenerate and boundary cases of the HIP path against the oracle (through
the C ABI): lone atoms (no neighbours: the network of an all-zero
descriptor, no force), dimers on both sides of the 3.5 A and 5.2 A cutoffs,
collinear and right-angle trimers, a batch of molecules of one, two and
three atoms next to larger ones (ragged tiles, tiles mixing molecules), and
capacity overflow reported as an error, and invalid positions (NaN, Inf,
coincident atoms) rejected before any device work.
"""

import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL_F = {"fp32": 1e-4, "bf16x3": 1e-3}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ctx(species, weights, **kw):
    import paper_2412_18271_amd as P
    species = np.asarray(species, dtype=np.int32)
    return P.Context(species, synth.MASSES_AMU[species], weights, kw.pop("mol_offsets", None), **kw)


@pytest.fixture(scope="module")
def weights():
    return synth.xavier_weights(0)


def _scale(Eio):
    # energy errors of the network are set by its activations, not by the
    # size of E_i (which vanishes without neighbours: zero biases): below
    # S = sum |E_i| = 1 eV the tolerances apply in eV
    return max(np.abs(Eio).sum(), 1.0)


def _compare(ctx, pos, species, weights, dtype):
    E, F = ctx.compute(pos)
    Eo, Eio, Fo = oracle.energy_forces(pos, np.asarray(species, np.int32), weights)
    dE = abs(E[0] - Eo) / _scale(Eio)
    dF = np.abs(F - Fo).max()
    return dE, dF, F


@pytest.mark.parametrize("dtype", ["fp32", "bf16x3"])
def test_lone_atoms(weights, dtype):
    """One atom of each element, each alone in its own context: energy of the
    all-zero descriptor, zero force."""
    for e in range(4):
        ctx = _ctx([e], weights, dtype=dtype, path="fused")
        dE, dF, F = _compare(ctx, np.array([[1.0, -2.0, 3.0]]), [e], weights, dtype)
        _say("lone element %d %s: |dE| %.2e" % (e, dtype, dE))
        assert np.all(F == 0.0)
        assert dE <= 1e-12
        ctx.close()


@pytest.mark.parametrize("dtype,path", [("fp32", "fused"), ("fp32", "plain"), ("bf16x3", "fused")])
def test_dimers_across_cutoffs(weights, dtype, path):
    """H-O dimers just inside and outside both cutoffs and very close."""
    for r in (0.3, 1.0, 3.4999, 3.5001, 5.1999, 5.2001, 7.0):
        pos = np.array([[0.0, 0.0, 0.0], [r * 0.6, r * 0.8, 0.0]])
        ctx = _ctx([0, 3], weights, dtype=dtype, path=path)
        dE, dF, F = _compare(ctx, pos, [0, 3], weights, dtype)
        _say("dimer r=%.4f %s %s: |dE|/S %.2e max|dF| %.2e" % (r, dtype, path, dE, dF))
        assert dF <= TOL_F[dtype]
        assert dE <= (1e-6 if dtype == "fp32" else 1e-5)
        if r > 5.2:
            assert np.all(F == 0.0)
        ctx.close()


@pytest.mark.parametrize("dtype", ["fp32", "bf16x3"])
def test_trimers_special_angles(weights, dtype):
    """C-H-N trimers: collinear (theta = 180 deg), right angle, and an
    acute angle with both arms just inside 3.5 A."""
    cases = {
        "collinear": np.array([[0.0, 0.0, 0.0], [1.1, 0.0, 0.0], [-1.4, 0.0, 0.0]]),
        "right": np.array([[0.0, 0.0, 0.0], [1.1, 0.0, 0.0], [0.0, 1.4, 0.0]]),
        "acute": np.array([[0.0, 0.0, 0.0], [3.49, 0.0, 0.0], [3.4 * np.cos(0.2), 3.4 * np.sin(0.2), 0.0]]),
    }
    for name, pos in cases.items():
        ctx = _ctx([1, 0, 2], weights, dtype=dtype, path="fused")
        dE, dF, F = _compare(ctx, pos, [1, 0, 2], weights, dtype)
        _say("trimer %s %s: |dE|/S %.2e max|dF| %.2e" % (name, dtype, dE, dF))
        assert dF <= TOL_F[dtype]
        assert np.abs(F.sum(axis=0)).max() <= 1e-6
        ctx.close()


@pytest.mark.parametrize("dtype,path", [("fp32", "fused"), ("bf16x3", "fused"), ("fp32", "plain")])
def test_batch_of_tiny_and_ragged_molecules(weights, dtype, path):
    """Molecules of 1, 2, 3, 22, 1 and 57 atoms in one context: per-molecule
    energies and forces equal the oracle's on each molecule alone."""
    rng = np.random.Generator(np.random.PCG64(71))
    sizes = [1, 2, 3, 22, 1, 57]
    pos, spec = [], []
    for k, n in enumerate(sizes):
        p = synth.rsa_ball(n, 100 + k) if n > 1 else np.zeros((1, 3))
        pos.append(p + 1000.0 * k)
        spec.append(rng.integers(0, 4, size=n).astype(np.int32))
    pos, spec = np.concatenate(pos), np.concatenate(spec)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    ctx = _ctx(spec, weights, dtype=dtype, path=path, mol_offsets=off)
    E, F = ctx.compute(pos)
    for m in range(len(sizes)):
        sl = slice(off[m], off[m + 1])
        Eo, Eio, Fo = oracle.energy_forces(pos[sl], spec[sl], weights)
        dE = abs(E[m] - Eo) / _scale(Eio)
        dF = np.abs(F[sl] - Fo).max()
        assert dF <= TOL_F[dtype], (m, dF)
        assert dE <= (1e-6 if dtype == "fp32" else 5e-5), (m, dE)
    _say("ragged batch %s %s ok" % (dtype, path))
    ctx.close()


@pytest.mark.parametrize("T,dtype", [(0, "fp32"), (5, "fp32"), (10, "fp32"), (12, "fp32"), (14, "fp32"),
                                     (15, "fp32"), (16, "bf16x3")])
def test_capacity_overflow_is_an_error(weights, T, dtype):
    """200 atoms packed into a 3 A ball: every atom has ~199 neighbours within
    5.2 A, beyond the 160 radial entries held per atom and the pair-list
    capacity; the evaluation completes with clamped lists and the call
    reports NNP_ERR_STATE with the observed maxima (one wave per atom, and
    10-atom tiles pooling the largest angular load, 96 entries per atom).
    Regression: neighbours past the radial capacity that lie within 3.5 A
    were once counted as angular entries without being written, so the
    adjoint read stale neighbour indices."""
    import paper_2412_18271_amd as P
    pos = synth.rsa_ball(200, 5, density=200 / (4.0 / 3.0 * np.pi * 27.0), d_min=0.3)
    assert np.sqrt(((pos[:, None] - pos[None]) ** 2).sum(-1)).max() < 6.2
    ctx = _ctx(np.zeros(200, np.int32), weights, dtype=dtype, path="fused", atoms_per_tile=T)
    with pytest.raises(P.NNPError) as ei:
        ctx.compute(pos)
    _say("overflow:", ei.value)
    assert "capacity exceeded" in str(ei.value)
    ctx.close()


def test_capacity_overflow_during_md_is_reported(weights):
    """The same packed ball advanced by MD steps: the steps themselves only
    enqueue work, and the energy log and the state then refuse to hand out
    results computed on clamped environments (NNP_ERR_STATE), while the
    counters still show the observed maxima."""
    import paper_2412_18271_amd as P
    pos = synth.rsa_ball(200, 5, density=200 / (4.0 / 3.0 * np.pi * 27.0), d_min=0.3)
    ctx = _ctx(np.zeros(200, np.int32), weights, dtype="bf16x3", path="fused")
    ctx.set_state(pos, np.zeros_like(pos))
    ctx.step(0.5, 3, graph=True)
    for call in (lambda: ctx.energy_log(4), ctx.get_state):
        with pytest.raises(P.NNPError) as ei:
            call()
        assert ei.value.status == 6 and "capacity exceeded" in str(ei.value), ei.value
    st = ctx.stats()
    _say("overflow in MD:", st)
    assert st["max_radial"] > 160 and st["steps"] == 3
    ctx.close()


@pytest.mark.parametrize("path", ["fused", "plain"])
def test_invalid_positions_are_rejected_and_context_recovers(weights, path):
    """NaN or infinite coordinates and two atoms at one point are rejected on
    the host before any device work (status NNP_ERR_NONFINITE = 2), both as
    the first positions a context sees and later, by compute and by
    set_state; valid positions then give the same result as before."""
    import paper_2412_18271_amd as P
    s = synth.make_config("mol22")

    def broken():
        for kind in ("nan", "inf", "coincident"):
            p = s.pos.copy()
            if kind == "nan":
                p[7, 1] = np.nan
            elif kind == "inf":
                p[3, 2] = -np.inf
            else:
                p[11] = p[4]
            yield kind, p

    fresh = P.Context.from_system(s, dtype="fp32", path=path)
    for kind, p in broken():
        with pytest.raises(P.NNPError) as ei:
            fresh.compute(p)
        assert ei.value.status == 2, (kind, ei.value)
    E0, F0 = fresh.compute(s.pos)
    Eo, Eio, Fo = oracle.energy_forces(s.pos, s.species, s.weights)
    assert np.abs(F0 - Fo).max() <= TOL_F["fp32"]
    for kind, p in broken():
        with pytest.raises(P.NNPError) as ei:
            fresh.compute(p)
        assert ei.value.status == 2, (kind, ei.value)
        with pytest.raises(P.NNPError) as ei:
            fresh.set_state(p, s.vel)
        assert ei.value.status == 2, (kind, ei.value)
        _say("%s positions rejected (%s path): %s" % (kind, path, ei.value))
    E1, F1 = fresh.compute(s.pos)
    assert E1[0] == E0[0] and np.array_equal(F1, F0)
    fresh.set_state(s.pos, s.vel)
    fresh.step(0.5, 5)
    x, _, _, _ = oracle.vv(s.pos, s.vel, s.masses, s.species, s.weights, 0.5, 5)
    assert np.abs(fresh.get_state()["pos"] - x).max() <= 1e-5
    fresh.close()
