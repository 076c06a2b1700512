"""The split evaluation (descriptor kernel -> G in HBM, network over wide
same-element tiles -> dE/dG in HBM, adjoint kernel) against the FP64 oracle
through the C ABI, at every descriptor-tile and network-tile size, and the
autotuner that picks between it and the fused kernel.

Tolerances are those of the fused path's network dtypes: split BF16
|dE|/S <= 1e-5, max|dF| <= 1e-3 eV/A, |dE_i| <= 1e-4 eV; single-pass BF16
max|dF| <= 3e-2 eV/A, |dE_i| <= 2e-2 eV (reported, not the 1e-2 bar).  The
split mode's backward takes celu'(z) from h = celu(z) held as hi + lo BF16
(relative 2^-17), which adds at most ~1e-6 relative to a derivative: inside
the same bars.
"""

import json
import os
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

# single-pass BF16: the total energy is reported, not gated (as for the
# fused path); forces and per-atom energies keep the fused path's bars
TOL = {"bf16x3": dict(E=1e-5, F=1e-3, Ei=1e-4), "bf16": dict(E=float("inf"), F=3e-2, Ei=2e-2)}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ctx(system, **kw):
    import paper_2412_18271_amd as P
    return P.Context.from_system(system, **kw)


_ORACLE = {}


def _oracle(s):
    if s.name not in _ORACLE:
        _ORACLE[s.name] = oracle.system_energy_forces(s)
    return _ORACLE[s.name]


@pytest.mark.parametrize("dtype,T,nt", [("bf16x3", 5, 64), ("bf16x3", 4, 32), ("bf16x3", 7, 48),
                                        ("bf16x3", 10, 16), ("bf16x3", 0, 0), ("bf16", 5, 64), ("bf16", 10, 32)])
@pytest.mark.parametrize("name", ["mol22", "cluster2500"])
def test_split_energy_forces_match_oracle(make_system, name, dtype, T, nt):
    s = make_system(name)
    Eo, Eio, Fo = _oracle(s)
    _say("split", name, dtype, "tile", T, "network tile", nt)
    with _ctx(s, path="split", dtype=dtype, atoms_per_tile=T, network_tile=nt) as ctx:
        E, F = ctx.compute(s.pos)
        Ei = ctx.atom_energies()
    S = np.abs(Eio).sum()
    dE, dF, dEi = abs(E.sum() - Eo.sum()) / S, np.abs(F - Fo).max(), np.abs(Ei - Eio).max()
    _say("  |dE|/S %.3e  max|dF| %.3e  max|dEi| %.3e" % (dE, dF, dEi))
    t = TOL[dtype]
    assert dE <= t["E"] and dF <= t["F"] and dEi <= t["Ei"]


def test_split_energy_only_and_md_graph_equals_eager(make_system):
    """Energy-only evaluation (network forward alone) equals the oracle's
    energy; 60 MD steps from a graph and launched one by one are bitwise
    equal (same tiles, same rebalancing) and end within 1e-3 A of the
    oracle's trajectory of the 22-atom molecule."""
    s = make_system("mol22")
    Eo, _, _ = _oracle(s)
    with _ctx(s, path="split", dtype="bf16x3", return_mode="energy") as ctx:
        E, F = ctx.compute(s.pos)
        assert F is None and abs(E.sum() - Eo.sum()) <= 1e-5 * np.abs(_oracle(s)[1]).sum()
    out = []
    for graph in (True, False):
        with _ctx(s, path="split", dtype="bf16x3") as ctx:
            ctx.set_state(s.pos, s.vel)
            ctx.step(0.5, 60, graph=graph)
            out.append(ctx.get_state())
    for k in ("pos", "vel", "forces"):
        assert np.array_equal(out[0][k], out[1][k]), k
    x, v, U, K = oracle.vv(s.pos, s.vel, s.masses, s.species, s.weights, 0.5, 60)
    dx = np.abs(out[0]["pos"] - x).max()
    _say("  60 steps: max|dx| vs oracle %.2e" % dx)
    assert dx <= 1e-3


def test_split_cluster23k_sampled_and_md(make_system):
    """23,000 atoms (cell lists): energy and 48 sampled atoms against the
    oracle on their exact local environments, then 40 MD steps with
    rebuilds and 24 sampled atoms at the new positions."""
    from tests.test_gpu_large import _check_sampled
    s = make_system("cluster23k")
    with _ctx(s, path="split", dtype="bf16x3") as ctx:
        E, F = ctx.compute(s.pos)
        Eo, Eio, _ = oracle.energy_forces(s.pos, s.species, s.weights, forces=False)
        dE = abs(E[0] - Eo) / np.abs(Eio).sum()
        _say("split cluster23k |dE|/S %.3e" % dE)
        assert dE <= 1e-5
        _check_sampled(ctx, s, s.pos, F, "bf16x3", 48, 7)
        ctx.set_state(s.pos, s.vel)
        ctx.step(0.5, 40, graph=True)
        st = ctx.get_state()
        assert ctx.stats()["rebuilds"] >= 2
        E2, F2 = ctx.compute(st["pos"])
        _check_sampled(ctx, s, st["pos"], F2, "bf16x3", 24, 8)


def test_split_batch256_per_molecule(make_system):
    s = make_system("batch256")
    Eo, Eio, Fo = _oracle(s)
    with _ctx(s, path="split", dtype="bf16x3") as ctx:
        E, F = ctx.compute(s.pos)
        Ei = ctx.atom_energies()
    Sm = np.array([np.abs(Eio[s.molecule(m)]).sum() for m in range(s.n_molecules)])
    dE = (np.abs(E - Eo) / Sm).max()
    dF = np.abs(F - Fo).max()
    dEi = np.abs(Ei - Eio).max()
    _say("split batch256: max per-molecule |dE|/S %.3e  max|dF| %.3e  max|dEi| %.3e" % (dE, dF, dEi))
    assert dE <= 5e-5 and dF <= 1e-3 and dEi <= 1e-4


def test_split_periodic_box(make_system):
    s = make_system("box2500")
    _, _, F_ref = oracle.periodic_energy_forces(s.pos, s.species, s.weights, s.box)
    with _ctx(s, path="split", dtype="bf16x3") as ctx:
        _, F = ctx.compute(s.pos)
    dF = np.abs(F - F_ref).max()
    _say("split box2500 max|dF| %.3e" % dF)
    assert dF <= 1e-3


def test_autotune_cache_roundtrip_and_parity(make_system, tmp_path):
    """nnp_autotune times the fused and split configurations, writes its
    choice to the cache, a second context of the same size bucket reads it
    back without timing, and the tuned context still matches the oracle."""
    s = make_system("cluster2500")
    Eo, Eio, Fo = _oracle(s)
    cache = str(tmp_path / "tune.jsonl")
    with _ctx(s, path="fused", dtype="bf16x3") as ctx:
        ctx.set_state(s.pos, s.vel)
        ch = ctx.autotune(cache)
        _say("autotune choice", ch)
        assert not ch["from_cache"] and ch["path"] in ("fused", "split")
        E, F = ctx.compute(s.pos)
        assert np.abs(F - Fo).max() <= 1e-3
    lines = [json.loads(x) for x in open(cache)]
    assert len(lines) == 1
    rec = lines[0]
    _say("cache line", rec)
    assert rec["atoms_per_tile"] == ch["atoms_per_tile"] and rec["network_tile"] == ch["network_tile"]
    assert len(rec["ms_per_eval"]) >= 10  # fused tiles and split (tile x network tile) pairs
    with _ctx(s, path="fused", dtype="bf16x3") as ctx:
        ctx.set_state(s.pos, s.vel)
        ch2 = ctx.autotune(cache)
        assert ch2["from_cache"]
        assert (ch2["path"], ch2["atoms_per_tile"], ch2["network_tile"]) == (ch["path"], ch["atoms_per_tile"],
                                                                             ch["network_tile"])
        E2, F2 = ctx.compute(s.pos)
        assert np.abs(F2 - Fo).max() <= 1e-3
        ctx.set_state(s.pos, s.vel)
        ctx.step(0.5, 20)
        assert np.all(np.isfinite(ctx.get_state()["pos"]))
    assert len(open(cache).readlines()) == 1


@pytest.mark.parametrize("mode", ["recompute", "store"])
def test_split_autograd_matches_oracle(make_system, mode):
    """torch.autograd over the split path (the recompute mode runs the three
    split kernels forward and again with the adjoint; the stored mode keeps
    G and dE/dG) against the oracle's analytic gradient."""
    import torch
    from paper_2412_18271_amd.autograd import NNPModel
    s = make_system("cluster2500")
    _, Eio, Fo = _oracle(s)
    model = NNPModel.from_system(s, dtype="bf16x3", mode=mode, path="split", atoms_per_tile=5, network_tile=32)
    pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda", requires_grad=True)
    E = model(pos)
    E.sum().backward()
    torch.cuda.synchronize()
    dF = np.abs(-pos.grad.cpu().numpy() - Fo).max()
    _say("split autograd %s: max|grad + F| %.2e" % (mode, dF))
    assert dF <= 1e-3


def test_split_langevin_graph_equals_eager(make_system):
    """Langevin (BAOAB) steps on the split path: graph replay and launches one
    by one give bitwise equal trajectories across two calls (rebalancing and
    work order between blocks included)."""
    s = make_system("cluster2500")
    out = []
    for graph in (False, True):
        with _ctx(s, path="split", dtype="bf16x3") as ctx:
            ctx.set_state(s.pos, s.vel)
            ctx.set_thermostat(300.0, 0.1, 5)
            ctx.step(0.5, 120, graph=graph)
            ctx.step(0.5, 90, graph=graph)
            out.append(ctx.get_state())
    assert np.array_equal(out[0]["pos"], out[1]["pos"])
    assert np.array_equal(out[0]["vel"], out[1]["vel"])


def _expected_default_tile(species, dtype, ncu):
    """The documented default of the fused path: the smallest of 8, 10, 12-15
    (16 with the BF16 networks) atoms per tile that gives one workgroup per
    CU, else the one of 10, 12-15 (16) with the fewest rounds of one tile per
    CU times (21 + T) microseconds."""
    tmax = 16 if dtype in ("bf16", "bf16x3") else 15

    def tiles(T):
        return sum(-(-int((species == e).sum()) // T) for e in range(4))

    for T in (8, 10, 12, 13, 14, 15, 16):
        if T <= tmax and tiles(T) <= ncu:
            return T
    cands = [T for T in (10, 12, 13, 14, 15, 16) if T <= tmax]
    return min(cands, key=lambda T: (-(-tiles(T) // ncu) * (21 + T), cands.index(T)))


@pytest.mark.parametrize("name,dtype", [("mol22", "bf16x3"), ("cluster2500", "bf16x3"), ("cluster23k", "bf16x3"),
                                        ("cluster23k", "fp32"), ("batch256", "bf16x3"), ("batch256", "fp32")])
def test_default_tile_choice(make_system, name, dtype):
    """atoms_per_tile 0: the fused path's tile size, chosen when the positions
    are first set, follows the documented rule for this device's CU count."""
    import torch
    s = make_system(name)
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    with _ctx(s, path="fused", dtype=dtype) as ctx:
        ctx.set_state(s.pos, s.vel)
        cfg = ctx.config()
    T = _expected_default_tile(s.species, dtype, ncu)
    _say("default tile", name, dtype, cfg, "expected", T, "CUs", ncu)
    assert cfg["path"] == "fused" and cfg["atoms_per_tile"] == T
