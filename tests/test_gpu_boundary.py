"""Boundary behaviour through the C ABI on the GPU: the energy-only return
mode (the paper's energy-returning callable, Methods), graph pre-capture,
and checkpoint / resume of an MD run through nnp_get_state / nnp_set_state.
"""

import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ctx(system, **kw):
    import paper_2412_18271_amd as P
    return P.Context.from_system(system, **kw)


@pytest.mark.parametrize("name,dtype,path", [("mol22", "fp32", "fused"), ("cluster2500", "fp32", "fused"),
                                             ("cluster2500", "bf16x3", "fused"), ("mol22", "fp32", "plain")])
def test_energy_only_return_mode(make_system, name, dtype, path):
    """NNP_RETURN_ENERGY: the energy equals the oracle's, a forces argument
    is rejected, and the context's forces are never written by the
    energy-only evaluations (still zero from creation, and after a step the
    forces of that step stay untouched by a later energy-only call)."""
    import paper_2412_18271_amd as P
    s = make_system(name)
    Eo, Eio, Fo = oracle.energy_forces(s.pos, s.species, s.weights)
    S = np.abs(Eio).sum()
    tol = {"fp32": 1e-6, "bf16x3": 1e-5}[dtype]
    ctx = _ctx(s, dtype=dtype, path=path, return_mode="energy")
    E, F = ctx.compute(s.pos)
    assert F is None
    _say("%s %s %s energy only: |dE|/S %.2e" % (name, dtype, path, abs(E[0] - Eo) / S))
    assert abs(E[0] - Eo) / S <= tol
    with pytest.raises(P.NNPError) as ei:
        ctx.compute(s.pos, forces=True)
    assert ei.value.status == 1
    st = ctx.get_state()
    assert not np.any(st["forces"]), "an energy-only evaluation wrote forces"
    # MD still differentiates the energy (the adjoint inside the step)
    ctx.set_state(s.pos, s.vel)
    ctx.step(0.5, 3, graph=False)
    st1 = ctx.get_state()
    assert np.abs(st1["forces"]).max() > 0
    E2, _ = ctx.compute(s.pos)
    st2 = ctx.get_state()
    assert abs(E2[0] - Eo) / S <= tol
    assert np.array_equal(st1["forces"], st2["forces"])
    ctx.close()


def test_energy_only_device_call_rejects_forces(make_system):
    import torch
    import paper_2412_18271_amd as P
    s = make_system("mol22")
    ctx = _ctx(s, dtype="fp32", return_mode="energy")
    ctx.set_state(s.pos, s.vel)
    pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    e = torch.zeros(1, dtype=torch.float64, device="cuda")
    f = torch.zeros((s.n_atoms, 3), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    with pytest.raises(P.NNPError) as ei:
        ctx.compute_device(pos.data_ptr(), True, e.data_ptr(), f.data_ptr())
    assert ei.value.status == 1
    ctx.compute_device(pos.data_ptr(), True, e.data_ptr(), None)
    ctx.stats()  # synchronises the context stream
    Eo, Eio, _ = oracle.energy_forces(s.pos, s.species, s.weights, forces=False)
    assert abs(float(e[0]) - Eo) <= 1e-6 * np.abs(Eio).sum()
    ctx.close()


def test_capture_then_step_replays_same_trajectory(make_system):
    """nnp_capture changes no state; steps replayed from the pre-captured
    graphs equal eager steps bitwise (a block of 200 and a remainder of
    130: two graphs, and the tiles rebalanced between them)."""
    s = make_system("cluster2500")
    out = []
    for mode in ("eager", "captured"):
        ctx = _ctx(s, dtype="bf16x3", path="fused")
        ctx.set_state(s.pos, s.vel)
        ctx.step(0.5, 5, graph=mode == "captured")
        if mode == "captured":
            before = ctx.get_state()
            ctx.capture(0.5, 330)
            after = ctx.get_state()
            for k in ("pos", "vel", "forces"):
                assert np.array_equal(before[k], after[k])
            assert ctx.stats()["steps"] == 5
        ctx.step(0.5, 330, graph=mode == "captured")
        out.append(ctx.get_state())
        assert ctx.stats()["steps"] == 335
        ctx.close()
    for k in ("pos", "vel", "forces"):
        assert np.array_equal(out[0][k], out[1][k])


def test_checkpoint_resume_bitwise_when_tiling_is_kept(make_system):
    """22 atoms (tiles of 8, no rebalancing): 100 steps in one call equal 50
    steps, a checkpoint taken with nnp_get_state, 20 more steps thrown away,
    the checkpoint restored with nnp_set_state and 50 steps -- bitwise in
    positions, velocities and forces; the energies of the resumed half equal
    to the FP64 summation order of their per-wave sums."""
    s = make_system("mol22")
    a = _ctx(s, dtype="fp32", path="fused")
    a.set_state(s.pos, s.vel)
    a.step(0.5, 100)
    ref = a.get_state()
    Ua, Ka = a.energy_log(51)
    a.close()
    b = _ctx(s, dtype="fp32", path="fused")
    b.set_state(s.pos, s.vel)
    b.step(0.5, 50)
    chk = b.get_state()
    b.step(0.5, 20)
    b.set_state(chk["pos"], chk["vel"])
    b.step(0.5, 50)
    res = b.get_state()
    Ub, Kb = b.energy_log(51)
    b.close()
    for k in ("pos", "vel", "forces"):
        assert np.array_equal(ref[k], res[k]), k
    np.testing.assert_allclose(Ub, Ua, rtol=1e-12, atol=0)
    np.testing.assert_allclose(Kb, Ka, rtol=1e-12, atol=0)


def test_checkpoint_resume_in_fresh_context(make_system):
    """The checkpoint of step 50 restored in a new context (whose internal
    atom order comes from the checkpoint's positions, so sums run in another
    order): the resumed trajectory ends within the paper's 1e-3 A trajectory
    bar of the oracle's 100-step trajectory (golden fixture)."""
    import json
    import os
    s = make_system("mol22")
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "mol22_oracle.json")))
    b = _ctx(s, dtype="fp32", path="fused")
    b.set_state(s.pos, s.vel)
    b.step(0.5, 50)
    chk = b.get_state()
    b.close()
    c = _ctx(s, dtype="fp32", path="fused")
    c.set_state(chk["pos"], chk["vel"])
    c.step(0.5, 50)
    res = c.get_state()
    U, K = c.energy_log(51)
    c.close()
    dx = np.abs(res["pos"] - np.array(ref["final_positions"])).max()
    dU = np.abs(U[:, 0] - np.array(ref["U"][50:])).max()
    _say("fresh-context resume: max|dx| %.2e A, max|dU| %.2e eV vs the oracle" % (dx, dU))
    assert dx <= 1e-3
    assert dU <= 1e-5


def test_checkpoint_resume_large_cluster(make_system):
    """2,500 atoms, split BF16, 10-atom tiles rebalanced by work: resuming
    from a checkpoint restarts from the initial tiling, so the resumed half
    rounds its pooled sums at other places; the two runs agree to the
    trajectory bar (1e-3 A) and the resumed state's forces match the oracle
    at its positions."""
    s = make_system("cluster2500")
    a = _ctx(s, dtype="bf16x3", path="fused")
    a.set_state(s.pos, s.vel)
    a.step(0.5, 100)
    ref = a.get_state()
    a.close()
    b = _ctx(s, dtype="bf16x3", path="fused")
    b.set_state(s.pos, s.vel)
    b.step(0.5, 50)
    chk = b.get_state()
    b.set_state(chk["pos"], chk["vel"])
    b.step(0.5, 50)
    res = b.get_state()
    b.close()
    dx = np.abs(ref["pos"] - res["pos"]).max()
    Eo, Eio, Fo = oracle.energy_forces(res["pos"], s.species, s.weights)
    dF = np.abs(res["forces"] - Fo).max()
    _say("resume: max|dx| %.2e  max|dF| vs oracle %.2e" % (dx, dF))
    assert dx <= 1e-3
    assert dF <= 1e-3
