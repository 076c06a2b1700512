"""The allocation-free stored-mode entry point (nnp_energy_device_static)
against the allocating one (nnp_energy_device with keep = 1), through the C
ABI: two calls in a row, the second on a smaller system, each equal to the
allocating call bitwise (same kernels, same inputs) and within the network
dtype's tolerance of the FP64 oracle; a reused scratch and a system above
the size limit are rejected."""

import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

TOL = {"fp32": (1e-6, 1e-4), "bf16x3": (1e-5, 1e-3)}  # |dE|/S, max|dF| (eV/A)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _device_call(ctx, s, static):
    import torch
    pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    F = torch.zeros((s.n_atoms, 3), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    if static:
        ctx.energy_device_static(pos.data_ptr(), True, E.data_ptr())
    else:
        ctx.energy_device(pos.data_ptr(), True, E.data_ptr(), True)
    ctx.forces_device(F.data_ptr())
    ctx.get_state()  # synchronises the context stream and checks device flags
    return E.cpu().numpy().copy(), F.cpu().numpy().copy()


@pytest.mark.parametrize("dtype", ["fp32", "bf16x3"])
def test_static_scratch_matches_allocating_entry_point(make_system, dtype):
    import paper_2412_18271_amd as P
    for name in ("cluster2500", "mol22"):  # the second call is smaller
        s = make_system(name)
        _say("static scratch: %s (%d atoms) %s" % (name, s.n_atoms, dtype))
        Eo, Eio, Fo = oracle.energy_forces(s.pos, s.species, s.weights)
        S = np.abs(Eio).sum()
        with P.Context.from_system(s, dtype=dtype, path="fused") as ctx:
            ctx.set_state(s.pos, s.vel)
            E_s, F_s = _device_call(ctx, s, static=True)
            E_a, F_a = _device_call(ctx, s, static=False)
            E_s2, F_s2 = _device_call(ctx, s, static=True)
        dE, dF = abs(E_s[0] - Eo) / S, float(np.abs(F_s - Fo).max())
        _say("  |dE|/S %.2e max|dF| %.2e" % (dE, dF))
        assert np.array_equal(F_s, F_a) and np.array_equal(F_s2, F_a)
        np.testing.assert_allclose(E_s, E_a, rtol=1e-12, atol=0)
        np.testing.assert_allclose(E_s2, E_a, rtol=1e-12, atol=0)
        tol_e, tol_f = TOL[dtype]
        assert dE <= tol_e and dF <= tol_f


def test_static_scratch_reuse_and_size_limit(make_system):
    import torch
    import paper_2412_18271_amd as P
    a_sys, b_sys = make_system("mol22"), make_system("cluster2500")
    a = P.Context.from_system(a_sys, dtype="fp32", path="fused")
    b = P.Context.from_system(b_sys, dtype="fp32", path="fused")
    try:
        for c, s in ((a, a_sys), (b, b_sys)):
            c.set_state(s.pos, s.vel)
        pa = torch.tensor(a_sys.pos, dtype=torch.float64, device="cuda")
        pb = torch.tensor(b_sys.pos, dtype=torch.float64, device="cuda")
        E = torch.zeros(1, dtype=torch.float64, device="cuda")
        F = torch.zeros((a_sys.n_atoms, 3), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        a.energy_device_static(pa.data_ptr(), True, E.data_ptr())
        b.energy_device_static(pb.data_ptr(), True, E.data_ptr())
        with pytest.raises(P.NNPError) as ei:
            a.forces_device(F.data_ptr())  # b's call replaced a's kept data
        assert ei.value.status == 6
        a.get_state()
        b.get_state()
    finally:
        a.close()
        b.close()
    big = make_system("cluster23k")
    with P.Context.from_system(big, dtype="fp32", path="fused") as c:
        c.set_state(big.pos, big.vel)
        p = torch.tensor(big.pos, dtype=torch.float64, device="cuda")
        E = torch.zeros(1, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        with pytest.raises(P.NNPError) as ei:
            c.energy_device_static(p.data_ptr(), True, E.data_ptr())
        assert ei.value.status == 1 and "8192" in ei.value.message
