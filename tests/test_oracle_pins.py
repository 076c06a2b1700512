"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test names what fixes the expected value: a library routine, a closed
form, an invariance of the model, finite differences, or an exact discrete
solution.  All run on the CPU.
"""

import math

import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

import oracle
import synth

KAPPA = 9.64853321e-3


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------- O1 pairs

@pytest.mark.parametrize("rc", [3.5, 5.2, 6.2])
def test_pairs_equal_kdtree(rc):
    """Brute-force ordered pair sets equal scipy's k-d tree pair query."""
    s = synth.make_config("cluster2500", n=300, pos_seed=5)
    got = {tuple(p) for p in oracle.pairs(s.pos, rc).tolist()}
    und = cKDTree(s.pos).query_pairs(rc * (1 - 1e-12))
    want = {(i, j) for i, j in und} | {(j, i) for i, j in und}
    assert got == want
    assert len(got) > 0


# ------------------------------------------------------------ O2/O3 dimer

def _dimer(r, s0=0, s1=0):
    pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    return pos, np.array([s0, s1], np.int32)


@pytest.mark.parametrize("r", [0.9, 1.5, 2.6, 3.0, 5.1999])
def test_dimer_radial_closed_form(r):
    """Two atoms: one neighbour each, so every radial sum is one term and
    there are no angular triples."""
    pos, sp = _dimer(r, 0, 3)  # H and O
    G = oracle.descriptors(pos, sp)
    cut = 0.5 * math.cos(math.pi * r / 5.2) + 0.5
    centres = [0.9 + 0.28 * k for k in range(16)]
    term = np.array([math.exp(-16.0 * (r - c) ** 2) * cut for c in centres])
    # the H atom sees an O neighbour (block 3), the O atom an H neighbour (block 0)
    np.testing.assert_allclose(G[0, 48:64], term, rtol=1e-14, atol=1e-300)
    np.testing.assert_allclose(G[1, 0:16], term, rtol=1e-14, atol=1e-300)
    mask = np.ones(384, bool)
    mask[48:64] = False
    assert np.all(G[0, mask] == 0.0)
    mask = np.ones(384, bool)
    mask[0:16] = False
    assert np.all(G[1, mask] == 0.0)


def test_dimer_cutoff_special_points():
    """fc(Rc/2) = 1/2, fc(Rc/3) = 3/4, fc(2Rc/3) = 1/4, fc(Rc) = 0."""
    for r, fc in [(2.6, 0.5), (5.2 / 3, 0.75), (2 * 5.2 / 3, 0.25)]:
        pos, sp = _dimer(r)
        G = oracle.descriptors(pos, sp)
        k = int(np.argmin([abs(0.9 + 0.28 * k - r) for k in range(16)]))
        x = r - (0.9 + 0.28 * k)
        assert G[0, k] == pytest.approx(fc * math.exp(-16 * x * x), rel=1e-13)
    pos, sp = _dimer(5.2)
    assert np.all(oracle.descriptors(pos, sp) == 0.0)


# ----------------------------------------------------------- O4 trimer

def _trimer(r, theta_deg, sj=0, sk=1, si=2):
    t = math.radians(theta_deg)
    pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0], [r * math.cos(t), r * math.sin(t), 0.0]])
    return pos, np.array([si, sj, sk], np.int32)


@pytest.mark.parametrize("theta", [60.0, 90.0, 120.0, 180.0])
def test_trimer_angular_closed_form(theta):
    """Centre with two neighbours at equal distance: exactly one triple.
    The expected value uses the angle form (1 + cos(theta' - t_n))^32 with
    theta' = acos(0.95 cos theta), a different route from the oracle's."""
    r = 2.5
    pos, sp = _trimer(r, theta)  # centre N, neighbours H (j) and C (k)
    G = oracle.descriptors(pos, sp)
    cut = 0.5 * math.cos(math.pi * r / 3.5) + 0.5
    thp = math.acos(0.95 * math.cos(math.radians(theta)))
    want = np.zeros(32)
    for m in range(4):
        B = math.exp(-8.0 * (r - (0.9 + 0.65 * m)) ** 2)
        for n in range(8):
            A = (1.0 + math.cos(thp - (2 * n + 1) * math.pi / 16)) ** 32
            want[8 * m + n] = 2.0 ** -31 * A * B * cut * cut
    p = 1  # HC
    got = G[0, 64 + 32 * p:64 + 32 * p + 32]
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-300)
    other = np.ones(320, bool)
    other[32 * p:32 * p + 32] = False
    assert np.all(G[0, 64:][other] == 0.0)
    assert np.all(np.isfinite(G))


def test_trimer_swap_symmetry_and_neighbour_view():
    """Swapping the two neighbours leaves the centre's features unchanged;
    at 90 degrees and r = 2.5 the neighbours are 3.54 A apart, so they have
    no triple of their own."""
    pos, sp = _trimer(2.5, 90.0, sj=0, sk=1)
    pos2, sp2 = _trimer(2.5, 90.0, sj=1, sk=0)
    G1 = oracle.descriptors(pos, sp)
    G2 = oracle.descriptors(pos2, sp2)
    np.testing.assert_allclose(G1[0], G2[0], rtol=1e-14)
    assert np.all(G1[1:, 64:] == 0.0)


def test_collinear_is_finite_and_smooth():
    """Reading of the collinear case: scaling cos by 0.95 keeps the angular
    term smooth, so the gradient is finite at 180 degrees and the energy is
    symmetric about it."""
    w = synth.xavier_weights(0)
    sp = np.array([2, 0, 1], np.int32)
    Es = []
    for th in (179.0, 180.0, 181.0):
        pos, _ = _trimer(2.0, th)
        E, _, F = oracle.energy_forces(pos, sp, w)
        assert np.all(np.isfinite(F))
        Es.append(E)
    assert Es[0] == pytest.approx(Es[2], rel=1e-12)


# ------------------------------------------------------------ O5 network

def test_mlp_matches_torch_linear_celu():
    """The per-element network equals torch.nn.functional.linear + celu
    (alpha = 0.1) in float64, and its input gradient equals autograd's."""
    torch = pytest.importorskip("torch")
    w = synth.xavier_weights(3)
    rng = _rng(7)
    shapes = ((160, 384), (128, 160), (96, 128), (1, 96))
    per = sum(o * i + o for o, i in shapes)
    for e in range(4):
        G = rng.uniform(0.0, 2.0, 384)
        E, g = oracle.mlp(e, w, G)
        x = torch.tensor(G, dtype=torch.float64, requires_grad=True)
        off = e * per
        h = x
        for li, (o, i) in enumerate(shapes):
            W = torch.tensor(w[off:off + o * i], dtype=torch.float64).reshape(o, i)
            off += o * i
            b = torch.tensor(w[off:off + o], dtype=torch.float64)
            off += o
            h = torch.nn.functional.linear(h, W, b)
            if li < 3:
                h = torch.nn.functional.celu(h, alpha=0.1)
        h.sum().backward()
        assert E == pytest.approx(float(h.detach()), rel=1e-13, abs=1e-15)
        # torch's CELU backward rebuilds exp(z/alpha) from the layer output,
        # which loses relative accuracy for very negative z: allow 1e-8 of
        # the gradient's scale.
        gt = x.grad.numpy()
        assert np.max(np.abs(g - gt)) <= 1e-8 * np.max(np.abs(gt))


def test_mlp_bias_layout():
    """Biases sit right after their weight matrix: a blob whose only
    non-zero entry is b4 of one element gives E = b4 for that element and 0
    for the others."""
    shapes = ((160, 384), (128, 160), (96, 128), (1, 96))
    per = sum(o * i + o for o, i in shapes)
    for e in range(4):
        w = np.zeros(4 * per, np.float32)
        w[e * per + per - 1] = 0.75
        for q in range(4):
            E, _ = oracle.mlp(q, w, np.ones(384))
            assert E == (0.75 if q == e else 0.0)


# ------------------------------------------------------------ O7 forces

def _fd_forces(pos, sp, w, h=1e-4):
    F = np.zeros_like(pos)
    for a in range(pos.shape[0]):
        for c in range(3):
            p = pos.copy()
            p[a, c] += h
            Ep = oracle.energy_forces(p, sp, w, forces=False)[0]
            p[a, c] -= 2 * h
            Em = oracle.energy_forces(p, sp, w, forces=False)[0]
            F[a, c] = -(Ep - Em) / (2 * h)
    return F


@pytest.mark.parametrize("name,n", [("mol22", None), ("cluster2500", 48)])
def test_forces_central_difference(make_system, name, n):
    """Analytic forces equal central finite differences of the energy
    (h = 1e-4 A, truncation error ~1e-8 eV/A) to 1e-6 eV/A."""
    s = make_system(name) if n is None else synth.make_config(name, n=n, pos_seed=9)
    _, _, F = oracle.energy_forces(s.pos, s.species, s.weights)
    Ffd = _fd_forces(s.pos, s.species, s.weights)
    assert np.max(np.abs(F - Ffd)) < 1e-6
    assert np.max(np.abs(F)) > 1e-2


def test_forces_match_torch_autograd():
    """Energy and forces equal an independent float64 PyTorch statement of
    the model whose forces come from autograd (N = 10)."""
    pytest.importorskip("torch")
    from tests import torch_model
    s = synth.make_config("mol22", n=10, counts=(4, 3, 2, 1), cube=5.5, pos_seed=4)
    E, _, F = oracle.energy_forces(s.pos, s.species, s.weights)
    Et, Ft = torch_model.energy_forces(s.pos, s.species, s.weights)
    assert E == pytest.approx(Et, rel=1e-12, abs=1e-13)
    np.testing.assert_allclose(F, Ft, rtol=1e-9, atol=1e-11)


def test_forces_on_selected_atoms_and_local_environment(make_system):
    """Forces on chosen atoms, computed from the 10.4 A environment alone,
    equal the full-molecule forces (only E_i with r_ia < 5.2 depend on x_a
    and each of those depends only on atoms within 5.2 of i)."""
    s = make_system("cluster2500")
    _, _, F = oracle.energy_forces(s.pos, s.species, s.weights)
    sel = np.array([0, 17, 1333, 2499])
    np.testing.assert_allclose(oracle.forces_on(s.pos, s.species, s.weights, sel), F[sel],
                               rtol=1e-12, atol=1e-13)
    for a in sel:
        env = oracle.local_environment(s.pos, int(a), 10.4)
        loc = int(np.nonzero(env == a)[0][0])
        Fa = oracle.forces_on(s.pos[env], s.species[env], s.weights, [loc])[0]
        np.testing.assert_allclose(Fa, F[a], rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------- invariants

def test_invariances(make_system):
    """E is invariant under rigid motion and same-element permutation; the
    net force and net torque vanish."""
    s = make_system("cluster2500")
    sub = synth.make_config("cluster2500", n=400, pos_seed=13)
    pos, sp, w = sub.pos, sub.species, sub.weights
    E, Ei, F = oracle.energy_forces(pos, sp, w)
    S = np.abs(Ei).sum()
    assert np.linalg.norm(F.sum(0)) < 1e-10 * S
    assert np.linalg.norm(np.cross(pos, F).sum(0)) < 1e-10 * S * 10.0
    R = Rotation.random(random_state=3).as_matrix()
    shift = np.array([3.3, -1.7, 12.0])
    pos2 = pos @ R.T + shift
    E2, _, F2 = oracle.energy_forces(pos2, sp, w)
    assert abs(E2 - E) < 1e-12 * S
    np.testing.assert_allclose(F2, F @ R.T, atol=1e-10)
    rng = _rng(11)
    perm = np.arange(pos.shape[0])
    for e in range(4):
        idx = np.nonzero(sp == e)[0]
        perm[idx] = rng.permutation(idx)
    E3, _, F3 = oracle.energy_forces(pos[perm], sp[perm], w)
    assert abs(E3 - E) < 1e-12 * S
    np.testing.assert_allclose(F3, F[perm], atol=1e-12)
    assert s.n_atoms == 2500


# ------------------------------------------------------------ O8 VV

def test_vv_harmonic_exact_discrete_solution():
    """On E = sum x^2 (the paper's Model42) velocity Verlet is the linear
    recurrence x_{n+1} - 2 x_n + x_{n-1} = -(w dt)^2 x_n with w^2 = 2 kappa / m,
    solved exactly by A cos(n W dt) + B sin(n W dt), cos(W dt) = 1 - (w dt)^2 / 2."""
    rng = _rng(1)
    n, dt, steps = 6, 0.5, 400
    m = np.array([1.008, 12.011, 14.007, 15.999, 2.0, 40.0])
    x0 = rng.normal(size=(n, 3))
    v0 = rng.normal(size=(n, 3)) * 0.01
    x, v, U, K = oracle.vv(x0, v0, m, np.zeros(n, np.int32), None, dt, steps, model=1)
    w2 = 2.0 * KAPPA / m
    cosW = 1.0 - w2 * dt * dt / 2.0
    Wdt = np.arccos(cosW)
    x1 = x0 + dt * v0 + 0.5 * dt * dt * (-w2[:, None] * x0)
    B = (x1 - x0 * cosW[:, None]) / np.sin(Wdt)[:, None]
    xs = x0 * np.cos(steps * Wdt)[:, None] + B * np.sin(steps * Wdt)[:, None]
    np.testing.assert_allclose(x, xs, rtol=0, atol=1e-11)
    assert U[0] == pytest.approx((x0 ** 2).sum(), rel=1e-15)


def test_vv_energy_error_scales_as_dt_squared():
    """Second order: halving dt divides the energy-error amplitude by 4."""
    rng = _rng(2)
    n = 4
    m = np.array([1.008, 12.011, 14.007, 15.999])
    x0 = rng.normal(size=(n, 3))
    v0 = rng.normal(size=(n, 3)) * 0.02
    amp = []
    for dt, steps in ((1.0, 400), (0.5, 800)):
        _, _, U, K = oracle.vv(x0, v0, m, np.zeros(n, np.int32), None, dt, steps, model=1)
        H = U + K
        amp.append(np.max(np.abs(H - H[0])))
    assert amp[0] / amp[1] == pytest.approx(4.0, rel=0.1)


def test_vv_nve_network_drift_second_order(make_system):
    """The network model conserves H = U + K to second order in dt over
    50 fs of the 22-atom molecule."""
    s = make_system("mol22")
    amp = []
    for dt, steps in ((0.5, 100), (0.25, 200)):
        _, _, U, K = oracle.vv(s.pos, s.vel, s.masses, s.species, s.weights, dt, steps)
        H = U + K
        amp.append(np.max(np.abs(H - H[0])))
    assert amp[0] < 1e-3
    assert 3.0 < amp[0] / amp[1] < 5.0


# ------------------------------------------------- O9/O10 Langevin (BAOAB)

KB = 8.617333262e-5


@pytest.mark.parametrize("ctr,key", [
    ([1, 0, 0, 0], [0, 0]),
    ([42, 7, 3, 9], [123456789, 987654321]),
    ([2**63 + 5, 2**64 - 1, 17, 2**40], [2**64 - 1, 2**32 + 1]),
])
def test_philox_matches_numpy(ctr, key):
    """Philox4x64-10 equals numpy's independent implementation (which
    advances its counter by one before producing a block)."""
    g = np.random.Philox(counter=np.array([ctr[0] - 1] + ctr[1:], np.uint64), key=np.array(key, np.uint64))
    want = g.random_raw(4)
    np.testing.assert_array_equal(oracle.philox4x64(ctr, key), want)


def test_langevin_noise_is_independent_standard_normal():
    """Box-Muller values over 8,000 (atom, step) counters: moments of N(0, 1),
    Kolmogorov-Smirnov against the normal CDF, no correlation between the
    three components or between consecutive steps, a different seed gives
    different values."""
    from scipy import stats
    z = np.array([oracle.langevin_noise(11, a, s) for a in range(200) for s in range(40)])
    assert z.shape == (8000, 3)
    flat = z.ravel()
    assert abs(flat.mean()) < 0.03
    assert abs(flat.var() - 1.0) < 0.03
    assert abs(stats.kurtosis(flat, fisher=False) - 3.0) < 0.15
    assert stats.kstest(flat, "norm").pvalue > 1e-3
    c = np.corrcoef(z.T)
    assert np.abs(c - np.eye(3)).max() < 0.05
    zz = z.reshape(200, 40, 3)
    lag = (zz[:, 1:] * zz[:, :-1]).mean()
    assert abs(lag) < 0.03
    assert not np.allclose(oracle.langevin_noise(12, 0, 0), oracle.langevin_noise(11, 0, 0))
    assert np.array_equal(oracle.langevin_noise(11, 5, 9), zz[5, 9])


def test_langevin_without_friction_is_velocity_verlet(make_system):
    """friction 0: a = 1 and no noise, and the two half drifts make one whole
    drift, so BAOAB is velocity Verlet (to rounding)."""
    s = make_system("mol22")
    x1, v1, U1, K1 = oracle.langevin(s.pos, s.vel, s.masses, s.species, s.weights, 0.5, 100, 300.0, 0.0, 3)
    x2, v2, U2, K2 = oracle.vv(s.pos, s.vel, s.masses, s.species, s.weights, 0.5, 100)
    np.testing.assert_allclose(x1, x2, rtol=0, atol=1e-9)
    np.testing.assert_allclose(U1 + K1, U2 + K2, rtol=0, atol=1e-9)


def test_langevin_free_particles_are_ornstein_uhlenbeck():
    """No forces: v_{n+1} = a v_n + sqrt(1 - a^2) sigma z exactly, so from
    v = 0 the variance after n steps is (1 - a^{2n}) kT kappa / m, and the
    stationary lag-1 correlation is a = exp(-gamma dt).  Tolerances are
    four standard errors of the 18,000-value estimates."""
    n, dt, T, fric = 6000, 0.5, 300.0, 50.0
    rng = _rng(21)
    m = rng.uniform(1.0, 16.0, n)
    x0 = rng.normal(size=(n, 3))
    v0 = np.zeros((n, 3))
    a = math.exp(-fric * 1e-3 * dt)
    sp = np.zeros(n, np.int32)
    x, v, _, _ = oracle.langevin(x0, v0, m, sp, None, dt, 40, T, fric, 5, model=2)
    u = v / np.sqrt(KB * T * KAPPA / m)[:, None]
    assert u.var() == pytest.approx(1.0 - a ** 80, abs=0.037)
    x, v, _, _ = oracle.langevin(x, v, m, sp, None, dt, 160, T, fric, 5, first_step=40, model=2)
    _, v2, _, _ = oracle.langevin(x, v, m, sp, None, dt, 1, T, fric, 5, first_step=200, model=2)
    u, u2 = (w / np.sqrt(KB * T * KAPPA / m)[:, None] for w in (v, v2))
    assert u.var() == pytest.approx(1.0, abs=0.042)
    assert (u * u2).mean() / (u * u).mean() == pytest.approx(a, abs=0.007)


@pytest.mark.parametrize("dt", [2.0, 7.0])
def test_langevin_harmonic_configurations_exact(dt):
    """BAOAB samples the configurational Boltzmann distribution of a harmonic
    potential exactly at any stable step (Leimkuhler and Matthews 2013): on
    E = sum x^2, <x^2> = kT/2 per coordinate even at omega dt ~ 1, where
    splittings in another order are off by (omega dt / 2)^2 ~ 25 %.  The
    whole-step velocities carry the known bias <K> = 3/2 n kT (1 - (omega dt)^2 / 4)."""
    n, T, fric = 4000, 300.0, 20.0
    rng = _rng(22)
    m = np.ones(n)
    x = rng.normal(size=(n, 3)) * 0.1
    v = np.zeros((n, 3))
    sp = np.zeros(n, np.int32)
    x, v, _, _ = oracle.langevin(x, v, m, sp, None, dt, 300, T, fric, 7, model=1)
    xs, ks = [], []
    for blk in range(10):
        x, v, _, K = oracle.langevin(x, v, m, sp, None, dt, 30, T, fric, 7, first_step=300 + 30 * blk, model=1)
        xs.append((x ** 2).mean())
        ks.append(K[-1])
    wdt = math.sqrt(2.0 * KAPPA) * dt
    assert np.mean(xs) / (KB * T / 2) == pytest.approx(1.0, abs=0.02)
    assert np.mean(ks) / (1.5 * n * KB * T) == pytest.approx(1.0 - wdt ** 2 / 4, abs=0.02)


# -------------------------------------------------- periodic boxes (images)

def _supercell(pos, box, axis):
    shift = np.zeros(3)
    shift[axis] = box[axis]
    big = np.array(box, dtype=float)
    big[axis] *= 2
    return np.concatenate([pos, pos + shift]), big


def test_periodic_large_box_equals_gas_phase(make_system):
    """A molecule in a box much larger than its extent and the 10.4 A reach
    (shifted so that wrapping moves atoms across faces) has its gas-phase
    energy and forces."""
    s = make_system("mol22")
    pos = s.pos + np.array([-5.0, 37.0, 100.0])
    E, Ei, F = oracle.periodic_energy_forces(pos, s.species, s.weights, [60.0, 61.0, 62.0])
    Eg, Eig, Fg = oracle.energy_forces(s.pos, s.species, s.weights)
    assert E == pytest.approx(Eg, rel=1e-12)
    np.testing.assert_allclose(F, Fg, rtol=0, atol=1e-10)


@pytest.mark.parametrize("axis", [0, 2])
def test_periodic_supercell_is_two_copies(make_system, axis):
    """The box doubled along one axis with the atoms copied is the same
    crystal: twice the energy, the same forces on both copies.  A missing or
    doubly counted image breaks this."""
    s = make_system("box250")
    E1, Ei1, F1 = oracle.periodic_energy_forces(s.pos, s.species, s.weights, s.box)
    p2, b2 = _supercell(s.pos, s.box, axis)
    E2, Ei2, F2 = oracle.periodic_energy_forces(p2, np.concatenate([s.species, s.species]), s.weights, b2)
    assert E2 == pytest.approx(2 * E1, rel=1e-12)
    np.testing.assert_allclose(F2[:250], F1, rtol=0, atol=1e-10)
    np.testing.assert_allclose(F2[250:], F1, rtol=0, atol=1e-10)
    assert np.abs(F1).max() > 0.1


def test_periodic_forces_finite_differences(make_system):
    """Central differences of the periodic energy (h = 1e-4 A) moving one atom
    (the images follow through the wrap) equal the analytic forces."""
    s = make_system("box250")
    _, _, F = oracle.periodic_energy_forces(s.pos, s.species, s.weights, s.box)
    h = 1e-4
    for a in (0, 77, 249):
        for c in range(3):
            e = []
            for sign in (1, -1):
                p = s.pos.copy()
                p[a, c] += sign * h
                e.append(oracle.periodic_energy_forces(p, s.species, s.weights, s.box, forces=False)[0])
            assert -(e[0] - e[1]) / (2 * h) == pytest.approx(F[a, c], abs=2e-6)


def test_periodic_translation_and_net_force(make_system):
    """Translating every atom (any vector, wrapped or not) changes nothing;
    the forces sum to zero."""
    s = make_system("box250")
    E, Ei, F = oracle.periodic_energy_forces(s.pos, s.species, s.weights, s.box)
    E2, Ei2, F2 = oracle.periodic_energy_forces(s.pos + np.array([31.7, -5.2, 13.57 * 3 + 0.4]),
                                               s.species, s.weights, s.box)
    assert E2 == pytest.approx(E, rel=1e-12)
    np.testing.assert_allclose(F2, F, rtol=0, atol=1e-10)
    assert np.abs(F.sum(axis=0)).max() < 1e-9


def test_periodic_local_environment_matches_images(make_system):
    """For a box wider than 20.8 A, the gas-phase force on an atom among the
    nearest images within 10.4 A (the route the large-system GPU tests take)
    equals the explicit-image periodic force."""
    s = synth.make_config("box250", n=1000)
    assert s.box[0] > 20.8
    _, _, F = oracle.periodic_energy_forces(s.pos, s.species, s.weights, s.box)
    for a in (3, 500, 999):
        idx, x = oracle.periodic_local_environment(s.pos, s.box, a, 10.4)
        loc = int(np.nonzero(idx == a)[0][0])
        Fa = oracle.forces_on(x, s.species[idx], s.weights, [loc])[0]
        np.testing.assert_allclose(Fa, F[a], rtol=0, atol=1e-11)


def test_two_force_providers_add(make_system):
    """Model 3 (network plus the harmonic sum x^2 as a second force provider):
    the starting energy is the sum of the two providers' energies, and the
    combined NVE dynamics conserves H to second order in dt."""
    s = make_system("mol22")
    x = s.pos - s.pos.mean(axis=0)
    _, _, U, K = oracle.vv(x, s.vel, s.masses, s.species, s.weights, 0.5, 0, model=3)
    E = oracle.energy_forces(x, s.species, s.weights, forces=False)[0]
    assert U[0] == pytest.approx(E + (x ** 2).sum(), rel=1e-14)
    amp = []
    for dt, steps in ((0.5, 100), (0.25, 200)):
        _, _, U, K = oracle.vv(x, s.vel, s.masses, s.species, s.weights, dt, steps, model=3)
        amp.append(np.max(np.abs(U + K - U[0] - K[0])))
    assert 3.0 < amp[0] / amp[1] < 5.0


def test_periodic_vv_large_box_equals_gas_phase_vv(make_system):
    """The periodic velocity-Verlet loop in a box far wider than the 10.4 A
    reach (the molecule straddling a face, so that wrapping moves atoms
    across it) follows the gas-phase velocity Verlet of the C oracle, which
    the harmonic closed form pins: positions, velocities, potential and
    kinetic energy at every step.  A wrong kick order, a missing half kick or
    a wrong kinetic-energy unit breaks it."""
    s = make_system("mol22")
    pos = s.pos + np.array([-5.0, 37.0, 100.0])
    box = [60.0, 61.0, 62.0]
    x, v, U, K = oracle.periodic_vv(pos, s.vel, s.masses, s.species, s.weights, box, 0.5, 12)
    xg, vg, Ug, Kg = oracle.vv(pos, s.vel, s.masses, s.species, s.weights, 0.5, 12)
    assert U.shape == Ug.shape == (13,) and K.shape == Kg.shape == (13,)
    np.testing.assert_allclose(x, xg, rtol=0, atol=1e-10)
    np.testing.assert_allclose(v, vg, rtol=0, atol=1e-10)
    np.testing.assert_allclose(U, Ug, rtol=0, atol=1e-10)
    np.testing.assert_allclose(K, Kg, rtol=0, atol=1e-10)
    assert np.abs(x - pos).max() > 1e-3  # the atoms did move
