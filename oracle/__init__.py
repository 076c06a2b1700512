"""FP64 CPU oracle (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use
this package.  It wraps ``nnp_oracle.c`` (plain C, IEEE double, OpenMP over
atoms) through ctypes and shares nothing with the HIP path.  Every function
operates on ONE molecule; callers loop over molecules of a batch.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nnp_oracle.c")
_SO = os.path.join(_HERE, "libnnp_oracle.so")
_lib = None

NFEAT = 384
RC_RAD = 5.2
RC_ANG = 3.5


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE semantics: no fast-math)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build(force=False)
    lib = ctypes.CDLL(_SO)
    P = ctypes.POINTER
    d, i, f = ctypes.c_double, ctypes.c_int, ctypes.c_float
    lib.oracle_pairs.restype = ctypes.c_long
    lib.oracle_pairs.argtypes = [i, P(d), d, P(i), P(i), ctypes.c_long]
    lib.oracle_descriptors.restype = None
    lib.oracle_descriptors.argtypes = [i, P(d), P(i), P(d)]
    lib.oracle_mlp.restype = None
    lib.oracle_mlp.argtypes = [i, P(f), P(d), P(d), P(d)]
    lib.oracle_energy_forces.restype = d
    lib.oracle_energy_forces.argtypes = [i, P(d), P(i), P(f), P(d), P(d)]
    lib.oracle_forces_on.restype = None
    lib.oracle_forces_on.argtypes = [i, P(d), P(i), P(f), i, P(i), P(d)]
    lib.oracle_vv.restype = None
    lib.oracle_vv.argtypes = [i, P(d), P(d), P(d), P(i), P(f), i, d, i, P(d), P(d)]
    u64, i64 = ctypes.c_uint64, ctypes.c_int64
    lib.oracle_philox4x64.restype = None
    lib.oracle_philox4x64.argtypes = [P(u64), P(u64), P(u64)]
    lib.oracle_langevin_noise.restype = None
    lib.oracle_langevin_noise.argtypes = [u64, i64, i64, P(d)]
    lib.oracle_langevin.restype = None
    lib.oracle_langevin.argtypes = [i, P(d), P(d), P(d), P(i), P(f), i, d, i, d, d, u64, i64, i64, P(d), P(d)]
    lib.oracle_threads.restype = i
    lib.oracle_threads.argtypes = []
    lib.oracle_set_threads.restype = None
    lib.oracle_set_threads.argtypes = [i]
    _lib = lib
    return lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _pos(p):
    return np.ascontiguousarray(p, dtype=np.float64).reshape(-1, 3)


def _sp(s):
    return np.ascontiguousarray(s, dtype=np.int32)


def _w(w):
    w = np.ascontiguousarray(w, dtype=np.float32)
    return w


def threads() -> int:
    return int(_load().oracle_threads())


def set_threads(t: int) -> None:
    _load().oracle_set_threads(int(t))


def pairs(pos, rc: float) -> np.ndarray:
    """Ordered pairs (i, j), i != j, r_ij < rc, lexicographic; shape (P, 2)."""
    lib = _load()
    p = _pos(pos)
    n = p.shape[0]
    cnt = lib.oracle_pairs(n, _ptr(p, ctypes.c_double), rc, None, None, 0)
    oi = np.empty(max(cnt, 1), np.int32)
    oj = np.empty(max(cnt, 1), np.int32)
    lib.oracle_pairs(n, _ptr(p, ctypes.c_double), rc, _ptr(oi, ctypes.c_int),
                     _ptr(oj, ctypes.c_int), cnt)
    return np.stack([oi[:cnt], oj[:cnt]], axis=1)


def descriptors(pos, species) -> np.ndarray:
    lib = _load()
    p, s = _pos(pos), _sp(species)
    G = np.zeros((p.shape[0], NFEAT), np.float64)
    lib.oracle_descriptors(p.shape[0], _ptr(p, ctypes.c_double), _ptr(s, ctypes.c_int),
                           _ptr(G, ctypes.c_double))
    return G


def mlp(element: int, weights, G) -> Tuple[float, np.ndarray]:
    """Energy of one atom and its gradient with respect to the 384 features."""
    lib = _load()
    G = np.ascontiguousarray(G, dtype=np.float64)
    E = np.zeros(1, np.float64)
    g = np.zeros(NFEAT, np.float64)
    w = _w(weights)
    lib.oracle_mlp(int(element), _ptr(w, ctypes.c_float), _ptr(G, ctypes.c_double),
                   _ptr(E, ctypes.c_double), _ptr(g, ctypes.c_double))
    return float(E[0]), g


def energy_forces(pos, species, weights, forces: bool = True):
    """Returns (E, E_i[n], F[n,3] or None) for one molecule."""
    lib = _load()
    p, s, w = _pos(pos), _sp(species), _w(weights)
    n = p.shape[0]
    Ei = np.zeros(n, np.float64)
    F = np.zeros((n, 3), np.float64) if forces else None
    E = lib.oracle_energy_forces(n, _ptr(p, ctypes.c_double), _ptr(s, ctypes.c_int),
                                 _ptr(w, ctypes.c_float), _ptr(Ei, ctypes.c_double),
                                 _ptr(F, ctypes.c_double) if forces else None)
    return float(E), Ei, F


def forces_on(pos, species, weights, sel) -> np.ndarray:
    lib = _load()
    p, s, w = _pos(pos), _sp(species), _w(weights)
    sel = np.ascontiguousarray(sel, dtype=np.int32)
    F = np.zeros((sel.shape[0], 3), np.float64)
    lib.oracle_forces_on(p.shape[0], _ptr(p, ctypes.c_double), _ptr(s, ctypes.c_int),
                         _ptr(w, ctypes.c_float), sel.shape[0], _ptr(sel, ctypes.c_int),
                         _ptr(F, ctypes.c_double))
    return F


def vv(pos, vel, masses, species, weights, dt: float, nsteps: int, model: int = 0):
    """NVE velocity Verlet.  model 0 = network, 1 = harmonic sum(x^2), 2 = no
    force, 3 = network plus harmonic.  Returns (x, v, U[nsteps+1], K[nsteps+1])."""
    lib = _load()
    x = _pos(pos).copy()
    v = _pos(vel).copy()
    m = np.ascontiguousarray(masses, dtype=np.float64)
    s = _sp(species)
    w = _w(weights) if weights is not None else np.zeros(1, np.float32)
    U = np.zeros(nsteps + 1, np.float64)
    K = np.zeros(nsteps + 1, np.float64)
    lib.oracle_vv(x.shape[0], _ptr(x, ctypes.c_double), _ptr(v, ctypes.c_double),
                  _ptr(m, ctypes.c_double), _ptr(s, ctypes.c_int), _ptr(w, ctypes.c_float),
                  int(model), float(dt), int(nsteps), _ptr(U, ctypes.c_double),
                  _ptr(K, ctypes.c_double))
    return x, v, U, K


def philox4x64(counter, key) -> np.ndarray:
    """Philox4x64-10 block of a 4-word counter under a 2-word key (O10)."""
    lib = _load()
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    lib.oracle_philox4x64(_ptr(c, ctypes.c_uint64), _ptr(k, ctypes.c_uint64), _ptr(out, ctypes.c_uint64))
    return out


def langevin_noise(seed: int, atom: int, step: int) -> np.ndarray:
    """The three standard normal values of caller atom `atom` in step `step` (O10)."""
    lib = _load()
    z = np.zeros(3, np.float64)
    lib.oracle_langevin_noise(int(seed), int(atom), int(step), _ptr(z, ctypes.c_double))
    return z


def langevin(pos, vel, masses, species, weights, dt: float, nsteps: int, temperature: float,
             friction: float, seed: int, first_index: int = 0, first_step: int = 0, model: int = 0):
    """BAOAB Langevin dynamics (O9): friction in 1/ps, temperature in K.
    model 0 = network, 1 = harmonic sum(x^2), 2 = no force.
    Returns (x, v, U[nsteps+1], K[nsteps+1])."""
    lib = _load()
    x = _pos(pos).copy()
    v = _pos(vel).copy()
    m = np.ascontiguousarray(masses, dtype=np.float64)
    s = _sp(species)
    w = _w(weights) if weights is not None else np.zeros(1, np.float32)
    U = np.zeros(nsteps + 1, np.float64)
    K = np.zeros(nsteps + 1, np.float64)
    lib.oracle_langevin(x.shape[0], _ptr(x, ctypes.c_double), _ptr(v, ctypes.c_double),
                        _ptr(m, ctypes.c_double), _ptr(s, ctypes.c_int), _ptr(w, ctypes.c_float),
                        int(model), float(dt), int(nsteps), float(temperature), float(friction),
                        int(seed), int(first_index), int(first_step), _ptr(U, ctypes.c_double),
                        _ptr(K, ctypes.c_double))
    return x, v, U, K


def local_environment(pos, centre: int, radius: float) -> np.ndarray:
    """Indices (ascending) of atoms closer than ``radius`` to atom ``centre``,
    the centre included.  Any quantity of the centre that depends only on
    atoms within that radius is reproduced exactly on this subset."""
    p = _pos(pos)
    d = np.sqrt(((p - p[centre]) ** 2).sum(axis=1))
    return np.nonzero(d < radius)[0].astype(np.int64)


KAPPA = 9.64853321e-3  # A fs^-2 per eV A^-1 amu^-1


def periodic_images(pos, box, reach: float):
    """Explicit periodic images of an orthorhombic box: the n atoms wrapped
    into [0, L) first (in input order), then every translated copy (integer
    multiples of the edges) lying closer than ``reach`` to the box.
    Returns (positions, index of the original atom of each row)."""
    p = _pos(pos)
    L = np.asarray(box, dtype=np.float64).reshape(3)
    n = p.shape[0]
    w = p - L * np.floor(p / L)
    k = [int(np.ceil(reach / L[d])) for d in range(3)]
    xs, ids = [w], [np.arange(n)]
    for sx in range(-k[0], k[0] + 1):
        for sy in range(-k[1], k[1] + 1):
            for sz in range(-k[2], k[2] + 1):
                if sx == 0 and sy == 0 and sz == 0:
                    continue
                q = w + np.array([sx, sy, sz]) * L
                out = np.maximum(0.0, np.maximum(-q, q - L))
                keep = np.sqrt((out * out).sum(axis=1)) < reach
                xs.append(q[keep])
                ids.append(np.nonzero(keep)[0])
    return np.concatenate(xs), np.concatenate(ids)


def periodic_energy_forces(pos, species, weights, box, forces: bool = True):
    """(E, E_i[n], F[n,3] or None) of the infinite periodic system built from
    the orthorhombic box ``box`` (edges in A).  Explicit images, no minimum
    image convention: E_i of an atom in the box is its gas-phase E_i among
    all images within 5.2 A; the force on atom a is minus the derivative of
    the energies of every atom of the crystal with respect to x_a alone
    (moving a together with its images changes sum_i E_i over the box by
    exactly that amount, by translation symmetry), i.e. the gather-form force
    on a among all images within 10.4 A, each of whose energies is complete."""
    sp = _sp(species)
    n = sp.shape[0]
    x5, i5 = periodic_images(pos, box, RC_RAD)
    _, Ei, _ = energy_forces(x5, sp[i5], weights, forces=False)
    Ei = Ei[:n].copy()
    F = None
    if forces:
        x10, i10 = periodic_images(pos, box, 2.0 * RC_RAD)
        F = forces_on(x10, sp[i10], weights, np.arange(n))
    return float(Ei.sum()), Ei, F


def periodic_local_environment(pos, box, centre: int, radius: float):
    """Atoms whose nearest image lies closer than ``radius`` to atom ``centre``
    (radius <= half the shortest edge, so the nearest image is the only one),
    the centre included.  Returns (indices ascending, positions of those
    nearest images, the centre at its own position)."""
    p = _pos(pos)
    L = np.asarray(box, dtype=np.float64).reshape(3)
    assert radius <= 0.5 * L.min()
    d = p - p[centre]
    d -= L * np.round(d / L)
    idx = np.nonzero(np.sqrt((d * d).sum(axis=1)) < radius)[0]
    return idx, p[centre] + d[idx]


def periodic_vv(pos, vel, masses, species, weights, box, dt: float, nsteps: int):
    """Velocity Verlet (O8) in the periodic box; positions stay unwrapped.
    Returns (x, v, U[nsteps+1], K[nsteps+1])."""
    x = _pos(pos).copy()
    v = _pos(vel).copy()
    m = np.asarray(masses, dtype=np.float64)[:, None]
    E, _, F = periodic_energy_forces(x, species, weights, box)
    U, K = [E], [0.5 * (m * v * v).sum() / KAPPA]
    for _ in range(nsteps):
        v += 0.5 * dt * KAPPA * F / m
        x += dt * v
        E, _, F = periodic_energy_forces(x, species, weights, box)
        v += 0.5 * dt * KAPPA * F / m
        U.append(E)
        K.append(0.5 * (m * v * v).sum() / KAPPA)
    return x, v, np.array(U), np.array(K)


def system_energy_forces(system, forces: bool = True):
    """Per-molecule energies (M,), per-atom energies (N,), forces (N,3);
    a system with a box is one periodic molecule."""
    if getattr(system, "box", None) is not None:
        E, Ei, F = periodic_energy_forces(system.pos, system.species, system.weights, system.box, forces)
        return np.array([E]), Ei, F
    M = system.n_molecules
    E = np.zeros(M)
    Ei = np.zeros(system.n_atoms)
    F = np.zeros((system.n_atoms, 3)) if forces else None
    for m in range(M):
        s = system.molecule(m)
        e, ei, f = energy_forces(system.pos[s], system.species[s], system.weights, forces)
        E[m] = e
        Ei[s] = ei
        if forces:
            F[s] = f
    return E, Ei, F
