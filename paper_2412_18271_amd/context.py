"""Python handle on one library context (names follow the C ABI)."""

from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _lib
from ._lib import NNPError


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


class Context:
    """Wraps nnp_create .. nnp_destroy.

    species, masses, weights and mol_offsets are copied by the library at
    creation.  ``stream`` is a raw hipStream_t (int; 0 is the null stream)
    or None for a stream the context owns.  ``return_mode`` is
    "energy_forces" or "energy" (compute() then returns the energy only).
    """

    def __init__(self, species, masses, weights, mol_offsets=None, dtype: str = "fp32",
                 path: str = "fused", rebuild_every: int = 20, skin: float = 1.0,
                 max_neighbors: int = 0, atoms_per_tile: int = 0, stream: Optional[int] = None,
                 return_mode: str = "energy_forces", network_tile: int = 0):
        self._lib = _lib.load()
        self._sp = np.ascontiguousarray(species, dtype=np.int32)
        self._m = np.ascontiguousarray(masses, dtype=np.float64)
        self._w = np.ascontiguousarray(weights, dtype=np.float32)
        n = int(self._sp.shape[0])
        if mol_offsets is None:
            self._off = np.array([0, n], dtype=np.int32)
        else:
            self._off = np.ascontiguousarray(mol_offsets, dtype=np.int32)
        self.n_atoms = n
        self.n_molecules = int(self._off.shape[0] - 1)
        self.dtype = dtype
        self.path = path
        self.return_mode = return_mode
        p = _lib.Params()
        p.n_atoms = n
        p.n_molecules = self.n_molecules
        p.mol_offsets = self._off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        p.species = self._sp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        p.masses = self._m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.weights = self._w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        p.weights_count = int(self._w.shape[0])
        p.mlp_dtype = _lib.DTYPES[dtype]
        p.path = _lib.PATHS[path]
        p.return_mode = _lib.RETURN_MODES[return_mode]
        p.rebuild_every = int(rebuild_every)
        p.skin = float(skin)
        p.max_neighbors = int(max_neighbors)
        p.atoms_per_tile = int(atoms_per_tile)
        p.stream = stream if stream else None
        p.use_stream = 0 if stream is None else 1
        p.network_tile = int(network_tile)
        h = ctypes.c_void_p()
        s = self._lib.nnp_create(ctypes.byref(p), ctypes.byref(h))
        if s != _lib.NNP_OK:
            raise NNPError(s, "nnp_create failed (message on stderr)")
        self._h = h

    @classmethod
    def from_system(cls, system, **kw):
        ctx = cls(system.species, system.masses, system.weights, system.mol_offsets, **kw)
        if getattr(system, "box", None) is not None:
            ctx.set_box(system.box)
        return ctx

    def set_box(self, box):
        """Orthorhombic periodic box edges (3,) in A, or None for the gas phase."""
        b = None if box is None else np.ascontiguousarray(box, dtype=np.float64).reshape(3)
        self._check(self._lib.nnp_set_box(self._h, _dptr(b)))

    # ------------------------------------------------------------------
    def _check(self, s):
        if s != _lib.NNP_OK:
            msg = self._lib.nnp_last_error(self._h)
            err, self._provider_error = getattr(self, "_provider_error", None), None
            raise NNPError(s, msg.decode() if msg else "") from err

    def close(self):
        if getattr(self, "_h", None):
            self._lib.nnp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------
    def _pos(self, pos):
        p = np.ascontiguousarray(pos, dtype=np.float64).reshape(self.n_atoms, 3)
        return p

    def compute(self, pos, forces: Optional[bool] = None, box=None):
        """Energies per molecule (M,) and forces (N, 3) (None if not asked;
        by default asked unless the context returns energy only)."""
        if forces is None:
            forces = self.return_mode != "energy"
        p = self._pos(pos)
        E = np.zeros(self.n_molecules, np.float64)
        F = np.zeros((self.n_atoms, 3), np.float64) if forces else None
        b = None if box is None else np.ascontiguousarray(box, dtype=np.float64)
        self._check(self._lib.nnp_compute(self._h, _dptr(p), _dptr(b), _dptr(E), _dptr(F)))
        return E, F

    def compute_device(self, d_pos: int, pos_is_f64: bool, d_energy: int, d_forces: Optional[int]):
        """Raw device-pointer evaluation on the context stream (no sync)."""
        self._check(self._lib.nnp_compute_device(self._h, ctypes.c_void_p(d_pos), int(pos_is_f64),
                                                 ctypes.c_void_p(d_energy),
                                                 ctypes.c_void_p(d_forces) if d_forces else None))

    def energy_device(self, d_pos: int, pos_is_f64: bool, d_energy: int, keep: bool):
        """Energy only, on the context stream (no sync); keep=True stores G
        and dE/dG for a following forces_device()."""
        self._check(self._lib.nnp_energy_device(self._h, ctypes.c_void_p(d_pos), int(pos_is_f64),
                                                ctypes.c_void_p(d_energy), 1 if keep else 0))

    def energy_device_static(self, d_pos: int, pos_is_f64: bool, d_energy: int):
        """Stored-mode energy (like energy_device(keep=True)) with G and
        dE/dG in the library's static device array: allocates nothing; at
        most 8,192 atoms; a later call on the same GPU replaces the kept data."""
        self._check(self._lib.nnp_energy_device_static(self._h, ctypes.c_void_p(d_pos), int(pos_is_f64),
                                                       ctypes.c_void_p(d_energy)))

    def forces_device(self, d_forces: int):
        self._check(self._lib.nnp_forces_device(self._h, ctypes.c_void_p(d_forces)))

    def set_state(self, pos=None, vel=None):
        p = self._pos(pos) if pos is not None else None
        v = self._pos(vel) if vel is not None else None
        self._check(self._lib.nnp_set_state(self._h, _dptr(p), _dptr(v)))

    def get_state(self):
        n, m = self.n_atoms, self.n_molecules
        pos, vel, frc = (np.zeros((n, 3)) for _ in range(3))
        pot, kin = np.zeros(m), np.zeros(m)
        self._check(self._lib.nnp_get_state(self._h, _dptr(pos), _dptr(vel), _dptr(frc), _dptr(pot),
                                            _dptr(kin)))
        return {"pos": pos, "vel": vel, "forces": frc, "pot": pot, "kin": kin}

    def step(self, dt: float, n_steps: int, graph: bool = True):
        self._check(self._lib.nnp_step(self._h, float(dt), int(n_steps), 1 if graph else 0))

    def capture(self, dt: float, n_steps: int):
        """Captures the graphs step(dt, n_steps) replays, without stepping."""
        self._check(self._lib.nnp_capture(self._h, float(dt), int(n_steps)))

    def add_force(self, fn, kind: str = "energy"):
        """Registers an extra force provider summed with the network (the
        paper's callback mechanism).  ``fn`` is called after every network
        evaluation with the positions, on the context's stream:

          kind="energy": fn(pos) -> energy; pos is a float64 CUDA tensor
              [n_atoms, 3] that requires grad, the energy a tensor of one or
              n_molecules elements; forces are minus its gradient (autograd);
          kind="forces": fn(pos) -> (energy, forces) as CUDA tensors;
          kind="numpy":  fn(pos) -> (energy, forces) with pos and the
              results as NumPy arrays (explicit forces, host code).
        """
        import contextlib
        import torch
        if kind not in ("energy", "forces", "numpy"):
            raise ValueError("kind must be 'energy', 'forces' or 'numpy'")
        n, m = self.n_atoms, self.n_molecules
        dev = torch.device("cuda", torch.cuda.current_device())
        pos_t = torch.zeros((n, 3), dtype=torch.float64, device=dev)
        f_t = torch.zeros((n, 3), dtype=torch.float64, device=dev)
        e_t = torch.zeros(m, dtype=torch.float64, device=dev)
        torch.cuda.synchronize(dev)

        def energies(E):
            E = torch.as_tensor(E, dtype=torch.float64, device=dev).reshape(-1)
            if E.numel() not in (1, m):
                raise ValueError("energy must have 1 or n_molecules elements")
            return E

        def call(user, n_atoms, n_mol, d_pos, d_f, d_e, stream):
            try:
                ctx = (torch.cuda.stream(torch.cuda.ExternalStream(stream, device=dev)) if stream
                       else contextlib.nullcontext())
                with ctx:
                    if kind == "energy":
                        with torch.enable_grad():
                            x = pos_t.detach().clone().requires_grad_(True)
                            E = energies(fn(x))
                            (g,) = torch.autograd.grad(E.sum(), x)
                        F = -g
                    elif kind == "forces":
                        E, F = fn(pos_t.detach().clone())
                        E = energies(E)
                    else:
                        E, F = fn(pos_t.cpu().numpy())
                        E = energies(np.asarray(E, dtype=np.float64))
                    f_t.copy_(torch.as_tensor(F, dtype=torch.float64, device=dev).reshape(n, 3))
                    e_t.copy_(E.detach().expand(m) if E.numel() == 1 else E.detach())
                return 0
            except Exception as exc:  # reported by the calling entry point
                self._provider_error = exc
                return 1

        cb = _lib.FORCE_FN(call)
        self._providers = getattr(self, "_providers", []) + [(cb, pos_t, f_t, e_t)]  # keep alive
        self._check(self._lib.nnp_add_force(self._h, cb, None, ctypes.c_void_p(pos_t.data_ptr()),
                                            ctypes.c_void_p(f_t.data_ptr()), ctypes.c_void_p(e_t.data_ptr())))

    def clear_forces(self):
        self._check(self._lib.nnp_clear_forces(self._h))
        self._providers = []

    def set_thermostat(self, temperature: float = 300.0, friction: float = 0.1, seed: int = 0):
        """Langevin dynamics (BAOAB) for the following steps: temperature in K,
        friction in 1/ps; friction 0 restores NVE velocity Verlet."""
        self._check(self._lib.nnp_set_thermostat(self._h, float(temperature), float(friction), int(seed)))

    def energy_log(self, count: int):
        m = self.n_molecules
        U = np.zeros((count, m))
        K = np.zeros((count, m))
        w = ctypes.c_int32(0)
        self._check(self._lib.nnp_energy_log(self._h, int(count), _dptr(U), _dptr(K), ctypes.byref(w)))
        return U[:w.value], K[:w.value]

    def stats(self):
        s = (ctypes.c_int64 * 7)()
        self._check(self._lib.nnp_stats(self._h, s))
        return {"evaluations": s[0], "rebuilds": s[1], "forced_rebuilds": s[2], "steps": s[3],
                "max_pairlist": s[4], "max_radial": s[5], "max_angular": s[6]}

    def config(self):
        """The kernel configuration in use: {path, atoms_per_tile, network_tile}."""
        c = (ctypes.c_int32 * 3)()
        self._check(self._lib.nnp_get_config(self._h, c))
        names = {v: k for k, v in _lib.PATHS.items()}
        return {"path": names.get(c[0], c[0]), "atoms_per_tile": int(c[1]), "network_tile": int(c[2])}

    def descriptors(self, pos):
        p = self._pos(pos)
        G = np.zeros((self.n_atoms, 384), np.float32)
        self._check(self._lib.nnp_debug_descriptors(
            self._h, _dptr(p), G.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return G

    def atom_energies(self):
        e = np.zeros(self.n_atoms)
        self._check(self._lib.nnp_debug_atom_energies(self._h, _dptr(e)))
        return e

    def device_bytes(self) -> int:
        b = ctypes.c_int64(0)
        self._check(self._lib.nnp_device_bytes(self._h, ctypes.byref(b)))
        return int(b.value)

    def autotune(self, cache_path: Optional[str] = None):
        """Times the candidate kernel configurations and keeps the fastest
        (or applies the cached choice); returns it as a dict."""
        ch = (ctypes.c_int32 * 4)()
        self._check(self._lib.nnp_autotune(self._h, cache_path.encode() if cache_path else None, ch))
        names = {v: k for k, v in _lib.PATHS.items()}
        self.path = names[ch[0]]
        return {"path": self.path, "atoms_per_tile": int(ch[1]), "network_tile": int(ch[2]),
                "from_cache": bool(ch[3])}

    def time_steps(self, dt: float, n: int):
        """n event-timed MD steps without a graph: average ms per step of
        (evaluation kernels, gather/integration kernel, whole step)."""
        ms = np.zeros(3)
        self._check(self._lib.nnp_time_steps(self._h, float(dt), int(n), _dptr(ms)))
        return float(ms[0]), float(ms[1]), float(ms[2])

    def time_kernels(self, reps: int = 50):
        """Average ms per launch of (evaluation kernels, gather kernel)."""
        ms = np.zeros(2)
        self._check(self._lib.nnp_time_kernels(self._h, int(reps), _dptr(ms)))
        return float(ms[0]), float(ms[1])
