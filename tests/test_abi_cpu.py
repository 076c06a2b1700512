"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/nnp.h declares, and rejects invalid arguments before
any device work."""

import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "nnp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(nnp_[a-z_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_function():
    import paper_2412_18271_amd as P
    lib = P.load()
    declared = _header_functions()
    assert "nnp_create" in declared and "nnp_step" in declared
    assert declared == set(P.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_status_strings():
    import paper_2412_18271_amd as P
    lib = P.load()
    assert lib.nnp_status_string(0) == b"NNP_OK"
    assert lib.nnp_status_string(3) == b"NNP_ERR_UNSUPPORTED"


def _params(P, s, **kw):
    p = P._lib.Params()
    sp = np.ascontiguousarray(s.species, np.int32)
    m = np.ascontiguousarray(s.masses, np.float64)
    w = np.ascontiguousarray(s.weights, np.float32)
    off = np.ascontiguousarray(s.mol_offsets, np.int32)
    keep = [sp, m, w, off]
    p.n_atoms = s.n_atoms
    p.n_molecules = s.n_molecules
    p.mol_offsets = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    p.species = sp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    p.masses = m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.weights = w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    p.weights_count = w.shape[0]
    p.mlp_dtype = 0
    p.path = 1
    p.rebuild_every = 20
    p.skin = 1.0
    p.max_neighbors = 0
    p.atoms_per_tile = 0
    p.use_stream = 0
    for k, v in kw.items():
        setattr(p, k, v)
    return p, keep


@pytest.mark.parametrize("field,value,status", [
    ("n_atoms", 0, 1),
    ("n_molecules", 0, 1),
    ("weights_count", 10, 1),
    ("mlp_dtype", 2, 3),
    ("mlp_dtype", 7, 1),
    ("path", 5, 1),
    ("rebuild_every", 0, 1),
    ("skin", -1.0, 1),
    ("max_neighbors", 300, 1),
    ("atoms_per_tile", 12, 1),
    ("atoms_per_tile", 16, 1),
])
def test_create_rejects_invalid_params(field, value, status):
    import paper_2412_18271_amd as P
    lib = P.load()
    s = synth.make_config("mol22")
    p, keep = _params(P, s, **{field: value})
    h = ctypes.c_void_p()
    assert lib.nnp_create(ctypes.byref(p), ctypes.byref(h)) == status
    assert not h.value


def test_create_rejects_bad_species_masses_offsets():
    import paper_2412_18271_amd as P
    lib = P.load()
    s = synth.make_config("mol22")
    bad = synth.make_config("mol22")
    bad.species = bad.species.copy()
    bad.species[3] = 4
    p, keep = _params(P, bad)
    h = ctypes.c_void_p()
    assert lib.nnp_create(ctypes.byref(p), ctypes.byref(h)) == 1
    bad = synth.make_config("mol22")
    bad.masses = bad.masses.copy()
    bad.masses[0] = 0.0
    p, keep = _params(P, bad)
    assert lib.nnp_create(ctypes.byref(p), ctypes.byref(h)) == 1
    p, keep = _params(P, s, n_molecules=2)
    off = np.array([0, 30, 22], np.int32)
    p.mol_offsets = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    assert lib.nnp_create(ctypes.byref(p), ctypes.byref(h)) == 1
    w = s.weights.copy()
    w[5] = np.nan
    p, keep = _params(P, s)
    p.weights = w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    assert lib.nnp_create(ctypes.byref(p), ctypes.byref(h)) == 2


def test_null_context_calls_fail_cleanly():
    import paper_2412_18271_amd as P
    lib = P.load()
    assert lib.nnp_compute(None, None, None, None, None) == 1
    assert lib.nnp_step(None, 0.5, 1, 0) == 1
    assert lib.nnp_set_state(None, None, None) == 1
    lib.nnp_destroy(None)
