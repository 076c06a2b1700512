"""Writes tests/golden/mol22_oracle.json from the FP64 oracle alone.

The 22-atom molecule (weights seed 0, positions seed 1, velocities seed 2):
energy, per-atom energies and forces at the initial positions, and the
potential/kinetic energy series and final positions of 100 velocity-Verlet
steps at dt = 0.5 fs.  Run from the repository root:

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    s = synth.make_config("mol22")
    E, Ei, F = oracle.energy_forces(s.pos, s.species, s.weights)
    x, v, U, K = oracle.vv(s.pos, s.vel, s.masses, s.species, s.weights, 0.5, 100)
    out = {
        "source": "oracle/nnp_oracle.c via tests/golden/make_golden.py",
        "workload": "mol22: 22 atoms (12 H, 6 C, 2 N, 2 O), 10 A cube, seeds w0 p1 v2",
        "energy": E, "atom_energies": Ei.tolist(), "forces": F.tolist(),
        "dt_fs": 0.5, "steps": 100, "U": U.tolist(), "K": K.tolist(),
        "final_positions": x.tolist(), "final_velocities": v.tolist(),
    }
    with open(os.path.join(HERE, "mol22_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
