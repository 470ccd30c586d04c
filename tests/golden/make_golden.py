"""Write the stored expected values under tests/golden/ by calling the CPU oracle only.

config1_L8_f64.json: the smallest workload -- L = 8 periodic lattice (512 spins),
binary64 spins, Philox seed 1 for the initial state (spins uniform on the sphere,
couplings N(0,1)) and the sweeps, T = 1.0, 10 sweeps of checkerboard Metropolis
with one hit (trial spin uniform on the sphere), no over-relaxation.  Stored per
sweep: tracked energy, recomputed energy, accepted moves, and the final spins.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle as O  # noqa: E402


def config1():
    L, seed, T = 8, 1, 1.0
    s, J = O.init(L, seed, np.float64)
    E = O.energy(L, s, J)
    rec = {"L": L, "seed": seed, "T": T, "k": 1, "n_or": 0, "dtype": "f64",
           "E0": E, "sweeps": []}
    for n in range(10):
        r = O.sweep(L, seed, s, J, T=T, k=1, n_sweeps=1, sweep0=n, E=E)
        E = r["E"]
        rec["sweeps"].append({"E_tracked": E, "E_recomputed": O.energy(L, s, J),
                              "accepted": r["n_accepted"], "flagged": r["n_flagged"]})
    rec["final_spins"] = s.tolist()
    return rec


if __name__ == "__main__":
    with open(os.path.join(HERE, "config1_L8_f64.json"), "w") as f:
        json.dump(config1(), f)
    print("wrote config1_L8_f64.json")
