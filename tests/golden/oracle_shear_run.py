"""Writes the FP64 oracle's state at sampled nodes of the reduced-precision
storage workload, at a 128^3 fallback size, to oracle_c4_recipe_128.json
beside this script; the GPU test compares its FP32, FP16 and BF16 storage
runs with it after 2000 steps.  Calls only the oracle (oracle/) and the
seeded input generators.

Workload: the 512^3 recipe at 128^3: D3Q27, tau = 0.55, rho = 1,
u_x = 0.01 sin(2 pi y / 128) plus solenoidal noise of max norm 1e-4 (seed
16220004), one component, the scheme without populations (FP64).  Recorded
every 500 steps: the 10 moments at 512 nodes drawn with a fixed seed, the
x-z average of u_x as a function of y (the shear wave), and the kinetic
energy.

    python tests/golden/oracle_shear_run.py   # about 15 min on 8 cores
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N, TAU, Q, STEPS, EVERY, NSAMPLE, SEED = 128, 0.55, 27, 2000, 500, 512, 20262003


def sample_nodes():
    rng = np.random.Generator(np.random.PCG64(SEED))
    return [tuple(int(v) for v in rng.integers(0, N, 3)) for _ in range(NSAMPLE)]


def diagnostics(M):
    """(u_x averaged over x and z as a function of y, kinetic energy) of a
    10-field state (rho, j, P), shape (10, n, n, n), x fastest."""
    ux = M[1] / M[0]
    return ux.mean(axis=(0, 2)).tolist(), float(((M[1] ** 2 + M[2] ** 2 + M[3] ** 2) / (2.0 * M[0])).sum())


def main():
    import oracle
    from paper_2301_01622_amd import inputs
    oracle._load()
    rho, u = inputs.shear_wave_with_noise(N, seed=inputs.SEED_C4, u0=0.01, noise=1e-4)
    H = oracle.equilibrium_moments(rho, u)
    nodes = sample_nodes()
    out = {"case": "c4_recipe_128", "n": N, "lattice": "D3Q27", "tau": TAU, "steps": STEPS, "every": EVERY,
           "source": "oracle.moment_run (FP64), written by tests/golden/oracle_shear_run.py",
           "sample_nodes": nodes, "t": [], "samples": [], "ux_profile": [], "kinetic_energy": []}
    path = os.path.join(HERE, "oracle_c4_recipe_128.json")
    t, t0 = 0, time.time()
    while True:
        prof, ke = diagnostics(H)
        out["t"].append(t)
        out["samples"].append([[float(H[f, z, y, x]) for f in range(10)] for (z, y, x) in nodes])
        out["ux_profile"].append(prof)
        out["kinetic_energy"].append(ke)
        with open(path + ".tmp", "w") as fh:
            json.dump(out, fh)
        os.replace(path + ".tmp", path)
        print(f"c4_recipe_128: t={t} ({time.time() - t0:.0f} s)", flush=True)
        if t >= STEPS:
            break
        H = oracle.moment_run(H, Q, TAU, EVERY)
        t += EVERY


if __name__ == "__main__":
    main()
