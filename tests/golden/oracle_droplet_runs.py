"""Writes the oracle's observables of two long two-component droplet runs to
JSON files beside this script; the GPU tests compare their FP32 runs with
them.  Calls only the oracle (oracle/) and the seeded input generators.

Runs (D3Q19, tau = 0.8, sigma = 0.01, beta = 0.7, the colour-gradient step of
Sec. III.A with the operators of Sec. III.B, FP64):

  c3_recipe_128 : the two-drop collision of the 512 x 256 x 256 workload at a
                  128^3 fallback size (drops of radius 20 at (34, 59, 64) and
                  (94, 69, 64), u_x = +-0.05, tanh width 1.5), 2000 steps;
  head_on_128   : the paper's head-on validation collision (Sec. IV, Figs.
                  4-5: drops of diameter 30, b = 0, U_rel = 0.25) with the
                  near-contact force A_h = 0.01 (probe range 4), 2000 steps.

Each case runs twice: from the initial state, and from the same state rounded
to FP32 (a perturbation of the size an FP32 run starts with).  Every 100 steps
the script records the observables (observables() below) of both runs, and
at a few steps the 11 moments at sampled nodes; the spread between the two
runs sets the GPU tests' tolerance.  The files are rewritten after every
100 steps, so a partial run is usable.  With --state-dir DIR the two
states are also saved there after every 100 steps, and a later call with
the same DIR resumes from the last recorded step.

    python tests/golden/oracle_droplet_runs.py [--state-dir DIR] [case ...]   # about 1-2 h per case on 8 cores

With --early it writes oracle_head_on_128_early.json instead: the first 40
steps of the head-on case, the 11 moments at the nodes of the film between
the drops every 10 steps (both runs).  In this case the film between the
drops is thin from the start (phi = -0.96 at the box centre), and the
oracle's own spread grows from the FP32 rounding level (1e-8) at step 40 to
1e-3 at step 60 at the film centre, where the colour gradient passes through
zero (recolouring with the smoothed normal amplifies short waves there);
the near-contact force first acts at about step 80.  Node-wise comparisons
at the strict bound are possible only before that growth.
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

TAU, SIGMA, BETA, Q = 0.8, 0.01, 0.7, 19
STEPS, EVERY = 2000, 100
SAMPLE_STEPS = (100, 200, 300, 500, 1000, 2000)


def observables(M: np.ndarray) -> dict:
    """Diagnostics of an 11-field state (rho1, rho2, j, P), shape
    (11, n, n, n), x fastest: mean of rho1 over nodes with rho1 > 0.5; the x
    and y centroids of rho1 over the half boxes x < n/2 and x >= n/2; kinetic
    energy sum |j|^2 / (2 rho); phi = (rho1 - rho2)/(rho1 + rho2) at node
    (n/2 - 1) along every axis; total rho1."""
    r1, r2 = M[0], M[1]
    n = r1.shape[2]
    rho = r1 + r2
    x = np.arange(n, dtype=np.float64)[None, None, :]
    y = np.arange(n, dtype=np.float64)[None, :, None]
    half = [x < n / 2.0, x >= n / 2.0]
    cent = []
    for m in half:
        w = r1 * m
        s = w.sum()
        cent += [float((w * x).sum() / s), float((w * y).sum() / s)]
    c = n // 2 - 1
    return {
        "mean_rho1": float(r1[r1 > 0.5].mean()),
        "centroids": cent,
        "kinetic_energy": float(((M[2] ** 2 + M[3] ** 2 + M[4] ** 2) / (2.0 * rho)).sum()),
        "phi_centre": float((r1[c, c, c] - r2[c, c, c]) / rho[c, c, c]),
        "mass_rho1": float(r1.sum()),
    }


def sample_nodes(n: int, case: str):
    """(z, y, x) nodes: along the collision axis through the gap between the
    drops, on the drop surfaces, in the drop cores, in the carrier, corners."""
    c = n // 2 - 1
    nodes = [(c, c, x) for x in range(c - 10, c + 12, 2)]
    if case == "c3_recipe_128":
        nodes += [(64, 59, 54), (64, 69, 74), (64, 59, 34), (64, 69, 94), (64, 79, 64), (64, 49, 64)]
    else:
        nodes += [(c, c, c - 30), (c, c, c + 30), (c, c + 15, c - 19), (c, c - 15, c + 19), (c + 15, c, c - 19)]
    nodes += [(0, 0, 0), (n - 1, n - 1, n - 1), (c, 0, c), (10, 100, 20)]
    return sorted(set(nodes))


def initial_state(case: str):
    import oracle
    from paper_2301_01622_amd import inputs
    if case == "c3_recipe_128":
        r1, r2, u = inputs.droplet_collision_128()
        A_h = 0.0
    elif case == "head_on_128":
        r1, r2, u = inputs.paper_collision("head_on", 128)
        A_h = inputs.PAPER_CASES["head_on"]["A_h"]
    else:
        raise ValueError(case)
    return oracle.equilibrium_moments2(r1, r2, u), A_h


def run(case: str, state_dir: str | None = None) -> str:
    import oracle
    oracle._load()
    H0, A_h = initial_state(case)
    hmax = 4 if A_h else 0
    A = oracle.sigma_to_A(SIGMA, TAU)
    n = H0.shape[-1]
    nodes = sample_nodes(n, case)
    states = {"x0": H0, "x0_fp32": H0.astype(np.float32).astype(np.float64)}
    out = {
        "case": case, "n": n, "lattice": "D3Q19", "tau": TAU, "sigma": SIGMA, "beta": BETA, "A_h": A_h,
        "h_max": hmax, "steps": STEPS, "every": EVERY,
        "source": "oracle.cg_moment_run (FP64), written by tests/golden/oracle_droplet_runs.py",
        "runs": {"x0": "the initial state", "x0_fp32": "the initial state rounded to FP32"},
        "t": [], "obs": {k: [] for k in states}, "sample_nodes": nodes, "samples": {k: {} for k in states},
    }
    path = os.path.join(HERE, f"oracle_{case}.json")
    t = 0
    # Saved states carry their step in the file name, so a kill between
    # writing them and the JSON file leaves a consistent pair behind.
    saved = lambda k, step: os.path.join(state_dir, f"{case}_{k}_t{step}.npy")
    if state_dir:
        os.makedirs(state_dir, exist_ok=True)
        if os.path.exists(path):
            with open(path) as fh:
                prev = json.load(fh)
            last = prev["t"][-1] if prev["t"] else None
            if last is not None and all(os.path.exists(saved(k, last)) for k in states):
                out, t = prev, last
                states = {k: np.load(saved(k, last)) for k in states}
                print(f"{case}: resuming at t={t}", flush=True)
    t0 = time.time()
    while True:
        if not out["t"] or out["t"][-1] != t:
            out["t"].append(t)
            for k, H in states.items():
                out["obs"][k].append(observables(H))
                if t in SAMPLE_STEPS:
                    out["samples"][k][str(t)] = [[float(H[f, z, y, x]) for f in range(11)] for (z, y, x) in nodes]
            if state_dir:
                for k, H in states.items():
                    np.save(saved(k, t), H)
            with open(path + ".tmp", "w") as fh:
                json.dump(out, fh)
            os.replace(path + ".tmp", path)
            if state_dir and t >= EVERY:
                for k in states:
                    if os.path.exists(saved(k, t - EVERY)):
                        os.remove(saved(k, t - EVERY))
        print(f"{case}: t={t} ({time.time() - t0:.0f} s)", flush=True)
        if t >= STEPS:
            break
        for k in states:
            states[k] = oracle.cg_moment_run(states[k], Q, TAU, A, BETA, EVERY, Ah=A_h, hmax=hmax)
        t += EVERY
    return path


EARLY_STEPS = (10, 20, 30, 40)


def early_nodes(n: int):
    """(z, y, x) nodes of the film between the head-on drops: lines through
    the film centre (n/2, n/2, n/2) along x, y and z, and the drop surfaces."""
    c = n // 2
    nodes = [(c, c, x) for x in range(c - 12, c + 13)]
    nodes += [(c, y, c) for y in range(c - 8, c + 9)] + [(z, c, c) for z in range(c - 8, c + 9)]
    nodes += [(c - 1, c + 1, c - 1), (c + 2, c - 3, c + 1), (c, c, c - 34), (c, c, c + 34), (c, c + 15, c - 19)]
    return sorted(set(nodes))


def run_early(case: str = "head_on_128") -> str:
    """The first steps of a case, the 11 moments at the film nodes every 10
    steps for both runs, and the number of nodes the near-contact force acts
    on (film distance found within h_max) in the unperturbed run."""
    import oracle
    oracle._load()
    H0, A_h = initial_state(case)
    hmax = 4 if A_h else 0
    A = oracle.sigma_to_A(SIGMA, TAU)
    n = H0.shape[-1]
    nodes = early_nodes(n)
    states = {"x0": H0, "x0_fp32": H0.astype(np.float32).astype(np.float64)}
    out = {"case": case, "n": n, "lattice": "D3Q19", "tau": TAU, "sigma": SIGMA, "beta": BETA, "A_h": A_h,
           "h_max": hmax, "source": "oracle.cg_moment_run (FP64), written by tests/golden/oracle_droplet_runs.py",
           "runs": {"x0": "the initial state", "x0_fp32": "the initial state rounded to FP32"},
           "sample_nodes": nodes, "t": [], "forced_nodes": [], "samples": {k: {} for k in states}}
    t, t0 = 0, time.time()
    for T in EARLY_STEPS:
        for k in states:
            states[k] = oracle.cg_moment_run(states[k], Q, TAU, A, BETA, T - t, Ah=A_h, hmax=hmax)
            out["samples"][k][str(T)] = [[float(states[k][f, z, y, x]) for f in range(11)] for (z, y, x) in nodes]
        t = T
        H = states["x0"]
        _, h = oracle.nc_force((H[0] - H[1]) / (H[0] + H[1]), Q, A_h, hmax) if A_h else (None, np.zeros(1))
        out["t"].append(T)
        out["forced_nodes"].append(int((h > 0).sum()))
        print(f"{case} early: t={T} ({time.time() - t0:.0f} s)", flush=True)
    path = os.path.join(HERE, f"oracle_{case}_early.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    return path


if __name__ == "__main__":
    args, state_dir = sys.argv[1:], None
    if args[:1] == ["--early"]:
        print(run_early(), flush=True)
        sys.exit(0)
    if args[:1] == ["--state-dir"]:
        state_dir, args = args[1], args[2:]
    for c in (args or ["c3_recipe_128", "head_on_128"]):
        print(run(c, state_dir), flush=True)
