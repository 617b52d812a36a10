"""Long two-component droplet runs on the GPU against observables the FP64
oracle wrote (tests/golden/oracle_<case>.json, written by
tests/golden/oracle_droplet_runs.py, which calls only the oracle):

  c3_recipe_128 : the two-drop collision of the 512 x 256 x 256 workload at a
                  128^3 fallback size (drops of radius 20, u_x = +-0.05), 2000
                  steps, the drops merging;
  head_on_128   : the paper's head-on validation collision (Sec. IV, Figs.
                  4-5: D = 30, b = 0, U_rel = 0.25) with the near-contact force
                  A_h = 0.01, 2000 steps.

Every 100 steps the GPU run's observables (the drop-averaged density
<rho1>_{rho1 > 0.5}, the half-box centroids, the kinetic energy, phi at the
box centre) are compared with the oracle's, and at a few steps the moments at
sampled nodes.

Two regimes.  Until the film between the drops thins (the last recorded step
with phi <= -0.95 at the box centre in the oracle's run, and every step
before it), the bound is ten times the oracle's own spread (its run from the
initial state against its run from the same state rounded to FP32) plus a
floor of the storage precision, node-wise included.  Once a film ruptures,
rounding of any kind decides where and when the neck opens: an FP64 GPU run
that agrees with the oracle to 1e-13 before contact differs from it by about
1e-2 lattice units in the centroids soon after, by more than ten times the
oracle's own spread, and node values in the neck differ by O(1).  From there
on the observables are held to the tolerances of the droplet-collision
configuration instead (centroids within 0.05 lattice units, the drop-averaged
density within 1e-4 relative, the kinetic energy within 1e-3 relative);
phi at the centre and the sampled nodes are reported, not compared.  The
drop-averaged density also moves by membership of single nodes near
rho1 = 0.5 (each by at most 0.5/count); ten such nodes are allowed."""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
sys.path.insert(0, GOLDEN)
import oracle_droplet_runs as G  # noqa: E402  (the observables; no oracle call at test time)

from paper_2301_01622_amd import inputs as I  # noqa: E402

# Floors of the contact-free regime per storage precision.
FLOORS = {
    "f64": {"centroids": 1e-9, "kinetic_energy_rel": 1e-10, "phi_centre": 1e-10, "samples_rel": 1e-10},
    "f32": {"centroids": 1e-4, "kinetic_energy_rel": 5e-5, "phi_centre": 1e-5, "samples_rel": 1e-5},
}
# Tolerances after a film has thinned (the droplet-collision configuration's).
AFTER = {"centroids": 0.05, "mean_rho1_rel": 1e-4, "kinetic_energy_rel": 1e-3}


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _golden(case):
    path = os.path.join(GOLDEN, f"oracle_{case}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written yet (tests/golden/oracle_droplet_runs.py)")
    return json.load(open(path))


def _initial(case):
    if case == "c3_recipe_128":
        return I.droplet_collision_128()
    return I.paper_collision("head_on", 128)


def _contact_free_until(g):
    """Last recorded step up to which phi at the box centre stayed <= -0.95
    in the oracle's run."""
    last = g["t"][0]
    for t, o in zip(g["t"], g["obs"]["x0"]):
        if o["phi_centre"] > -0.95:
            break
        last = t
    return last


@pytest.mark.parametrize("case", ["c3_recipe_128", "head_on_128"])
@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_long_droplet_run_matches_oracle_observables(case, storage):
    from paper_2301_01622_amd.lbm import LBM
    g = _golden(case)
    T, every, tc = g["t"][-1], g["every"], _contact_free_until(g)
    _say(f"{case} {storage}: {T} steps against the oracle's observables (contact-free until step {tc})")
    r1, r2, u = _initial(case)
    n = g["n"]
    sim = LBM((n, n, n), 19, g["tau"], species=2, storage=storage, sigma=g["sigma"], beta=g["beta"],
              nc_A=g["A_h"], nc_hmax=g["h_max"])
    sim.set_equilibrium(torch.from_numpy(np.stack([r1, r2])).cuda(), torch.from_numpy(u).cuda())
    nodes = [tuple(v) for v in g["sample_nodes"]]
    fl = FLOORS[storage]
    worst, fails = {}, []
    for i, t in enumerate(g["t"]):
        if i:
            sim.step(every)
        M = sim.get_moments(torch.float64, device="cpu").numpy()
        got = G.observables(M)
        ref, per = g["obs"]["x0"][i], g["obs"]["x0_fp32"][i]
        flips = 10 * 0.5 / float((M[0] > 0.5).sum())
        sp = {k: np.abs(np.asarray(ref[k]) - np.asarray(per[k])) for k in ("mean_rho1", "centroids",
                                                                             "kinetic_energy", "phi_centre")}
        if t <= tc:
            checks = {
                "mean_rho1": (got["mean_rho1"], ref["mean_rho1"], 10 * sp["mean_rho1"] + flips),
                "centroids": (got["centroids"], ref["centroids"], 10 * sp["centroids"] + fl["centroids"]),
                "kinetic_energy": (got["kinetic_energy"], ref["kinetic_energy"],
                                   10 * sp["kinetic_energy"] + fl["kinetic_energy_rel"] * abs(ref["kinetic_energy"])),
                "phi_centre": (got["phi_centre"], ref["phi_centre"], 10 * sp["phi_centre"] + fl["phi_centre"]),
            }
            if str(t) in g["samples"]["x0"]:
                A = np.array(g["samples"]["x0"][str(t)])
                B = np.array(g["samples"]["x0_fp32"][str(t)])
                S = np.array([[M[f, z, y, x] for f in range(11)] for (z, y, x) in nodes])
                checks["samples"] = (S, A, 10 * np.abs(A - B) + fl["samples_rel"] * np.abs(A).max())
        else:
            checks = {
                "mean_rho1": (got["mean_rho1"], ref["mean_rho1"],
                              max(AFTER["mean_rho1_rel"] * abs(ref["mean_rho1"]), flips)),
                "centroids": (got["centroids"], ref["centroids"], AFTER["centroids"]),
                "kinetic_energy": (got["kinetic_energy"], ref["kinetic_energy"],
                                   AFTER["kinetic_energy_rel"] * abs(ref["kinetic_energy"])),
            }
            _say(f"    t={t:5d} reported: phi at the centre {got['phi_centre']:+.4f} (oracle {ref['phi_centre']:+.4f})")
        for k, (a, b, bound) in checks.items():
            err = np.abs(np.asarray(a) - np.asarray(b))
            ratio = float(np.max(err / np.asarray(bound)))
            worst[k] = max(worst.get(k, 0.0), ratio)
            if ratio > 1.0:
                fails.append(f"t={t} {k}: err {np.max(err):.3e} bound {np.min(bound):.3e}")
    sim.close()
    _say(f"  largest error / bound per observable: {worst}")
    assert not fails, fails[:10]
