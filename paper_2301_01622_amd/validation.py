"""The paper's validation experiment on the GPU (Sec. IV): two drops of
diameter 30 in a periodic 128^3 box, viscosity ratio one, run side by side
with the moment scheme (this library's step) and the colour-gradient LB with
stored populations (the same-GPU baseline), comparing

  * the drop-averaged density <rho1>_{rho1 > 0.5} over time (the paper's
    Figs. 2, 5 and 7), and
  * the local relative difference |rho1_N - rho1_P| / max(rho1_N) at three
    probe sites: near an interface, between the drops, far from them (Fig. 3).

Cases: "off_axis" (b = 0.85, U_rel = 0.5, near-contact strength A_h = 0.01:
the bouncing collision of Figs. 1-3), "head_on" (b = 0, U_rel = 0.25,
A_h = 0.01: Figs. 4-5), "coalescence" (the off-axis collision with A_h = 0:
Figs. 6-7), and "head_on_coalescence" (head-on with A_h = 0).  The phase
field phi = 2 rho1/rho - 1 at the box centre, where the drops meet, is
recorded too: it stays negative while a film separates them.
Readings of the parameters the paper leaves to an external table: tau = 0.8,
sigma = 0.01, beta = 0.7, near-contact probe range h_max = 4; the impact
parameter b is in units of D (b = 0.85: centres 25.5 apart across the
motion); the relative impact velocity U_rel is in units of the capillary
velocity sigma/(rho nu) = 0.1 (U_rel = 0.5: drops at +-0.025; head-on
U_rel = 0.25: +-0.0125); the drops start 38 apart along x (8 lattice units
between the interfaces: their profiles overlap by less than 1 % and no film
is within the near-contact range, and the drops, which the carrier fluid
slows down, meet after about 10^2 steps, where the paper's Figs. 2 and 5
place the start of the interaction; starting 48 apart they stop before
touching).  The paper prints no values for these curves (its
figures are not available), so the comparison is reported, not pinned.

    python -m paper_2301_01622_amd.validation [case] [steps] [every]
"""
from __future__ import annotations

import json
import sys

import numpy as np
import torch

from . import inputs
from .lbm import LBM

TAU, SIGMA, BETA, HMAX = inputs.PAPER_TAU, inputs.PAPER_SIGMA, inputs.PAPER_BETA, inputs.PAPER_HMAX
CASES = inputs.PAPER_CASES


def setup(case: str, n: int = 128):
    """(rho1, rho2, u) for the case on an n^3 box (drops of diameter 30 n/128)."""
    return inputs.paper_collision(case, n)


def probes(n: int = 128):
    """Near an interface, between the drops, far from them ((z, y, x), 0-based)."""
    s = n / 128.0
    return {"interface": (int(64 * s) - 1, int(64 * s) - 1, int(32 * s) - 1),
            "between": (int(64 * s) - 1, int(64 * s) - 1, int(64 * s) - 1),
            "far": (n - 1, n - 1, n - 1)}


def run(case: str = "off_axis", steps: int = 8000, every: int = 100, n: int = 128, q: int = 19) -> dict:
    r1, r2, u = setup(case, n)
    prim = torch.from_numpy(np.stack([r1, r2])).cuda()
    uu = torch.from_numpy(u).cuda()
    sims = {}
    A_h = CASES[case]["A_h"]
    for scheme in ("moment", "population"):
        s = LBM((n, n, n), q, TAU, species=2, storage="f32", sigma=SIGMA, beta=BETA, scheme=scheme, nc_A=A_h,
                nc_hmax=HMAX if A_h else 0)
        s.set_equilibrium(prim, uu)
        sims[scheme] = s
    pr = probes(n)
    out = {"case": case, "n": n, "lattice": f"D3Q{q}", "steps": steps, "every": every, "A_h": A_h,
           "h_max": HMAX if A_h else 0, "t": [], "mean_rho1_moment": [], "mean_rho1_population": [],
           "phi_centre_moment": [], "phi_centre_population": [], "probe_rel_diff": {k: [] for k in pr}}
    c = n // 2 - 1
    t = 0
    while True:
        both = {k: s.get_moments(torch.float64)[:2] for k, s in sims.items()}
        m = {k: v[0] for k, v in both.items()}
        out["t"].append(t)
        for k in ("moment", "population"):
            r = m[k]
            out[f"mean_rho1_{k}"].append(float(r[r > 0.5].mean()))
            r1c, r2c = float(both[k][0, c, c, c]), float(both[k][1, c, c, c])
            out[f"phi_centre_{k}"].append((r1c - r2c) / (r1c + r2c))
        rmax = float(m["moment"].max())
        for k, (z, y, x) in pr.items():
            out["probe_rel_diff"][k].append(abs(float(m["moment"][z, y, x] - m["population"][z, y, x])) / rmax)
        if t >= steps:
            break
        for s in sims.values():
            s.step(every)
        t += every
    for s in sims.values():
        s.close()
    a = np.array(out["mean_rho1_moment"])
    b = np.array(out["mean_rho1_population"])
    out["summary"] = {
        "max_rel_diff_mean_rho1": float(np.abs(a - b).max() / np.abs(b).max()),
        "max_probe_rel_diff": {k: float(max(v)) for k, v in out["probe_rel_diff"].items()},
        "max_phi_centre": {k: float(max(out[f"phi_centre_{k}"])) for k in ("moment", "population")},
    }
    return out


if __name__ == "__main__":
    case = sys.argv[1] if len(sys.argv) > 1 else "off_axis"
    steps = int(sys.argv[2]) if len(sys.argv) > 2 else 8000
    every = int(sys.argv[3]) if len(sys.argv) > 3 else 100
    res = run(case, steps, every)
    print(json.dumps(res["summary"]))
    print(json.dumps(res))
