"""Throughput of the moment-only lattice Boltzmann step on one MI355X.

Workload: 256^3 periodic box, D3Q27, one component, FP32 moments
(rho, j, P: 10 values per node), tau = 0.6, random solenoidal velocity
(seed 16220002, max |u| = 1e-3).  A step is one full time step of the
scheme; the library advances two steps per kernel launch (a sweep that
carries each tile through both), and the one-step-per-launch kernel is
timed beside it.  The population-storing BGK scheme (two
copies, and in place with one copy) is timed on the same box and GPU, and the
FP64 CPU oracle on the host cores.

Prints one JSON line (see the keys below).  MLUPS follows the paper's
definition (Sec. IV.A, Eq. 12): nodes / (1e6 x seconds per step).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM roofline, moment-LB vs population-LB on 1 MI355X; adjoint/forward cost"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "moment_sweep2_256cube_d3q27_f32_traffic.json")
KERNEL_SOURCES = ["moment_step2.hip", "moment_math.hpp", "lattice.hpp", "storage.hpp", "tile_common.hpp", "layout.hpp"]
STEPS_PER_LAUNCH = 2  # the throughput path advances two steps per kernel launch


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2301_01622_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(n_nodes: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; otherwise None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash() or t.get("n_nodes") != n_nodes:
        return None
    return t.get("bytes_per_launch")


def gpu_warmup(sim, min_ms: float) -> float:
    """Runs steps of `sim` until at least `min_ms` of wall-clock time has
    passed, so the clocks and caches of the GPU are in their steady state
    before the first timed region.  Returns the time spent (ms)."""
    import torch
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < min_ms:
        sim.step(20)  # several launches per synchronisation, so the GPU stays busy
        torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3


def time_steps(sim, stream, steps: int, warmup: int, repeats: int = 3) -> dict:
    """`warmup` untimed steps, then `repeats` timed regions of exactly `steps`
    steps, each bracketed by a device synchronisation on both sides.  Per
    region: kernel time from HIP events on the library's stream (no host
    synchronisation inside the region), and end-to-end wall-clock time of the
    same region including the host's launches and the final synchronisation
    (the paper's t_s of Eq. 12).  Returns the medians (ms per step) and the
    per-region kernel times."""
    import torch
    sim.step(warmup)
    torch.cuda.synchronize()
    kern, e2e = [], []
    for _ in range(max(repeats, 1)):
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        start.record(stream)
        sim.step(steps)
        end.record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kern.append(start.elapsed_time(end) / steps)
        e2e.append((t1 - t0) * 1e3 / steps)
    return {"ms": statistics.median(kern), "e2e_ms": statistics.median(e2e), "repeats": [round(v, 5) for v in kern]}


def _log(msg: str) -> None:
    """Progress of the legs on stderr (the JSON line goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _rate(N: int, ms: float) -> float:
    return round(N / (ms * 1e-3) / 1e6, 1)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n: int, q: int, tau: float, steps: int, rho, u):
    """The FP64 C oracle as it stands, on the host cores: `steps` steps of the
    benchmark box with every OpenMP thread (the reported value), plus small
    bounded side samples: one thread on a 64^3 box of the same recipe, the
    population-storing oracle on 128^3, and the 32^3 D3Q19 Taylor-Green case."""
    import ctypes

    import oracle
    from oracle import build as obuild
    from paper_2301_01622_amd import inputs

    oracle._load()
    gomp = ctypes.CDLL("libgomp.so.1")  # the OpenMP runtime the oracle links
    threads = int(gomp.omp_get_max_threads())

    def mlups(nodes, nsteps, dt):
        return round(nodes * nsteps / dt / 1e6, 3)

    H = oracle.equilibrium_moments(rho, u)
    t0 = time.perf_counter()
    oracle.moment_run(H, q, tau, steps)
    dt = time.perf_counter() - t0
    del H
    side = {}
    # one thread, 64^3 of the same recipe, 2 steps
    r6, u6 = inputs.random_solenoidal_box(64, inputs.SEED_C2, umax=1e-3)
    H6 = oracle.equilibrium_moments(r6, u6)
    gomp.omp_set_num_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.moment_run(H6, q, tau, 2)
        side["single_thread_64cube_d3q27"] = mlups(64 ** 3, 2, time.perf_counter() - t1)
    finally:
        gomp.omp_set_num_threads(threads)
    # the population-storing BGK oracle, 128^3 D3Q27, 4 steps, all threads
    r7, u7 = inputs.random_solenoidal_box(128, inputs.SEED_C2, umax=1e-3)
    f7 = oracle.populations_from_moments(oracle.equilibrium_moments(r7, u7), q)
    t1 = time.perf_counter()
    oracle.population_run(f7, q, tau, 4)
    side["population_oracle_128cube_d3q27"] = mlups(128 ** 3, 4, time.perf_counter() - t1)
    del f7
    # the 32^3 D3Q19 FP64 Taylor-Green case, 100 steps, all threads
    rt, ut = inputs.taylor_green_2d(32, 0.01)
    Ht = oracle.equilibrium_moments(rt, ut)
    t1 = time.perf_counter()
    oracle.moment_run(Ht, 19, 0.8, 100)
    side["taylor_green_32cube_d3q19_100_steps"] = mlups(32 ** 3, 100, time.perf_counter() - t1)
    return {
        "value": mlups(n ** 3, steps, dt),
        "unit": "MLUPS",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{steps} full time steps of the same {n}^3 D3Q{q} box (FP64 C oracle, OpenMP, {threads} threads, "
                  f"{dt:.1f} s)",
        "cpu_model": _cpu_model(),
        "compiler": " ".join([obuild.COMPILER, *obuild.FLAGS]),
        "side_samples_mlups": side,
    }


def adjoint_cost(sim, stream, steps: int, fwd_ms: float, algo_bytes: int = 120,
                 note: str = "one species, same 256^3 D3Q27 FP32 box; algorithmic bytes of the adjoint step "
                             "120 B/node", single_ms: float | None = None, repeats: int = 3):
    """Time of one discrete-adjoint step, alone and with the recomputation of
    the forward state it needs (lbm_step_state into a checkpoint slot), on the
    benchmark box, relative to one forward step (and, if given, to one step of
    the single-step forward kernel).  Medians over `repeats` timed regions."""
    import torch
    st = sim.new_checkpoint()
    slot = sim.new_checkpoint()
    sim.save_state(st)
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    pub = torch.randn((sim.nfields,) + sim.shape, generator=g, device="cuda", dtype=sim.real_dtype)
    # the rollout's path: co-states in the library's stored layout; where the
    # context runs two-step sweeps the rollout recomputes and reverses pairs
    # of steps in one pass each
    lam, lam_b = sim.new_costate(), sim.new_costate()
    sim.costate_to_stored(pub, lam)
    dtau = torch.zeros(1, dtype=torch.float64, device="cuda")
    pairs = getattr(sim, "sweeps", False)
    if pairs:
        st1, slot2 = sim.new_checkpoint(), sim.new_checkpoint()
        sim.step_state(st, st1)

    def adjoint_call():
        if pairs:
            sim.adjoint_step2_stored(st1, st, lam, lam_b, dtau)
        else:
            sim.adjoint_step_stored(st, lam, lam_b, dtau)

    def recompute_call():
        if pairs:
            sim.step_state2(st, slot, slot2)
        else:
            sim.step_state(st, slot)

    per = 2 if pairs else 1
    calls = max(steps // per, 25)
    for _ in range(5):
        adjoint_call()
        recompute_call()
    torch.cuda.synchronize()
    adjs, recs = [], []
    for _ in range(max(repeats, 1)):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(stream)
        for _ in range(calls):
            adjoint_call()
        e[1].record(stream)
        for _ in range(calls):
            recompute_call()
        e[2].record(stream)
        torch.cuda.synchronize()
        adjs.append(e[0].elapsed_time(e[1]) / (calls * per))
        recs.append(e[1].elapsed_time(e[2]) / (calls * per))
    adj, rec = statistics.median(adjs), statistics.median(recs)
    N = sim.n_nodes
    extra = {}
    if single_ms:
        extra = {"ms_forward_single_step_kernel": round(single_ms, 5),
                 "adjoint_plus_recompute_over_single_step_kernel": round((adj + rec) / single_ms, 3)}
    return {
        **extra,
        "steps_per_call": per,
        "steps_timed": calls * per,
        "ms_forward_step": round(fwd_ms, 5),
        "ms_adjoint_step": round(adj, 5),
        "ms_recompute_step": round(rec, 5),
        "adjoint_over_forward": round(adj / fwd_ms, 3),
        "adjoint_plus_recompute_over_forward": round((adj + rec) / fwd_ms, 3),
        "adjoint_hbm_frac": round(algo_bytes * N / (adj * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "note": note,
    }


def _create(LBM, shape, *args, **kw):
    """Creates a context and measures the device memory it takes with
    hipMemGetInfo (through torch), returning (sim, bytes)."""
    import torch
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    sim = LBM(shape, *args, **kw)
    torch.cuda.synchronize()
    return sim, free0 - torch.cuda.mem_get_info()[0]


def two_component(steps: int, warmup: int, repeats: int):
    """512 x 256 x 256 two-component droplet collision (D3Q19, FP32, tau = 0.8,
    sigma = 0.01, beta = 0.7): drops of radius 40 at +-0.05 along x."""
    import numpy as np
    import torch
    from paper_2301_01622_amd import inputs
    from paper_2301_01622_amd.lbm import LBM

    shape = (256, 256, 512)
    r1, r2, u = inputs.droplet_collision_512(shape)
    prim, uu = torch.from_numpy(np.stack([r1, r2])).cuda(), torch.from_numpy(u).cuda()
    del r1, r2, u
    stream = torch.cuda.Stream()
    N = 512 * 256 * 256
    with torch.cuda.stream(stream):
        sim = LBM((512, 256, 256), 19, 0.8, species=2, storage="f32", sigma=0.01, beta=0.7, stream=stream)
        sim.set_equilibrium(prim, uu)
        tm = time_steps(sim, stream, steps, warmup, repeats)
        ms = tm["ms"]
        state_bytes, step_bytes = sim.memory_info()
        adjoint = adjoint_cost(sim, stream, steps, ms, algo_bytes=132, repeats=repeats,
                               note="two species, same 512x256x256 D3Q19 FP32 box; algorithmic bytes of the "
                                    "adjoint step 132 B/node (state, co-state in and out); the two kernels move "
                                    "180 B/node (colour-gradient co-state through HBM)")
        sim.close()
        ps = LBM((512, 256, 256), 19, 0.8, species=2, storage="f32", sigma=0.01, beta=0.7, scheme="population",
                 stream=stream)
        ps.set_equilibrium(prim, uu)
        ptm = time_steps(ps, stream, steps, warmup, repeats)
        pms = ptm["ms"]
        p_state, p_step = ps.memory_info()
        ps.close()
        # The paper's split schedule of the same step: phase-field, collision
        # and streaming passes (same results, more bytes moved).
        sp = LBM((512, 256, 256), 19, 0.8, species=2, storage="f32", sigma=0.01, beta=0.7, split=True, stream=stream)
        sp.set_equilibrium(prim, uu)
        stm = time_steps(sp, stream, steps, warmup, repeats)["ms"]
        _, sp_step = sp.memory_info()
        sp.close()
        # The same collision with the near-contact force (A_h = 0.01, 4 probes).
        nc = {}
        for scheme in ("moment", "population"):
            ns = LBM((512, 256, 256), 19, 0.8, species=2, storage="f32", sigma=0.01, beta=0.7, scheme=scheme,
                     stream=stream, nc_A=0.01, nc_hmax=4)
            ns.set_equilibrium(prim, uu)
            t = time_steps(ns, stream, steps, warmup, repeats)
            ns.close()
            nc[scheme] = {"value": _rate(N, t["ms"]), "unit": "MLUPS", "ms_per_step": round(t["ms"], 5)}
        nc["speedup_vs_population_lb"] = round(nc["population"]["ms_per_step"] / nc["moment"]["ms_per_step"], 3)
        # The same collision on the D3Q27 lattice.
        q27 = LBM((512, 256, 256), 27, 0.8, species=2, storage="f32", sigma=0.01, beta=0.7, stream=stream)
        q27.set_equilibrium(prim, uu)
        t27 = time_steps(q27, stream, steps, warmup, repeats)["ms"]
        q27.close()
    return {
        "workload": "512x256x256 two-component droplet collision, D3Q19, FP32 (rho-1, rho1, j, P), tau=0.8, "
                    "sigma=0.01, beta=0.7, R=40, u=+-0.05",
        "value": _rate(N, ms),
        "unit": "MLUPS",
        "steps": steps,
        "ms_per_step": round(ms, 5),
        "ms_per_step_end_to_end": round(tm["e2e_ms"], 5),
        "hbm_frac": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "bytes_per_node_state": state_bytes // N,
        "population_lb": {
            "scheme": "colour-gradient LB with stored populations (2 x 19 FP32 per node, density pass + "
                      "collision pass per step)",
            "value": _rate(N, pms),
            "unit": "MLUPS",
            "ms_per_step": round(pms, 5),
            "bytes_per_node_state": p_state // N,
        },
        "speedup_vs_population_lb": round(pms / ms, 3),
        "split_approach": {
            "scheme": "moment LB as the split approach (phase-field, collision and streaming passes)",
            "value": _rate(N, stm),
            "unit": "MLUPS",
            "ms_per_step": round(stm, 5),
            "bytes_per_node_step": sp_step // N,
            "hbm_frac": round(sp_step / (stm * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "fused_speedup": round(stm / ms, 3),
        },
        "near_contact": {"A_h": 0.01, "h_max": 4, **nc},
        "d3q27": {"value": _rate(N, t27), "unit": "MLUPS", "ms_per_step": round(t27, 5)},
        "adjoint": adjoint,
    }


# The paper's own benchmark (Sec. IV.A): 128^3, two components, D3Q19, the
# off-axis collision with the near-contact force, on one V100 16 GB; the paper
# does not state the precision (FP32 inferred from its memory figures).
PAPER_V100 = {"moment_mlups": 622.0, "population_mlups": 277.0, "moment_gb": 0.6782, "population_gb": 1.1411,
              "hardware": "NVIDIA Tesla V100 16 GB", "note": "context only: other hardware and code"}


def paper_workload(steps: int, warmup: int, repeats: int):
    """The paper's benchmark shape on this GPU: 128^3 periodic box, D3Q19,
    two components, head-off-axis collision of two drops of diameter 30
    (b = 0.85, U_rel = 0.5), near-contact force A_h = 0.01 (probe range 4),
    tau = 0.8, sigma = 0.01, beta = 0.7, FP32; moment scheme against the
    colour-gradient LB with stored populations."""
    import numpy as np
    import torch
    from paper_2301_01622_amd import validation
    from paper_2301_01622_amd.lbm import LBM

    n = 128
    N = n ** 3
    r1, r2, u = validation.setup("off_axis", n)
    prim, uu = torch.from_numpy(np.stack([r1, r2])).cuda(), torch.from_numpy(u).cuda()
    stream = torch.cuda.Stream()
    out = {"workload": "128^3 two-component head-off-axis droplet collision (D = 30, b = 0.85, U_rel = 0.5), "
                       "D3Q19, FP32, near-contact force A_h = 0.01 (h_max = 4), tau = 0.8, sigma = 0.01, beta = 0.7",
           "steps": steps}
    with torch.cuda.stream(stream):
        for scheme in ("moment", "population"):
            sim, mem = _create(LBM, (n, n, n), 19, validation.TAU, species=2, storage="f32", sigma=validation.SIGMA,
                               beta=validation.BETA, scheme=scheme, stream=stream, nc_A=0.01,
                               nc_hmax=validation.HMAX)
            sim.set_equilibrium(prim, uu)
            t = time_steps(sim, stream, steps, warmup, repeats)
            state_bytes, _ = sim.memory_info()
            sim.close()
            out[scheme] = {"value": _rate(N, t["ms"]), "unit": "MLUPS", "ms_per_step": round(t["ms"], 5),
                           "value_end_to_end": _rate(N, t["e2e_ms"]),
                           "ms_per_step_end_to_end": round(t["e2e_ms"], 5),
                           "device_bytes": mem, "device_gib": round(mem / 2 ** 30, 4),
                           "bytes_per_node_state": state_bytes // N}
    out["speedup_vs_population_lb"] = round(out["population"]["ms_per_step"] / out["moment"]["ms_per_step"], 3)
    out["memory_saving"] = round(1.0 - out["moment"]["device_bytes"] / out["population"]["device_bytes"], 4)
    out["paper_v100"] = PAPER_V100
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed regions of --steps steps each; the median is reported")
    ap.add_argument("--gpu-warmup-ms", type=float, default=300.0,
                    help="wall-clock GPU warm-up before the first timed region")
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-population", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--no-two-component", action="store_true")
    ap.add_argument("--no-paper-workload", action="store_true")
    ap.add_argument("--no-reduced-precision", action="store_true")
    ap.add_argument("--side-steps", type=int, default=100,
                    help="minimum timed steps of each side leg (two-component, paper workload, adjoint)")
    ap.add_argument("--steps-per-sweep", type=int, default=STEPS_PER_LAUNCH, choices=(1, 2),
                    help="steps per launch of the measured path (1: the one-step kernel and one-step adjoint)")
    ap.add_argument("--calibrate-copy", type=int, default=10,
                    help="also time this many state copies (plain copy kernel of known size)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the library runs on one GPU; a multi-GPU halo exchange is not implemented)", file=sys.stderr)
        return 2

    import torch
    from paper_2301_01622_amd import inputs
    from paper_2301_01622_amd.lbm import LBM

    n, q, tau = args.n, 27, 0.6
    rho, u = inputs.random_solenoidal_box(n, inputs.SEED_C2, umax=1e-3)
    rho_d, u_d = torch.from_numpy(rho).cuda(), torch.from_numpy(u).cuda()
    stream = torch.cuda.Stream()
    N = n ** 3
    side = max(args.steps, args.side_steps)
    reps = args.repeats

    with torch.cuda.stream(stream):
        spl = args.steps_per_sweep
        _log(f"headline: {n}^3 D3Q27 FP32, {args.steps} steps x {reps}")
        sim, sim_mem = _create(LBM, (n, n, n), q, tau, storage="f32", stream=stream, steps_per_sweep=spl)
        sim.set_equilibrium(rho_d, u_d)
        warm_ms = gpu_warmup(sim, args.gpu_warmup_ms)
        sim.set_equilibrium(rho_d, u_d)
        head = time_steps(sim, stream, args.steps, args.warmup, reps)
        ms = head["ms"]
        state_bytes, step_bytes = sim.memory_info()

        _log("one step per launch, adjoint, copy, split, population legs")
        # One step per launch, for comparison with the two-step sweeps.
        s1 = LBM((n, n, n), q, tau, storage="f32", stream=stream, steps_per_sweep=1)
        s1.set_equilibrium(rho_d, u_d)
        ms1 = time_steps(s1, stream, side, args.warmup, reps)["ms"]
        s1.close()

        adjoint = adjoint_cost(sim, stream, side, ms, single_ms=ms1, repeats=reps,
                               note="one species, same 256^3 D3Q27 FP32 box; the rollout's path: two adjoint steps "
                                    "per call (lbm_adjoint_step2_stored) and two recomputed states per call "
                                    "(lbm_step_state2); algorithmic bytes of one adjoint step 120 B/node (the "
                                    "two-step pass moves 80 B/node and step)")
        copy = None
        if args.calibrate_copy > 0:
            buf = sim.new_checkpoint()
            sim.save_state(buf)
            torch.cuda.synchronize()
            c0 = torch.cuda.Event(enable_timing=True)
            c1 = torch.cuda.Event(enable_timing=True)
            c0.record(stream)
            for _ in range(args.calibrate_copy):
                sim.save_state(buf)
            c1.record(stream)
            torch.cuda.synchronize()
            cms = c0.elapsed_time(c1) / args.calibrate_copy
            copy = {"bytes_per_launch": 2 * sim.state_bytes, "ms": round(cms, 5),
                    "gbs": round(2 * sim.state_bytes / (cms * 1e-3) / 1e9, 1)}
            del buf
        sim.close()

        # The paper's split approach on the same box: a collision pass, then
        # the streaming pass (same results, more bytes moved).
        sp = LBM((n, n, n), q, tau, storage="f32", stream=stream, split=True)
        sp.set_equilibrium(rho_d, u_d)
        sms = time_steps(sp, stream, side, args.warmup, reps)["ms"]
        _, s_step = sp.memory_info()
        sp.close()
        split = {
            "scheme": "moment LB as the split approach (collision pass + streaming pass, two launches)",
            "value": _rate(N, sms),
            "unit": "MLUPS",
            "ms_per_step": round(sms, 5),
            "bytes_per_node_step": s_step // N,
            "hbm_frac": round(s_step / (sms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "fused_speedup": round(sms / ms, 3),
        }

        pop = None
        if not args.no_population:
            ps, p_mem = _create(LBM, (n, n, n), q, tau, storage="f32", scheme="population", stream=stream)
            ps.set_equilibrium(rho_d, u_d)
            pms = time_steps(ps, stream, side, args.warmup, reps)["ms"]
            p_state, p_step = ps.memory_info()
            ps.close()
            pop = {
                "value": _rate(N, pms),
                "unit": "MLUPS",
                "ms_per_step": round(pms, 5),
                "hbm_frac": round(p_step / (pms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "bytes_per_node_state": p_state // N,
                "device_bytes_per_node": round(p_mem / N, 2),
            }
            # The same BGK scheme in place (AA pattern): one copy of the
            # populations, the same bytes moved per step.
            pa, a_mem = _create(LBM, (n, n, n), q, tau, storage="f32", scheme="population_aa", stream=stream)
            pa.set_equilibrium(rho_d, u_d)
            ams = time_steps(pa, stream, side, args.warmup, reps)["ms"]
            a_state, a_step = pa.memory_info()
            pa.close()
            pop["in_place"] = {
                "scheme": "population-storing BGK in place (AA pattern, one copy)",
                "value": _rate(N, ams),
                "unit": "MLUPS",
                "ms_per_step": round(ams, 5),
                "hbm_frac": round(a_step / (ams * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "bytes_per_node_state": a_state // N,
                "device_bytes_per_node": round(a_mem / N, 2),
            }
    del rho_d, u_d

    two = None
    if not args.no_two_component:
        _log("two-component 512x256x256 legs")
        two = two_component(side, args.warmup, reps)

    paper = None
    if not args.no_paper_workload:
        _log("paper workload 128^3")
        paper = paper_workload(side, args.warmup, reps)

    # Reduced-precision storage on 512^3 D3Q27 (tau = 0.55, shear wave plus
    # solenoidal noise): FP16 and BF16 moments, FP32 arithmetic.
    reduced = None
    if not args.no_reduced_precision:
        _log("reduced-precision 512^3 legs")
        reduced = {"workload": "512^3 periodic box, D3Q27, tau=0.55, u_x = 0.01 sin(2 pi y/512) + solenoidal noise "
                               "1e-4 (seed 16220004), 16-bit moments (rho-1, j, S scaled), FP32 arithmetic"}
        rho5, u5 = inputs.shear_wave_with_noise(512, seed=inputs.SEED_C4, u0=0.01, noise=1e-4)
        r5, v5 = torch.from_numpy(rho5).cuda(), torch.from_numpy(u5).cuda()
        del rho5, u5
        rs = torch.cuda.Stream()
        with torch.cuda.stream(rs):
            for st in ("f16", "bf16", "f32"):
                sm = LBM((512, 512, 512), q, 0.55, storage=st, stream=rs)
                sm.set_equilibrium(r5, v5)
                t = time_steps(sm, rs, max(side // 5, 20), 4, reps)["ms"]
                b_state, b_step = sm.memory_info()
                sm.close()
                reduced[st] = {"value": _rate(512 ** 3, t), "unit": "MLUPS",
                               "ms_per_step": round(t, 5), "bytes_per_node_state": b_state // 512 ** 3,
                               "bytes_per_node_step": b_step // 512 ** 3}
        del r5, v5

    mlups = N / (ms * 1e-3) / 1e6
    # Roofline of the sweep kernel: algorithmic bytes per launch (80 B per node
    # and step, two steps) over the launch time (two steps).
    launch_ms = spl * ms
    achieved = spl * step_bytes / (launch_ms * 1e-3) / 1e9
    traffic_bytes = measured_traffic(N) if spl == STEPS_PER_LAUNCH else None
    line = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{n}^3 periodic box, D3Q27, one component, FP32 moments (rho, j, P), tau=0.6, "
                        "random solenoidal velocity seed 16220002 max|u|=1e-3",
            "nodes": N,
            "lattice": "D3Q27",
            "storage": "f32",
        },
        "timing": {
            "gpu_warmup_ms": round(warm_ms, 1),
            "repeats": reps,
            "ms_per_step_repeats": head["repeats"],
            "statistic": "median over the repeats; each repeat times exactly `steps` steps with HIP events on "
                         "the library's stream, synchronised on both sides",
            "ms_per_step_end_to_end": round(head["e2e_ms"], 5),
            "value_end_to_end": _rate(N, head["e2e_ms"]),
            "side_leg_steps": side,
        },
        "roofline": {
            "bound": "hbm",
            "frac_kind": "effective",
            "limiter": "alu/lds",
            "kernel": "k_moment_sweep2 (two steps per launch)" if spl == 2 else "k_moment_tile (one step per launch)",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": round(traffic_bytes / (launch_ms * 1e-3) / 1e9, 1) if traffic_bytes else None,
            "steps_per_launch": spl,
            "ms_per_launch": round(launch_ms, 5),
            "algorithmic_bytes_per_launch": spl * step_bytes,
            "note": "achieved = algorithmic bytes of the step (every moment read and written once per node and "
                    "step, 80 B) x steps per launch / launch time.  The two-step sweep moves the state once per "
                    "launch, so this is an effective figure of the step, not HBM traffic; the HBM bytes the kernel "
                    "causes ('traffic', rocprofv3 FETCH_SIZE + WRITE_SIZE) are about half of it.  The kernel is "
                    "bound by vector ALU and LDS issue, not by HBM",
        },
        "single_step_kernel": {
            "value": _rate(N, ms1),
            "unit": "MLUPS",
            "ms_per_step": round(ms1, 5),
            "hbm_frac": round(step_bytes / (ms1 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        },
        "bytes_per_node_state": state_bytes // N,
        "device_bytes_per_node": round(sim_mem / N, 2),
        "copy_kernel": copy,
        "population_lb": pop,
    }
    if traffic_bytes:
        line["roofline"]["traffic_bytes_per_launch"] = traffic_bytes
        line["roofline"]["traffic_over_algorithmic"] = round(traffic_bytes / (spl * step_bytes), 4)
        line["roofline"]["traffic_frac"] = round(traffic_bytes / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    line["adjoint"] = adjoint
    line["split_approach"] = split
    if two:
        line["two_component"] = two
    if paper:
        line["paper_workload"] = paper
    if reduced:
        line["reduced_precision_storage"] = reduced
    if copy:
        line["roofline"]["frac_of_measured_copy"] = round(achieved / copy["gbs"], 4)
        line["single_step_kernel"]["frac_of_measured_copy"] = round(step_bytes / (ms1 * 1e-3) / 1e9 / copy["gbs"], 4)
    if pop:
        line["speedup_vs_population_lb"] = round(mlups / pop["value"], 3)
        line["speedup_vs_population_lb_in_place"] = round(mlups / pop["in_place"]["value"], 3)
    if not args.no_cpu_baseline:
        _log("CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(n, q, tau, args.cpu_steps, rho, u)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
