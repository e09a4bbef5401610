"""Benchmark: biased LJ atom-steps/s of the batched float32 path on one MI355X,
beside the plain float64 single-system path and the FP64 CPU oracle.

Workload (default): the largest batched single-GPU configuration, the 3D AFM
model (fcc 18x18x6 cells + R = 5 hemispherical tip, 8072 atoms) at 256 stepped
slider positions spread over one lattice period (2,066,432 atoms), slope bias
on, Langevin T = 0.1, gamma = 1, dt = 0.005.  Other workloads: --config C2 |
C3 | C4 | C5a | P2 | P3.  Inputs are synthetic lattices built by hd_inputs
(seeded).
--bias picks the bias variables: the slope alone (default) or the slope, the
curvature and the distance alone or two of them combined by eq. 13.

Setup (untimed): a FIRE quench on the GPU (hd_quench) gives each system's
basin reference r_O; an unbiased pre-run samples the bias variables, and the
thresholds of the slope and the curvature are their 5% and 50% quantiles, of
the distance its 95% and 50% quantiles (full bias up to the median distance,
none beyond the 95% one); dV_max = 5 kT, m = 2.  The timed
region is K steps of every system with inputs resident in HBM; neighbour-list
rebuilds are included.  It is timed --repeats times (each exactly K steps,
each bracketed by device synchronisations) and the median is reported; the
float64 legs are timed the same way over the same K steps.

Output: one JSON line (rank 0, one GPU).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "biased LJ atom-steps/s: batched FP32 vs plain FP64, force rel err ≤1e-5"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFS = 157.3
CSRC = os.path.join(ROOT, "paper_0909_5215_amd", "csrc")

# HBM bytes per launch of the stepping kernel, from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of this benchmark, each
# scaled by what the counter reads for a plain 256 MiB device copy run in the
# same process (FETCH_SIZE reads 131093 KiB for 262144 KiB moved: factor 2.0;
# WRITE_SIZE reads 262144 KiB: factor 1.0).  Keyed by workload and kernel, and
# tied to a hash of the kernel's sources: once they change, the figure no
# longer describes the kernel and the traffic is reported as null.
HBM_COUNTERS = {
    ("C2", "k_small<float, 2, 0, 512, false>"): {
        "src": ("hd_small.hip", "hd_device.h"), "sha": "c978c2324d5a47e0",
        "fetch_kib": 1013.2, "fetch_scale": 2.0, "write_kib": 2776.8, "write_scale": 1.0,
    },
    ("C2", "k_small<float, 2, 0, 512, true>"): {
        "src": ("hd_small.hip", "hd_device.h"), "sha": "c978c2324d5a47e0",
        "fetch_kib": 1003.0, "fetch_scale": 2.0, "write_kib": 2329.6, "write_scale": 1.0,
    },
    # the grid step as a whole: every kg_* launch of the float32 run (the
    # fused kick-drift, the rebuild launches, pairs, reduce) summed and
    # divided by its steps (per_step: scaled by the steps one launch covers)
    ("C5b", "grid step (kg_* kernels, timed as a whole)"): {
        "src": ("hd_grid.hip", "hd_device.h"), "sha": "f1d497e1e1363c4b",
        "fetch_kib": 437075.9, "fetch_scale": 2.0, "write_kib": 332248.3, "write_scale": 1.0,
        "per_step": True,
    },
}

# VALU wave-instructions of one launch of the stepping kernel (rocprofv3 --pmc
# SQ_INSTS_VALU, summed over the XCDs) and the steps that launch ran; tied to
# the kernel's sources like the HBM figures.  The chip issues at most one
# wave-instruction per CU per cycle (four SIMDs, 4 cycles per 64-lane
# instruction): 256 x 2.4 GHz = 614.4 G/s.
VALU_ISSUE_PEAK_G = 256 * 2.4
VALU_COUNTERS = {
    ("C2", "k_small<float, 2, 0, 512, false>"): {
        "src": ("hd_small.hip", "hd_device.h"), "sha": "c978c2324d5a47e0",
        "insts_valu": 831826855.1, "steps": 2000,
    },
    ("C2", "k_small<float, 2, 0, 512, true>"): {
        "src": ("hd_small.hip", "hd_device.h"), "sha": "c978c2324d5a47e0",
        "insts_valu": 798284070.6, "steps": 2000,
    },
    ("C5b", "grid step (kg_* kernels, timed as a whole)"): {
        "src": ("hd_grid.hip", "hd_device.h"), "sha": "f1d497e1e1363c4b",
        "insts_valu": 316915043.5, "steps": 1,
    },
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--config", default="C5b")
    ap.add_argument("--repeats", type=int, default=5, help="timed runs of K steps each; the median is reported")
    ap.add_argument("--bias", default="slope", choices=sorted(BIAS_CHOICES),
                    help="bias variables (eq. 13 combines two)")
    ap.add_argument("--thermostat", default="langevin", choices=["langevin", "nhc"],
                    help="Langevin BAOAB or the Nose-Hoover chain (3 thermostats, tau = 0.5)")
    ap.add_argument("--plain-steps", type=int, default=0, help="steps per system of the plain path (0 = the same K steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--skin", type=float, default=None,
                    help="neighbour-list skin of every system (default: the workload's, 0.3)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shape")
    ap.add_argument("--extras", action="store_true",
                    help="also time the lowest-eigenvalue search and its gradient on the paper's 3D model, "
                         "and one cycle of the parallel slider-position algorithm on this workload")
    ap.add_argument("--half-lists", type=int, choices=[0, 1], default=None,
                    help="with --no-autotune: LDS-resident float32 pair pass on half (1) or full (0) lists")
    ap.add_argument("--quench-steps", type=int, default=20000, help="FIRE iteration cap of the r_O quench")
    ap.add_argument("--prerun-steps", type=int, default=2000)
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (HBM counter calibration)")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def workload(name):
    from hd_inputs import CONFIGS
    specs = CONFIGS[name]()
    desc = {
        "C1": "2D LJ AFM 40x10+10x8 (480 atoms), 1 system, continuous sliding v=0.01",
        "C2": "2D LJ AFM 40x10+10x8 (480 atoms) x 32 slider positions, slope bias on",
        "C3": "3D LJ AFM fcc 20x20x6 + R=8 tip (10742 atoms) x 64 slider positions, slope bias on",
        "C4": "128 uneven 2D/3D instances (log-uniform 500-50k atoms), slope bias on",
        "C5a": "3D LJ AFM fcc 100x100x25 + R=20 tip (1017285 atoms), 1 system, slope bias on",
        "C5b": "3D LJ AFM fcc 18x18x6 + R=5 tip (8072 atoms) x 256 slider positions, slope bias on",
        "P2": "the paper's 2D model: triangular 80 + tip 33 (113 atoms), k = 5, T = 0.01 "
              "x 256 slider positions dx_S = 0.01, slope bias on",
        "P3": "the paper's 3D model: fcc 1800 + conical tip 183 with harmonic tip bonds (1983 atoms) "
              "x 256 slider positions dx_S = 0.01, slope bias on",
    }[name]
    return specs, desc


# bias variables: 0 slope (eq. 5), 1 curvature (eq. 6), 2 distance (eq. 7),
# 3 the lowest eigenvalue along a rotated mode (eq. 15)
BIAS_CHOICES = {"slope": (0, -1), "curvature": (1, -1), "distance": (2, -1), "eigenvalue": (3, -1),
                "slope+curvature": (0, 1), "slope+distance": (0, 2), "curvature+distance": (1, 2),
                "slope+eigenvalue": (0, 3)}
# the eigenvalue variable's mode estimate: a seeded random start, rotated
# once per step with this step (stable for these models' Hessian spectra)
MODE_ALPHA = 2e-4


def thresholds(var, samples):
    """Critical values (lower, upper) of a switch from unbiased samples."""
    a = np.asarray(samples)
    if var == 2:   # the distance: biased below a small value
        lo, hi = np.quantile(a, 0.95), np.quantile(a, 0.5)
        if not lo > hi:
            lo = hi + 1e-3 * (abs(hi) + 1.0)
    else:
        lo, hi = np.quantile(a, 0.05), np.quantile(a, 0.5)
        if not hi > lo:
            hi = lo + 1e-3 * (abs(lo) + 1.0)
    return float(lo), float(hi)


def prepare(hd, specs, quench_steps, prerun_steps, block):
    """Basin references by a FIRE quench, bias thresholds from an unbiased
    pre-run (both on the GPU, untimed).  Returns specs with rO and bias set and
    a checkpoint per system to start the timed runs from."""
    q = [s.copy() for s in specs]
    for s in q:
        s.bias_on, s.v_slider = 0, 0.0
    ctx = hd.make_context(q, precision=hd.HD_FP64, init_velocities=False, block_threads=block)
    t0 = time.perf_counter()
    iters, _, minima = ctx.quench(range(len(q)), ftol=1e-6, max_iters=quench_steps)
    quench = {"kind": "FIRE on the GPU (hd_quench), float64, all systems at once", "ftol": 1e-6,
              "seconds": round(time.perf_counter() - t0, 3), "converged": sum(1 for i in iters if i >= 0),
              "systems": len(iters), "max_iterations": max(abs(i) for i in iters)}
    log(f"FIRE quench: {quench}")
    for k, s in enumerate(specs):
        s.rO = minima[k]
    ctx.close()
    pre = [s.copy() for s in specs]
    for s in pre:
        s.bias_on = 0
    # float64 pre-run: the float32 stepping kernel then runs only in the
    # warm-up and the timed region, so its profile rows are the timed launches
    ctx = hd.make_context(pre, precision=hd.HD_FP64, init_velocities=True, block_threads=block)
    for k, s in enumerate(specs):
        ctx.set_positions(k, s.rO)       # start from the quenched basin
    ctx.step(prerun_steps // 2)
    samples = [[] for _ in specs]
    nsamp = 100
    every = max(1, prerun_steps // (2 * nsamp))
    for _ in range(nsamp):
        ctx.step(every)
        for k, sc in enumerate(ctx.scalars_batch()):
            samples[k].append((sc["g"], sc["kappa"], sc["d"], sc["lambda"]))
    states = []
    for k, s in enumerate(specs):
        v = np.array(samples[k])
        s.bias_on, s.m_b = 1, 2
        s.dv_max = 5.0 * s.kT
        s.g_lo, s.g_hi = thresholds(s.bias_var1, v[:, s.bias_var1])
        if s.bias_var2 >= 0:
            s.b2_lo, s.b2_hi = thresholds(s.bias_var2, v[:, s.bias_var2])
        states.append(ctx.get_state(k))
    ctx.close()
    return specs, states, quench


def interacting_pairs(specs, positions, max_systems=4):
    """Interacting unordered pairs per atom (r < rc, neither fixed-fixed nor
    rigid-rigid) and algorithmic float32 pair flops per atom-step, counted
    with a k-d tree on up to max_systems systems spread over the batch."""
    from scipy.spatial import cKDTree
    idx = sorted({int(round(k * (len(specs) - 1) / max(max_systems - 1, 1))) for k in range(max_systems)})
    pairs = flops = atoms = 0
    for k in idx:
        s, x = specs[k], np.asarray(positions[k])
        pts = x.T.copy()
        box = []
        for d in range(s.dim):
            if s.periodic[d]:
                pts[:, d] = np.mod(pts[:, d], s.box[d])
                box.append(s.box[d])
            else:
                lo = pts[:, d].min()
                pts[:, d] -= lo
                box.append(2.0 * (pts[:, d].max() + 2.0 * s.rc) + 1.0)   # open axis: no image within reach
        ij = cKDTree(pts, boxsize=np.array(box)).query_pairs(s.rc * (1.0 - 1e-12), output_type="ndarray")
        ri, rj = s.role[ij[:, 0]], s.role[ij[:, 1]]
        keep = ~(((ri == 1) & (rj == 1)) | ((ri == 2) & (rj == 2)))
        npair = int(keep.sum())
        pairs += npair
        flops += npair * (44 if s.dim == 2 else 57)
        atoms += s.n
    return pairs / atoms, flops / atoms


def src_hash(files):
    import hashlib
    m = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            m.update(fh.read())
    return m.hexdigest()[:16]


def stepping_kernel(specs, sched):
    """Name of the kernel that carries the float32 steps under the chosen
    launch shape: the LDS-resident kernel when every system runs in it, the
    one-workgroup global kernel, or the grid kernels timed together as one
    step."""
    nmax = max(s.n for s in specs)
    dim = specs[0].dim
    same_dim = all(s.dim == dim for s in specs)
    if sched["lds_resident"] and nmax <= 1024 and same_dim:
        half = "true" if sched.get("small_half_lists") else "false"
        return f"k_small<float, {dim}, 0, {sched['small_block']}, {half}>"
    if sched["persistent_large"] and same_dim:
        return f"k_batched<float, {dim}, 0, {sched['large_block']}>"
    return "grid step (kg_* kernels, timed as a whole)"


def make_run_ctx(hd, specs, states, precision, exec_mode, block):
    ctx = hd.Context(precision, 0, None, exec_mode, block, 0)
    for s in specs:
        ctx.add_system(s)
    ctx.finalize()
    for k, st in enumerate(states):
        ctx.set_state(k, st)
    return ctx


def extras(hd, torch, specs, states):
    """Untimed-path operations of the method, timed on their own: the
    lowest Hessian eigenvalue (Lanczos over GPU H u products) and its
    gradient on the paper's 3D model at its FIRE minimum; one placement and
    one cycle of the parallel slider-position algorithm on this workload."""
    from hd_inputs import build_3d_cone
    from paper_0909_5215_amd.sliding import ParallelSliding
    out = {}
    cone = build_3d_cone()
    c = hd.make_context([cone], precision=hd.HD_FP64, exec_mode=hd.HD_EXEC_GRID, init_velocities=False)
    c.quench([0], ftol=1e-8, max_iters=50000, set_reference=True)
    _, _, (xm,) = c.quench([0], ftol=1e-8, max_iters=50000)
    c.set_positions(0, xm)
    t0 = time.perf_counter()
    eps, iters, mode = c.min_mode(0, max_iter=400, tol=1e-9)
    t1 = time.perf_counter()
    c.min_mode_gradient(0, mode)
    t2 = time.perf_counter()
    out["min_mode"] = {"model": "the paper's 3D model (1983 atoms) at its FIRE minimum, float64, grid kernels",
                       "eps": eps, "lanczos_iterations": iters, "seconds": round(t1 - t0, 4),
                       "ms_per_hu_product": round((t1 - t0) * 1e3 / max(abs(iters), 1), 4),
                       "gradient_seconds": round(t2 - t1, 4)}
    c.close()
    log(f"extras: min_mode {out['min_mode']}")
    ctx = make_run_ctx(hd, specs, states, hd.HD_FP32C, hd.HD_EXEC_BATCHED, 0)
    dx = specs[1].x_slider - specs[0].x_slider if len(specs) > 1 else 0.01
    ps = ParallelSliding(ctx, x0=specs[0].x_slider, dx=dx, dtau=1000 * specs[0].dt, threshold=0.5,
                         ftol=1e-6, max_quench=20000, chunk=100, check_every=5)
    ctx.sync(); torch.cuda.synchronize()
    t0 = time.perf_counter()
    ps.start(0)
    ctx.sync(); torch.cuda.synchronize()
    t1 = time.perf_counter()
    cyc = ps.run_cycle()
    ctx.sync(); torch.cuda.synchronize()
    t2 = time.perf_counter()
    out["sliding_cycle"] = {"positions": len(specs), "dtau": ps.dtau, "start_seconds": round(t1 - t0, 4),
                            "cycle_seconds": round(t2 - t1, 4),
                            "check_quench_seconds": round(ps.quench_seconds, 4),
                            "check_ftol": ps.check_ftol, "steps_max": int(max(cyc.steps)),
                            "transitions": int(sum(cyc.transitions)), "k_star": cyc.k_star}
    ctx.close()
    log(f"extras: sliding {out['sliding_cycle']}")
    return out


def time_steps(torch, ctx, steps):
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms, launches = ctx.last_step_timing()
    return wall, ev_ms, launches


def time_repeats(torch, ctx, steps, repeats):
    """repeats timed runs of exactly `steps` steps; the run of median wall
    time (wall, HIP-event ms, launches) and every run's wall time."""
    runs = [time_steps(torch, ctx, steps) for _ in range(max(1, repeats))]
    order = sorted(range(len(runs)), key=lambda r: runs[r][0])
    med = runs[order[len(runs) // 2]]
    return med, [round(r[0], 6) for r in runs]


def cpu_baseline(specs, states_x, budget_s):
    """The FP64 oracle as it stands, timed on the host cores on a bounded
    sample of the same workload: every system (or as many as there are
    threads) for a number of steps chosen to fill about budget_s seconds."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as orc
    orc.build(force=False)
    cores = min(len(os.sched_getaffinity(0)), 16)
    nsys = min(len(specs), max(cores, 1))
    systems = []
    for k in range(nsys):
        s = specs[k]
        o = orc.OracleSystem(s)              # same drive reference as the GPU runs
        o.set_positions(states_x[k][0])
        o.set_velocities(states_x[k][1])
        systems.append(o)
    # calibrate
    t0 = time.perf_counter()
    systems[0].step(5)
    per_step = max(time.perf_counter() - t0, 1e-6) / 5
    steps = max(5, int(budget_s / per_step * min(1.0, cores / nsys)))
    steps = min(steps, 100000)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        list(ex.map(lambda o: o.step(steps), systems))
    wall = time.perf_counter() - t0
    atoms = sum(specs[k].n for k in range(nsys))
    # one core alone, a short bounded run of the first system
    one_steps = max(5, int(2.0 / per_step))
    t0 = time.perf_counter()
    systems[0].step(one_steps)
    one = specs[0].n * one_steps / (time.perf_counter() - t0)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": atoms * steps / wall, "unit": "atom-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{nsys} of {len(specs)} systems x {steps} steps (FP64 oracle, one thread per system)",
            "value_one_core": one, "cpu_model": model}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent slider positions would be split across GPUs with no per-step communication)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_0909_5215_amd import hd
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(3)
    torch.cuda.init()

    if args.copy_calib:
        # a plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE
        # counters calibrate the traffic of the kernels profiled beside it
        nbytes = args.copy_calib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {nbytes} bytes read and written per copy, 3 copies")
        del src, dst

    specs, desc = workload(args.config)
    v1, v2 = BIAS_CHOICES[args.bias]
    for k, s in enumerate(specs):
        if args.skin is not None:
            s.skin = args.skin
        s.bias_var1, s.bias_var2 = v1, v2
        if 3 in (v1, v2):
            s.mode = np.random.default_rng(9000 + k).standard_normal(s.pos.shape)
            s.mode_alpha = MODE_ALPHA
        if args.thermostat == "nhc":
            s.thermostat, s.nhc_len, s.nhc_tau = 1, 3, 0.5
    ckey = args.config if args.bias == "slope" else f"{args.config}/{args.bias}"
    if args.thermostat != "langevin":
        ckey += f"/{args.thermostat}"
    n_atoms = sum(s.n for s in specs)
    dim = specs[0].dim
    log(f"{args.config}: {len(specs)} systems, {n_atoms} atoms")
    specs, states, quench = prepare(hd, specs, args.quench_steps, args.prerun_steps, args.block)
    log("prepared (quench + pre-run)")

    # ---- batched float32 path ------------------------------------------------
    ctx = make_run_ctx(hd, specs, states, hd.HD_FP32C, hd.HD_EXEC_BATCHED, args.block)
    trials = []
    if not args.no_autotune:
        # launch shape from the autotuner (untimed; the state is left as it was)
        _, trials = ctx.autotune(min_ms=20.0, max_steps=8192)
    elif args.half_lists is not None:
        shape = ctx.schedule()
        shape["small_half_lists"] = args.half_lists
        ctx.set_schedule(shape)
    sched = ctx.schedule()
    log(f"schedule: {sched} ({len(trials)} shapes timed)")
    ctx.step(args.warmup)
    reb0 = [ctx.scalars(k)["n_rebuilds"] for k in range(len(specs))]
    (wall, ev_ms, launches), walls = time_repeats(torch, ctx, args.steps, args.repeats)
    value = n_atoms * args.steps / wall
    reb1 = [ctx.scalars(k)["n_rebuilds"] for k in range(len(specs))]
    rebuild_rate = float(np.mean(np.array(reb1) - np.array(reb0))) * 1000.0 / (args.steps * len(walls))
    flags = [ctx.scalars(k)["flags"] for k in range(len(specs))]
    t_hyper = [ctx.scalars(k)["t_hyper"] for k in range(len(specs))]
    t_md = [ctx.scalars(k)["t_md"] for k in range(len(specs))]
    log(f"batched fp32: {value:.4g} atom-steps/s, wall {wall:.3f}s, events {ev_ms:.1f} ms over {launches} launches")
    states_x = [(ctx.positions(k), ctx.velocities(k)) for k in range(len(specs))]

    # roofline of the dominant kernel (timed with HIP events on the stream it
    # runs on, averaged over its launches in the timed region): the
    # algorithmic bytes are the per-atom state read and written once per step
    # (x and v read+written, r_O read, float64): 5*D*8 bytes per atom-step
    alg_bytes_per_step = sum(5 * s.dim * 8 * s.n for s in specs)
    bytes_per_atom_step = alg_bytes_per_step / n_atoms
    kname = stepping_kernel(specs, sched)
    if kname.startswith("grid step"):
        # the grid kernels of one step are timed together as one unit
        steps_per_launch = 1.0
        avg_launch_s = (ev_ms / 1e3) / args.steps
    else:
        steps_per_launch = args.steps / max(launches, 1)
        avg_launch_s = (ev_ms / 1e3) / max(launches, 1)
    achieved = alg_bytes_per_step * steps_per_launch / avg_launch_s / 1e9
    traffic, traffic_bytes = None, None
    rec = HBM_COUNTERS.get((ckey, kname))
    if rec and src_hash(rec["src"]) == rec["sha"]:
        traffic_bytes = 1024.0 * (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"])
        if rec.get("per_step"):
            traffic_bytes *= steps_per_launch
        traffic = round(traffic_bytes / avg_launch_s / 1e9, 4)
    # measured VALU issue of the stepping kernel (counters above), against the
    # chip and against the CUs the launch occupies (one workgroup per system
    # for the LDS-resident kernel)
    issue = None
    vrec = VALU_COUNTERS.get((ckey, kname))
    if vrec and src_hash(vrec["src"]) == vrec["sha"]:
        rate = vrec["insts_valu"] * steps_per_launch / vrec["steps"] / avg_launch_s / 1e9
        cus = min(256, len(specs)) if kname.startswith("k_small") else 256
        issue = {"unit": "G wave-instr/s", "achieved": round(rate, 2), "peak": VALU_ISSUE_PEAK_G,
                 "frac": round(rate / VALU_ISSUE_PEAK_G, 4), "cus_occupied": cus,
                 "frac_of_occupied_cus": round(rate / (cus * 2.4), 4)}
    roof = {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": traffic,
            "kernel": kname, "avg_launch_ms": round(avg_launch_s * 1e3, 4),
            "steps_per_launch": steps_per_launch, "bytes_per_atom_step": round(bytes_per_atom_step, 3),
            "traffic_bytes_per_launch": traffic_bytes}

    # the arithmetic side: algorithmic float32 flops of the pair pass (44 per
    # interacting unordered pair in 2D, 57 in 3D), pairs counted on the host
    # at the end of the timed run, against the float32 vector peak
    ppa, fpa = interacting_pairs(specs, [x for x, _ in states_x])
    valu = {"bound": "alu", "achieved": round(fpa * value / 1e12, 4), "peak": FP32_PEAK_TFS, "unit": "TFLOP/s",
            "frac": round(fpa * value / 1e12 / FP32_PEAK_TFS, 6), "pairs_per_atom": round(ppa, 3),
            "flops_per_atom_step": round(fpa, 2)}

    # ---- plain float64 single-system path -----------------------------------
    plain = None
    if not args.no_plain:
        pctx = make_run_ctx(hd, specs, states, hd.HD_FP64, hd.HD_EXEC_SEQUENTIAL, args.block)
        psteps = args.plain_steps or args.steps
        pctx.step(min(args.warmup, psteps))
        (pwall, pev, pl), pwalls = time_repeats(torch, pctx, psteps, args.repeats)
        pval = n_atoms * psteps / pwall
        plain = {"value": pval, "unit": "atom-steps/s", "steps": psteps, "repeats": len(pwalls),
                 "walls_s": pwalls, "ms_per_step": pwall * 1e3 / psteps,
                 "kind": "plain FP64, one system at a time, per-step kernels replayed from HIP graphs"}
        log(f"plain fp64: {pval:.4g} atom-steps/s")
        pctx.close()

    # ---- the same batched path in float64 ------------------------------------
    fp64b = None
    if not args.no_plain:
        bctx = make_run_ctx(hd, specs, states, hd.HD_FP64, hd.HD_EXEC_BATCHED, args.block)
        if not args.no_autotune:
            bctx.autotune(min_ms=20.0, max_steps=8192)
        bsteps = args.steps
        bctx.step(args.warmup)
        (bwall, _, _), bwalls = time_repeats(torch, bctx, bsteps, args.repeats)
        fp64b = {"value": n_atoms * bsteps / bwall, "unit": "atom-steps/s", "steps": bsteps,
                 "repeats": len(bwalls), "walls_s": bwalls,
                 "ms_per_step": bwall * 1e3 / bsteps, "schedule": {k: v for k, v in bctx.schedule().items()
                                                                   if k != "ms_per_step"}}
        log(f"batched fp64: {fp64b['value']:.4g} atom-steps/s")
        bctx.close()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(specs, states_x, args.cpu_seconds)
        log(f"cpu oracle: {cpu['value']:.4g} atom-steps/s on {cpu['cores']} cores")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "repeats": len(walls),
        "walls_s": walls,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {desc}", "bias": args.bias, "thermostat": args.thermostat,
                   "skin": specs[0].skin,
                   "systems": len(specs), "atoms": n_atoms,
                   "dim": dim, "parallelism": "batch of independent slider positions, 1 GPU"},
        "roofline": roof,
        "roofline_valu": valu,
        "valu_issue": issue,
        "schedule": {k: sched[k] for k in ("lds_resident", "small_block", "persistent_large", "large_block")},
        "autotune_trials": [{k: (round(v, 6) if isinstance(v, float) else v) for k, v in t.items()} for t in trials],
        "cpu_baseline": cpu,
        "fp64_plain": plain,
        "fp64_batched": fp64b,
        "speedup_vs_fp64_plain": (value / plain["value"]) if plain else None,
        "unstable_systems": int(sum(1 for f in flags if f & 1)),
        "list_rebuilds_per_1000_steps": rebuild_rate,
        "mean_boost": float(np.mean(np.array(t_hyper) / np.maximum(np.array(t_md), 1e-300))),
        "r_O_quench": quench,
    }
    if args.extras:
        out["extras"] = extras(hd, torch, specs, states)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
