"""Benchmark: DEM + fluid-coupling steps on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c1|c0|c3|c3k] [--no-cpu]
                [--skin-factor F] [--lanes L] [--graphs 0|1] [--tune]

Workload c1: 200 000 polydisperse spheres in the hollow cylinder with the radial
Darcy inflow (mixed precision: FP64 positions/velocities, FP32 forces), inputs
resident in HBM before the timed region.  A step is one pass of the whole hot
path: kick/drift with outlet removal, neighbour-list rebuild when the skin is
exceeded, coupling (porosity, drag, cell drag source) every couple_every steps,
pair forces, fixed-order gather, walls, second kick.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# neighbour skin / smallest radius: c1 tuned over its 5 000-step run (the cavity face erodes and
# particles speed up, so a wider skin pays); the boxes keep the library default
SKIN_FACTOR = {"c1": 1.2, "c0": 0.4, "c3": 0.4, "c3k": 0.4, "f2": 0.4, "c4": 1.2}
LANES = 2           # lanes per particle of the row gather (the library default in half-pair mode)


KERNEL_SOURCES = {"step": ["dem_step.hip", "dem_device.h", "dem_internal.h"],
                  "fluid": ["dem_fluid.hip", "dem_device.h", "dem_internal.h"]}


def source_hash(files=None):
    """SHA-256 prefix of the kernel sources (a class's own files, or all)."""
    d = os.path.join(ROOT, "paper_2211_06142_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(files if files else os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def alg_bytes(cls, n_alive, n_pairs, n_cells, rsz):
    """Algorithmic bytes per launch of each kernel class: the per-unit figures
    of the method's state (mixed: FP64 x, v and FP32 omega, F, history; FP64
    mode: all FP64) times the units one launch processes.
      particle update: read x, v, omega, radius, flags; write x, v, omega
                       mixed 24+24+12+4+4 + 60 = 128 B, FP64 156 B
      half pair:       pair key 8 + history read and write + flags
                       mixed 8 + 24 + 4 = 36 B, FP64 60 B
      fluid cell:      u, grad p in, porosity and drag source out = 40 B
    The fused step kernel is one particle update plus one pass over the
    pairs; the coupling launch reads position, radius and velocity and writes
    the held force of every particle (24+4+24+12 = 64 B) and does one cell
    pass; the prologue is one particle update."""
    per_p = 128 if rsz == 4 else 156
    per_pair = 36 if rsz == 4 else 60
    if cls == "step":
        return n_alive * per_p + n_pairs * per_pair
    if cls == "prologue":
        return n_alive * per_p
    if cls == "fluid":
        return n_alive * 64 + n_cells * 40
    if cls == "rebuild":
        # one sort and permutation of the particle update state, one pass over the new pairs
        return n_alive * 2 * per_p + n_pairs * per_pair
    return 0


def load_traffic(kernel, workload, pair_mode="half"):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources (and, for the step class, in the
    same pair mode)."""
    path = os.path.join(ROOT, "profiles", "%s_%s_pmc.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash(d.get("sources")):
        return None
    if kernel == "step" and d.get("pair_mode", "half") != pair_mode:
        return None
    return d.get("traffic_bytes_per_launch")


def host_cpu():
    """The host's CPU model and the logical CPUs this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0))}


def cpu_baseline(w, budget_s=25.0):
    """The FP64 oracle on the same workload, single thread, bounded sample:
    the workload's own run length (c0: its 1 000 steps) or as many steps as the
    budget holds (about 1.5 s per step at 200 000 spheres, so some 15-20 steps,
    one or two coupling evaluations)."""
    import oracle
    from oracle import cg
    mat = cg.scale_material(w["material"], w.get("k", 1.0))
    op = oracle.make_params(mat, w["dt"], g=w["g"], walls=w["walls"], grid=w["grid"], fluid=w["fluid"],
                            outlet=w["outlet"])
    t0 = time.perf_counter()
    sim = oracle.OracleSim(op, w["x"], w["r"], bond_at_init=True)
    sim.set_fluid(w["u_cell"], w["gradp_cell"])
    t_init = time.perf_counter() - t0
    steps = 0
    t0 = time.perf_counter()
    while True:
        sim.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el > budget_s or steps >= w.get("steps", 200):
            break
    nal = int(sim.state()["alive"].sum())
    return {"value": nal * steps / el, "unit": "particle-steps/s", "cores": 1, "kind": "oracle", "host": host_cpu(),
            "sample": "%s: %d particles, first %d steps from the initial packing (incl. one coupling "
                      "evaluation per %d steps), %.1f s; setup %.1f s excluded"
                      % (w["name"], len(w["r"]), steps, w["fluid"]["couple_every"], el, t_init)}


def _oracle_sample(w, steps):
    """One ensemble sample on the FP64 oracle for `steps` steps from its
    initial packing: (particle-steps done, stepping seconds, setup seconds)."""
    import oracle
    from oracle import cg
    mat = cg.scale_material(w["material"], w.get("k", 1.0))
    op = oracle.make_params(mat, w["dt"], g=w["g"], walls=w["walls"], grid=w["grid"], fluid=w["fluid"],
                            outlet=w["outlet"])
    t0 = time.perf_counter()
    sim = oracle.OracleSim(op, w["x"], w["r"], bond_at_init=True)
    sim.set_fluid(w["u_cell"], w["gradp_cell"])
    t_init = time.perf_counter() - t0
    t0 = time.perf_counter()
    sim.step(steps)
    el = time.perf_counter() - t0
    done = float(sim.state()["alive"].sum()) * steps
    return done, el, t_init


def cpu_workers():
    """Worker processes for the all-core oracle run: the CPUs this process may
    use, at most 16 (the host share of one GPU)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def cpu_baseline_ensemble(ws, budget_s=25.0, steps=20, workers=1):
    """The FP64 oracle on the ensemble's samples in order, each for `steps`
    steps from its initial packing, until the budget is spent.  workers == 1:
    one sample at a time in this process (stepping time only); workers > 1:
    the samples are independent, so `workers` processes take them in order
    (the oracle itself stays single-threaded) and the rate is the work done
    over the wall time from the first submission to the last result, process
    start-up and per-sample setup included."""
    if workers <= 1:
        done, el, t_init, n_s = 0.0, 0.0, 0.0, 0
        for w in ws:
            d, e, t = _oracle_sample(w, steps)
            done, el, t_init, n_s = done + d, el + e, t_init + t, n_s + 1
            if el > budget_s:
                break
        how = "one at a time, single thread, %.1f s of stepping; setup %.1f s excluded" % (el, t_init)
    else:
        import concurrent.futures as cf
        import multiprocessing as mp
        t0 = time.perf_counter()
        done, n_s = 0.0, 0
        with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
            futs = [ex.submit(_oracle_sample, w, steps) for w in ws]
            for f in futs:   # in submission order; the pool works ahead
                d, _, _ = f.result()
                done, n_s = done + d, n_s + 1
                if time.perf_counter() - t0 > budget_s:
                    for g in futs:
                        g.cancel()
                    break
            # samples already running when the budget ran out finish; their work counts
            for g in futs[n_s:]:
                if not g.cancelled():
                    d, _, _ = g.result()
                    done, n_s = done + d, n_s + 1
        el = time.perf_counter() - t0
        how = ("%d worker processes (one single-threaded oracle each), %.1f s wall incl. process start-up "
               "and setup" % (workers, el))
    return {"value": done / el, "unit": "particle-steps/s", "cores": workers, "kind": "oracle", "host": host_cpu(),
            "sample": "%d of %d samples, %d steps each from their initial packings (incl. coupling "
                      "evaluations every %d steps), %s" % (n_s, len(ws), steps, ws[0]["fluid"]["couple_every"], how)}


MFMA_BF16_PEAK_TFLOPS = 2500.0
MLP_FLOP_FWD = 2 * (6 * 64 + 64 * 64 + 64 * 64 + 64 * 2)     # per sample


def time_events(torch, stream, fn, reps):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def closure_block(w, torch):
    """Network forward and training-step throughput (BF16 MFMA, FP32
    accumulation) at a batch of the workload's particle count, and the cost
    of the closure inside the coupling (features + inference for every
    particle), from instrumented coupling evaluations with and without it."""
    from paper_2211_06142_amd import dem
    n = len(w["r"])
    rng = np.random.default_rng(7)
    p0 = (rng.normal(0, 0.1, dem.MLP_NPARAMS)).astype(np.float32)
    net = dem.Mlp(p0)
    x = torch.as_tensor(rng.normal(size=(n, 6)).astype(np.float32), device="cuda")
    t = torch.as_tensor(rng.normal(0, 0.3, size=(n, 2)).astype(np.float32), device="cuda")
    y = torch.zeros((n, 2), dtype=torch.float32, device="cuda")
    stream = net.stream
    fwd = lambda: dem.dem_mlp_forward(net.h, x.data_ptr(), y.data_ptr(), n)
    fwd()
    ms_f = time_events(torch, stream, fwd, 50)
    trn = lambda: dem.dem_mlp_train_step(net.h, x.data_ptr(), t.data_ptr(), n, 1e-4)
    trn()
    ms_t = time_events(torch, stream, trn, 10)
    flop_f = MLP_FLOP_FWD * n
    out = {"batch": n, "forward_us": ms_f * 1e3, "forward_tflops": flop_f / (ms_f * 1e-3) / 1e12,
           "train_step_us": ms_t * 1e3, "train_tflops": 3 * flop_f / (ms_t * 1e-3) / 1e12,
           "mfma_peak_tflops": MFMA_BF16_PEAK_TFLOPS, "forward_frac": flop_f / (ms_f * 1e-3) / 1e12 / MFMA_BF16_PEAK_TFLOPS,
           "mfma": "v_mfma_f32_16x16x32_bf16 (hidden and output layers, weight gradients), "
                   "v_mfma_f32_16x16x16_bf16 (the 6 inputs, the 2 outputs backward)"}
    # closure inside the coupling: instrumented coupling class with and without
    norm = np.array([0.6, 0.05, 2.0, 1.0, 0.01, 4.0, 0.2, 0.05, 2.0, 1.0, 0.02, 3.0])
    per = {}
    for on in (False, True):
        sim = build_sim([w], SKIN_FACTOR["c1"], LANES, 0)
        if on:
            sim.set_closure(net, norm)
        sim.step(20)
        sim.profile(1)
        sim.step(200)
        prof = sim.read_profile()
        sim.profile(0)
        per[on] = prof["fluid"][0] * 1e3 / max(prof["fluid"][1], 1)
        sim.close()
    out["coupling_us_without"] = per[False]
    out["coupling_us_with"] = per[True]
    out["closure_us_per_evaluation"] = per[True] - per[False]
    net.close()
    return out


def parcel_layer_mass(wc):
    """Mass of one layer of parcels on the cavity face of a coarse cylinder:
    rho x solid fraction of the bed x cavity surface 2 pi r_cav h_bed x the
    parcels' mass-mean diameter."""
    r = wc["r"]
    r_cav = wc["outlet"][2]
    R = max(p[2] for kind, p in wc["walls"] if kind == 1)   # the outer cylinder wall
    h = wc["bed_top"]
    phi = float(np.sum(4.0 / 3.0 * np.pi * r ** 3)) / (np.pi * (R * R - r_cav * r_cav) * h)
    d = 2.0 * float(np.cbrt(np.mean(r ** 3)))
    return wc["material"]["rho"] * phi * 2.0 * np.pi * r_cav * h * d


def learned_cg_block(horizon, ks=(2, 3), c4=False):
    """The coarse-grained model against the fine run (the metric's second
    part), on three packings of the cylinder (seeds 0, 1, 2): for each k the
    closure is trained on the paired fine (c1) and coarse (c2, SSW) runs of
    seed 0, kept or dropped on seed 1 (kept only where it is not worse than the
    plain model), and the errors of the plain and the learned coarse model are
    reported on seed 2 (with c4: on the 2 000 000-grain cylinder and its k = 3
    parcels instead, run until the fine cylinder has produced ten layers of
    parcels from its cavity face), with the RMSRE over M(t).  The speedup is the fine run's
    wall time over the kept coarse model's on the reporting packing, both from
    the initial packing over the whole horizon."""
    import synth
    from paper_2211_06142_amd import closure_train as ct
    out = {"horizon_steps": horizon, "per_k": []}
    for k in ks:
        train = (synth.c1(seed=0), synth.c2(k, seed=0))
        judge = (synth.c1(seed=1), synth.c2(k, seed=1))
        report = (synth.c4(1), synth.c4(k)) if c4 else (synth.c1(seed=2), synth.c2(k, seed=2))
        layer = parcel_layer_mass(report[1]) if c4 else None
        res = ct.gain_test(train, judge, report, horizon=horizon, window=500, epochs=30,
                           report_mass=None if layer is None else 10.0 * layer,
                           log=lambda s: print("bench: learned-CG k=%d: %s" % (k, s), file=sys.stderr, flush=True))
        if layer is not None:
            res["parcel_layer_mass_kg"] = layer
        for key in ("net", "norm"):
            res.pop(key)
        for role in ("judge", "report"):
            res[role].pop("mass_series")
        res["within_5pct"] = bool(res["err_kept_cg"] <= 0.05)
        out["per_k"].append(res)
        print("bench: learned-CG k=%d done: report error plain %.4f learned %.4f (kept: %s), speedup %.2f" %
              (k, res["report"]["err_plain_cg"], res["report"]["err_learned_cg"],
               "learned" if res["closure_accepted"] else "plain", res["speedup_vs_fine"]), file=sys.stderr, flush=True)
    return out


def f2_fluid_setup(sim, w, u_inject=1e-4):
    """The paper's fluid run (section 3.1) on the f2 box: one coupling
    evaluation, then model A's pressure solve with the paper's boundary
    conditions (injection through the faces normal to y, top and bottom holes
    at the reference pressure); the equation is linear in the pressure, so the
    injection pressure is scaled to give the paper's injection velocity
    1e-4 m/s (superficial, mean over the open cells next to the injection
    face) and solved again; the fields go to the coupling."""
    import synth
    import torch
    sim.step(w["fluid"]["couple_every"])
    kind, pf = synth.f2_cell_kinds(w, 1.0)
    lo, hi, nn = w["grid"]
    nx, ny, nz = nn
    layer = np.zeros(nx * ny * nz, bool)
    for iz in range(nz):
        for ix in range(nx):
            layer[(iz * ny + 1) * nx + ix] = True
    layer &= kind == 0
    _, U, _, _, _ = sim.fluid_solve(kind, pf, max_iter=5000, rel_tol=1e-10)
    scale = u_inject / float(U[layer, 1].mean())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p, U, GP, it, rr = sim.fluid_solve(kind, pf * scale, max_iter=5000, rel_tol=1e-10)
    ms = (time.perf_counter() - t0) * 1e3
    sim.map_fluid(U, GP)
    return {"p_inject_pa": scale, "u_inject": float(U[layer, 1].mean()), "solve_iterations": it,
            "solve_rel_residual": rr, "solve_ms": ms, "p_max_pa": float(p.max())}


def calibrate_pmc(gib=2):
    """Known traffic for the HBM counters: three device copies of a buffer of
    `gib` GiB (far beyond the 256 MB Infinity Cache, so every byte crosses HBM:
    the buffer size read and written once each) and three read-only passes
    (a sum: the buffer read once).  Run under rocprofv3 --pmc FETCH_SIZE, then
    WRITE_SIZE; the counters of these kernels divided by the known bytes give the
    factors that turn the DEM kernels' counters into bytes."""
    import torch
    n = gib * 1024 ** 3 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    acc = 0.0
    for _ in range(3):
        acc += float(src.sum())
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "pmc", "bytes": 4 * n, "copies": 3, "reads": 3, "check": acc}), flush=True)


def build_sim(ws, skin_factor, lanes, graphs, pair_mode=None):
    from paper_2211_06142_amd import dem
    rmin = min(float(np.min(w["r"])) for w in ws)
    skin = skin_factor * rmin if skin_factor > 0 else 0.0
    params = [dem.params_from_workload(w, skin=skin) for w in ws]
    if len(ws) == 1:
        sim = dem.Simulation(params[0], ws[0]["x"], ws[0]["r"])
    else:
        offs = np.cumsum([0] + [len(w["r"]) for w in ws]).astype(np.int64)
        sim = dem.Simulation(params, np.concatenate([w["x"] for w in ws]), np.concatenate([w["r"] for w in ws]),
                             sample_offsets=offs)
    sim.map_fluid(np.concatenate([w["u_cell"] for w in ws]), np.concatenate([w["gradp_cell"] for w in ws]))
    sim.set_lanes(lanes)
    sim.set_graphs(graphs)
    if pair_mode is not None:
        sim.set_pair_mode(pair_mode)
    return sim


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="c1", choices=["c1", "c0", "c3", "c3k", "f2", "c4"],
                    help="c3k: the ensemble with per-sample coarse-graining k = 1, 2, 3; f2: the paper's own "
                    "setting (18 x 18 x 9 mm box, Table 2 sand, Table 3 material, dt 1e-8 s, top outlet)")
    ap.add_argument("--f2-k", type=int, default=1, help="coarse-graining factor of the f2 run (1 or 2, SSW)")
    ap.add_argument("--f2-protocol", action="store_true", help="f2 from the paper's stages: the generated bed "
                    "compressed by the top plate to 1 MPa (servo), then perforated, then the sand-production run")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=25.0, help="seconds of oracle stepping (cpu_baseline)")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle processes for an ensemble's cpu_baseline (0: all usable CPUs, at most 16)")
    ap.add_argument("--skin-factor", type=float, default=None,
                    help="neighbour skin as a multiple of the smallest radius (default per workload)")
    ap.add_argument("--lanes", type=int, default=LANES, help="lanes per particle of the step kernel")
    ap.add_argument("--graphs", type=int, default=0, help="replay recorded step windows in the timed region "
                    "(measured slower on this part: c1 0.0617 against 0.0595 ms per step, c3 0.645 against 0.626)")
    ap.add_argument("--pair-mode", default=None, choices=["full", "half"],
                    help="contact evaluation: full rows (each pair twice) or half pairs with force records")
    ap.add_argument("--tune", action="store_true", help="autotune skin and lanes before the timed run")
    ap.add_argument("--no-closure", action="store_true", help="skip the learned-closure measurement (network "
                    "throughput on the matrix cores, cost inside the coupling)")
    ap.add_argument("--no-learned-cg", action="store_true", help="skip the coarse-grained model against the "
                    "fine run (paired runs, closure training, produced-mass error and speedup)")
    ap.add_argument("--cg-horizon", type=int, default=20000, help="steps of the fine/coarse comparison")
    ap.add_argument("--cg-c4", action="store_true", help="the comparison on c4 (2 000 000 fine grains against "
                    "k = 3 parcels) instead of c1 against c2 (needs the c4 packings, about an hour to generate)")
    ap.add_argument("--calibrate-pmc", action="store_true", help="only run the counter calibration kernels "
                    "(a 2 GiB copy and read, run under rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.calibrate_pmc:
        calibrate_pmc()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU only; sharding the DEM step over several GPUs is designed but not "
              "implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2211_06142_amd import tune

    if args.workload == "c1":
        ws = [synth.c1()]
    elif args.workload == "f2" and args.f2_protocol:
        from paper_2211_06142_amd import paper_setting
        bed = synth.f2_bed(args.f2_k)
        t0 = time.perf_counter()
        comp = paper_setting.compress(bed, log=lambda m: print("bench: " + m, file=sys.stderr, flush=True))
        compression = {"stress_pa": comp["stress"], "plate_height_m": comp["plate_z"], "porosity": comp["porosity"],
                       "cycles": comp["cycles"], "steps": comp["steps"], "converged": comp["converged"],
                       "wall_s": time.perf_counter() - t0, "grains": len(bed["r"])}
        ws = [paper_setting.perforate(comp, bed)]
        comp["sim"].close()
        print("bench: compressed to %.4g Pa, porosity %.4f, plate %.4f mm" % (comp["stress"], comp["porosity"],
              comp["plate_z"] * 1e3), file=sys.stderr, flush=True)
    elif args.workload == "f2":
        if args.f2_k == 1:
            # all 250 000 Table 3 grains straight from the geometric packing: the
            # packing's overlaps under E = 20 GPa launch grains faster than half
            # the skin per step, which the library refuses (fault "too fast")
            print("bench.py: the f2 sample at k = 1 runs from its compressed state only: add --f2-protocol",
                  file=sys.stderr)
            sys.exit(2)
        ws = [synth.f2(args.f2_k)]
    elif args.workload == "c4":
        ws = [synth.c4(1)]
    elif args.workload == "c0":
        ws = [synth.c0()]
    else:
        ws = synth.c3(k_sweep=args.workload == "c3k")
    w = ws[0]
    if args.skin_factor is None:
        args.skin_factor = SKIN_FACTOR[args.workload]
    tuned = None
    if args.tune:
        best, table = tune.tune_workload(ws if len(ws) > 1 else w, log=lambda m: print(m, file=sys.stderr, flush=True))
        rmin = min(float(np.min(x["r"])) for x in ws)
        args.skin_factor, args.lanes = best["skin"] / rmin, best["lanes"]
        tuned = {"skin_factor": args.skin_factor, "lanes": args.lanes, "trials": table}
    sim = build_sim(ws, args.skin_factor, args.lanes, args.graphs, args.pair_mode)
    f2_fluid = f2_fluid_setup(sim, w) if args.workload == "f2" else None
    n_total = sum(len(x["r"]) for x in ws)
    print("bench: %s set up, %d particles in %d sample(s)" % (args.workload, n_total, len(ws)), file=sys.stderr,
          flush=True)
    sim.step(args.warmup)
    n0 = sim.state()["n_alive"]
    print("bench: %d warm-up steps done, %d rebuilds" % (args.warmup, sim.info()["rebuilds"]), file=sys.stderr,
          flush=True)
    stream = sim.stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    # timed region: the steps alone (no per-launch events inside)
    torch.cuda.synchronize()
    ev0.record(stream)
    t0 = time.perf_counter()
    sim.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    n1 = sim.state()["n_alive"]
    print("bench: %d timed steps done in %.1f ms" % (args.steps, ms), file=sys.stderr, flush=True)
    # instrumented pass for the kernel breakdown: HIP events recorded on the
    # context's stream around every launch of each kernel class
    # (timing launches one by one: with graphs on, these steps run without them)
    prof_steps = max(200, args.steps // 5)
    sim.profile(1)
    sim.step(prof_steps)
    prof = sim.read_profile()
    sim.profile(0)
    print("bench: %d instrumented steps done" % prof_steps, file=sys.stderr, flush=True)
    st = sim.state()
    inf = sim.info()
    n_alive = 0.5 * (n0 + n1)
    value = n_alive * args.steps / (ms * 1e-3)
    rsz = 8 if w["precision"] == "fp64" else 4
    roofline, kernels = None, None
    if prof:
        # the dominant class; launches that found a rebuild due (exit at entry) are excluded by the library
        dom = max(prof, key=lambda k: prof[k][0])
        dom_ms, dom_n = prof[dom]
        avg_s = dom_ms * 1e-3 / max(dom_n, 1)
        ab = alg_bytes(dom, n_alive, inf["n_pairs"], inf["ncell"], rsz)
        achieved = ab / avg_s / 1e9
        kernels = {k: {"total_ms": round(v[0], 3), "launches": v[1],
                       "avg_us": round(1e3 * v[0] / max(v[1], 1), 3),
                       "alg_GBs": round(alg_bytes(k, n_alive, inf["n_pairs"], inf["ncell"], rsz) /
                                        (v[0] * 1e-3 / max(v[1], 1)) / 1e9, 1) if v[1] else None,
                       "traffic": load_traffic(k, args.workload, args.pair_mode or "half")}
                   for k, v in prof.items()}
        roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": load_traffic(dom, args.workload, args.pair_mode or "half"),
                    "alg_bytes_per_launch": ab, "avg_launch_us": avg_s * 1e6, "instrumented_steps": prof_steps}
    if args.workload == "c3":
        desc = ("c3: batched ensemble of %d independent samples (crops of the settled C1 bed, 500-20 000 "
                "spheres each, surface energy 0.1-1.0 J/m^2, own walls and 8-16^3 fluid grid), %d spheres in "
                "total, dt 1e-7 s, coupling every %d steps" % (len(ws), n_total, w["fluid"]["couple_every"]))
        metric = "particle-steps/s, batched ensemble of 256 samples, 1 GPU"
    elif args.workload == "c3k":
        desc = ("c3k: batched ensemble of %d independent samples with coarse-graining k = 1, 2, 3 by turns "
                "(crops of the settled C1 bed and of its k = 2 and k = 3 parcel beds, 500-20 000 fine-equivalent "
                "grains each, surface energy 0.1-1.0 J/m^2, own walls and 8-16^3 fluid grid), %d spheres and "
                "parcels in total, dt 1e-7 s, coupling every %d steps" % (len(ws), n_total, w["fluid"]["couple_every"]))
        metric = "particle-steps/s, batched ensemble of 256 samples with k = 1, 2, 3, 1 GPU"
    elif args.workload == "f2":
        desc = ("f2: the paper's setting after perforation, %d %s (Table 2 sand%s, Table 3 material) in an 18 x 18 x 9 mm "
                "box with a 1.7 mm perforation tunnel and a 2.6 mm outlet hole in the top plate, 12x12x6 fluid grid, "
                "injection 1e-4 m/s through the faces normal to y (model A pressure solve), dt 1e-8 s, coupling every "
                "%d steps" % (len(w["r"]), "grains" if w["k"] == 1 else "SSW parcels",
                              "" if w["k"] == 1 else ", k = %g" % w["k"], w["fluid"]["couple_every"]))
        metric = "particle-steps/s at %d particles (paper setting), 1 GPU" % len(w["r"])
    elif args.workload == "c0":
        desc = ("c0: %d spheres settled in a 3 mm box (six walls), 8^3 fluid grid, uniform upward flow, FP64, "
                "dt 1e-7 s, coupling every %d steps" % (len(w["r"]), w["fluid"]["couple_every"]))
        metric = "particle-steps/s at %d particles, 1 GPU" % len(w["r"])
    else:
        desc = ("%s: %d polydisperse spheres (lognormal d, median 0.15 mm), hollow cylinder R 12 mm / cavity "
                "2 mm, 48x48x24 fluid grid, radial Darcy inflow, dt 1e-7 s, coupling every %d steps"
                % (w["name"], len(w["r"]), w["fluid"]["couple_every"]))
        if args.workload == "c4":
            desc = ("c4: %d polydisperse spheres (lognormal d, median 0.15 mm), the c1 cylinder scaled by 10^(1/3) "
                    "(R 25.85 mm / cavity 4.31 mm), 103x103x52 fluid grid, radial Darcy inflow, dt 1e-7 s, coupling "
                    "every %d steps" % (len(w["r"]), w["fluid"]["couple_every"]))
        metric = ("particle-steps/s at 200k particles, 1 GPU" if args.workload == "c1"
                  else "particle-steps/s at %d particles, 1 GPU" % len(w["r"]))
    out = {
        "metric": metric,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64-positions/f32-forces" if rsz == 4 else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "n_particles": n_total, "n_samples": len(ws), "n_alive_mean": n_alive,
                   "n_pairs": inf["n_pairs"], "rebuilds": inf["rebuilds"], "packing_sha256": w["sha256"][:16],
                   "produced_mass_kg": st["produced_mass"], "coordination": st["coordination"],
                   "broken_bonds": st["broken_bonds"], "skin_factor": args.skin_factor, "lanes": args.lanes,
                   "graphs": bool(args.graphs), "parallelism": "single GPU"},
        "roofline": roofline,
        "kernels": kernels,
        "wall_s": wall,
    }
    if tuned:
        out["config"]["tuned"] = tuned
    if f2_fluid:
        out["config"]["fluid_solve"] = f2_fluid
    if args.workload == "f2" and args.f2_protocol:
        out["config"]["compression"] = compression
    if not args.no_closure and len(ws) == 1:
        out["closure"] = closure_block(w, torch)
    sim.close()
    if not args.no_learned_cg and args.workload == "c1":
        out["learned_cg"] = (learned_cg_block(args.cg_horizon, ks=(3,), c4=True) if args.cg_c4
                             else learned_cg_block(args.cg_horizon))
    if not args.no_cpu:
        out["cpu_baseline"] = (cpu_baseline(w, args.cpu_budget) if len(ws) == 1
                               else cpu_baseline_ensemble(ws, args.cpu_budget,
                                                          workers=args.cpu_workers or cpu_workers()))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
