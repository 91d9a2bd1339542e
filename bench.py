#!/usr/bin/env python3
"""Throughput of the fused pseudopotential-LBM step on one MI355X.

Workload (the metric's configuration): droplet vaporisation on 512 x 512
periodic lattices, seeds 0-3 -- a liquid disk of radius 60 (seed-jittered by
+-0.5) at T_sat = 0.86 T_c in vapour held at 0.95 T_c on the outer ring,
Peng-Robinson EOS a = 2/49, b = 2/21, sigma = kappa = 0.1, all MRT rates
1.25, c_v = 6, lambda = 2/3, no gravity, energy equation on from step 0.  A
step advances the four seeds by one time step: the float32 shifted-storage
step runs them in one batched launch per step (graph-replayed), the float64
plain step one lattice after another.  The float32 accuracy is stated after
the configuration's 20,000 steps on all four seeds, whatever --steps is.

Prints ONE JSON line (last line of stdout) with the metric, the roofline
of the step kernel (HIP events around the timed launches), the float64
comparison, the single-lattice figures, an HBM-sized run (4096 x 4096 pool
boiling physics: walls, heater, gravity), the refinement ladder, the
adjoint, and the float64 oracle timed on one pinned host core.
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_bytes_per_node(fp32, thermal=True):
    """Populations in and out (9 + 9) and T in and out: 80 B (float32) /
    160 B (float64) per lattice update."""
    e = 4 if fp32 else 8
    return (18 + (2 if thermal else 0)) * e


def vaporisation_case(n=512, seed=0):
    import paper_2201_04560_amd as pp
    import workloads as wl

    a = 2.0 / 49.0
    Tc = pp.pr_critical_temperature(a)
    Tsat, Tout = 0.86 * Tc, 0.95 * Tc
    rv, rl, _ = pp.pr_maxwell(a, Tsat)
    rho, T = wl.droplet(n, n, 60.0 * n / 512, 4.6 / 5.0, rl, rv, Tsat, Tout, seed=seed)
    kw = dict(a=a, sigma=0.1, kappa=0.1, rho_l=rl, rho_v=rv, thermal=1, cv=6.0,
              lambda_l=2.0 / 3.0, lambda_v=2.0 / 3.0, t_side_dirichlet=1, t_side_val=Tout, rho_ref=rv)
    kw.update({k: v for k, v in wl.DROPLET_RATES.items()})
    bnd = dict(t_bottom_kind=1, t_bottom_val=Tout, t_top_kind=1, t_top_val=Tout)
    return n, n, kw, bnd, rho, T


def pool_case(nx=4096, ny=4096, level=5):
    """Pool boiling on nx x ny read as mesh `level` of the refinement
    procedure (Sec. 3) over a base mesh 2^level times coarser (a = 2/49,
    g = -3e-5 on the base mesh; a, sigma, kappa and g rescaled per mesh):
    liquid below 1400/2048 of the height at T_sat = 0.86 T_c, heater strip of
    width nx/8 at 0.95 T_c (wall density 3.44), adiabatic elsewhere, top
    wall at T_sat, seeded nucleation half-disk."""
    import workloads as wl
    from paper_2201_04560_amd.ladder import pool_level

    L = pool_level(level, base_nx=nx >> level, base_ny=ny >> level, steps0=0)
    lv, p = L["level"], L["params"]
    rho, T = wl.pool(nx, ny, ny * 1400.0 / 2048.0, 2.3 * 2 ** level, lv["rho_l"], lv["rho_v"],
                     lv["T"], seed_radius=8.0 * 2 ** level / 8.0, seed=0)
    kw = {k: getattr(p, k) for k in ("a", "b", "omega", "sigma", "kappa", "rho_l", "rho_v", "walls",
                                     "thermal", "gy", "cv", "lambda_l", "lambda_v", "rho_ref",
                                     "s_rho", "s_e", "s_zeta", "s_j", "s_q", "eta_l", "eta_v")}
    return nx, ny, kw, L["boundary"], rho, T


def device_key():
    """Architecture and compute-unit count of GPU 0 (the tile cache key)."""
    import torch

    pr = torch.cuda.get_device_properties(0)
    return f"{pr.gcnArchName.split(':')[0]}/{pr.multi_processor_count}CU"


def run_lattice(case, precision, warmup, steps, want_fields=True, tile_y=0, tune=None, strip_waves=0):
    """Warm up, then time `steps` launches of the step kernel: host wall
    clock around the whole region, and one pair of HIP events recorded on the
    lattice's stream around the same launches (their mean is the kernel's
    average launch duration, inter-launch gaps included).  tile_y = 0 with a
    TileCache picks the strip height with the library's autotuner."""
    import torch

    from paper_2201_04560_amd import Lattice, make_params

    nx, ny, kw, bnd, rho, T = case
    lat = Lattice(make_params(nx, ny, precision=precision, tile_y=tile_y, strip_waves=strip_waves,
                              **kw))
    lat.set_boundary(**bnd)
    lat.init_fields(rho, None, None, T)
    if tile_y == 0 and tune is not None:
        tune.tune(lat, device=device_key())
    if warmup:
        lat.step(warmup)
    lat.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    lat.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ev = lat.last_step_ms()
    out = dict(wall_s=t1 - t0, ev_ms=ev, kernel_ms_avg=ev / steps, launches=steps, tile_y=lat.tile_y,
               strip_waves=lat.strip_waves)
    if want_fields:
        out["fields"] = lat.fields()
        out["norms"] = lat.norms()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return out


SEEDS = (0, 1, 2, 3)


def vap_lattices(precision, seeds=SEEDS, tile_y=0, strip_waves=0, n=512, **over):
    """One initialised lattice of the vaporisation workload per seed."""
    from paper_2201_04560_amd import Lattice, make_params

    out = []
    for sd in seeds:
        nx, ny, kw, bnd, rho, T = vaporisation_case(n, seed=sd)
        lat = Lattice(make_params(nx, ny, precision=precision, tile_y=tile_y,
                                  strip_waves=strip_waves, **dict(kw, **over)))
        lat.set_boundary(**bnd)
        lat.init_fields(rho, None, None, T)
        out.append(lat)
    return out


def tune_vap_batch(tune, precision, seeds=SEEDS):
    """(strip height, waves per strip) of the batched launch of the seeds,
    from the tile cache or its autotuner (throwaway lattices)."""
    if tune is None:
        return 5, 2
    return tune.tune_batch(lambda: vap_lattices(precision, seeds), device=device_key(),
                           candidates=(4, 5, 6, 8, 10, 12, 13, 16, 20, 24, 32), steps=20,
                           waves=(1, 2), with_waves=True)


def pick_launch_mode(precision, tile_y, waves, seeds=SEEDS, steps=200):
    """Graph replay or direct launches for the batched step: the faster of
    the two over `steps` steps on throwaway lattices (on MI355X with ROCm 7
    the graph-replayed launches ran about 1 % slower than direct ones for
    this 25 us kernel; graphs pay off where launches are shorter than their
    host cost, as on the small meshes of the refinement ladder)."""
    best = None
    for use_graph in (True, False):
        r = run_vap_batch(precision, 20, steps, tile_y, waves, seeds, want_fields=False,
                          use_graph=use_graph)
        if best is None or r["wall_s"] < best[1]:
            best = (use_graph, r["wall_s"])
    return best[0]


def run_vap_batch(precision, warmup, steps, tile_y, waves, seeds=SEEDS, want_fields=True,
                  use_graph=True):
    """The seeds advanced together: one multi-lattice launch per step,
    repeated launch pairs replayed from a captured graph (use_graph) or
    launched one by one.  Host wall clock around the timed run; the batch's
    HIP events (recorded on its stream around the same launches) give the
    kernel's average launch duration."""
    import torch

    from paper_2201_04560_amd import Batch

    lats = vap_lattices(precision, seeds, tile_y, waves)
    b = Batch(lats)
    n = len(lats)
    if warmup:
        b.run([warmup] * n, use_graph=use_graph)
    # tables (and graphs) of the timed schedule set up ahead (no launch)
    b.prepare([steps] * n, use_graph=use_graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run([steps] * n, use_graph=use_graph)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms, launches, graphs = b.last_time()
    out = dict(wall_s=wall, ev_ms=ms, kernel_ms_avg=ms / max(launches, 1), launches=launches,
               graph_launches=graphs, tile_y=lats[0].tile_y, strip_waves=lats[0].strip_waves,
               use_graph=use_graph)
    if want_fields:
        out["fields"] = [lat.fields() for lat in lats]
        out["norms"] = [lat.norms() for lat in lats]
        out["populations0"] = lats[0].populations()
    b.close()
    for lat in lats:
        lat.close()
    torch.cuda.empty_cache()
    return out


def run_vap_plain(precision, warmup, steps, seeds=SEEDS, tile_y=0, waves=0, want_fields=True):
    """The plain step: the seeds one lattice after another, one launch per
    step each (the library's default strip height and waves per strip)."""
    import torch

    lats = vap_lattices(precision, seeds, tile_y, waves)
    for lat in lats:
        if warmup:
            lat.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for lat in lats:
        lat.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev = sum(lat.last_step_ms() for lat in lats)
    out = dict(wall_s=wall, ev_ms=ev, kernel_ms_avg=ev / (steps * len(lats)), launches=steps * len(lats),
               tile_y=lats[0].tile_y, strip_waves=lats[0].strip_waves)
    if want_fields:
        out["fields"] = [lat.fields() for lat in lats]
        out["norms"] = [lat.norms() for lat in lats]
    for lat in lats:
        lat.close()
    torch.cuda.empty_cache()
    return out


def batch_bitwise_vs_solo(res, precision, nsteps, seed=SEEDS[0]):
    """The batched run's first lattice against the same seed stepped alone
    (lbm_step, same strip height and waves): identical bits expected."""
    import torch

    lat = vap_lattices(precision, (seed,), res["tile_y"], res["strip_waves"])[0]
    lat.step(nsteps)
    same = bool(np.array_equal(lat.populations(), res["populations0"]))
    lat.close()
    torch.cuda.empty_cache()
    return same


def accuracy_20k(steps, tune, seeds=SEEDS):
    """Float32 shifted storage against the float64 step after the
    configuration's length on every seed: max relative rho / T deviation,
    mass, liquid fraction, droplet radius and coexistence densities; the
    float32 storage with rho_ref = the mean density on seed 0."""
    ty32, w32 = tune_vap_batch(tune, 1, seeds)
    t0 = time.perf_counter()
    r32 = run_vap_batch(1, 0, steps, ty32, w32, seeds)
    r64 = run_vap_batch(0, 0, steps, 5, 2, seeds)
    nx, ny, kw, bnd, rho0, T0 = vaporisation_case(512, seed=seeds[0])
    rl, rv = kw["rho_l"], kw["rho_v"]
    mid = 0.5 * (rl + rv)
    per = []
    for k, sd in enumerate(seeds):
        a, _, _, Ta = r32["fields"][k]
        c, _, _, Tc = r64["fields"][k]
        per.append({"seed": sd, "rho_max_rel": rel_err(a, c), "T_max_rel": rel_err(Ta, Tc),
                    "mass_rel": abs(r32["norms"][k]["mass"] / r64["norms"][k]["mass"] - 1),
                    "liquid_fraction_fp32": float((a > mid).mean()),
                    "liquid_fraction_fp64": float((c > mid).mean()),
                    "fp32": droplet_stats(a, rl, rv), "fp64": droplet_stats(c, rl, rv)})
    mean_ref = float(rho0.mean())
    lm = vap_lattices(1, (seeds[0],), 5, 2, rho_ref=mean_ref)[0]
    lm.step(steps)
    rm, _, _, Tm = lm.fields()
    lm.close()
    c, _, _, Tc = r64["fields"][0]
    return {"after_steps": steps, "seeds": list(seeds),
            "rho_max_rel": max(p["rho_max_rel"] for p in per),
            "T_max_rel": max(p["T_max_rel"] for p in per),
            "mass_rel": max(p["mass_rel"] for p in per),
            "per_seed": per,
            "fp32_rho_ref_mean_seed0": {"rho_ref": mean_ref, "rho_max_rel": rel_err(rm, c),
                                        "T_max_rel": rel_err(Tm, Tc), **droplet_stats(rm, rl, rv)},
            "wall_s": round(time.perf_counter() - t0, 2)}


def roofline(fp32, nodes, kernel_ms, traffic):
    b = alg_bytes_per_node(fp32) * nodes
    achieved = b / (kernel_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "alg_bytes_per_launch": b, "kernel_ms_avg": round(kernel_ms, 5)}


def measured_traffic(key, tile_y, waves):
    """HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a
    copy kernel of known size) from the committed counter summary, valid only
    for the kernel sources, strip height and waves per strip they were taken
    on."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
        h = hashlib.sha256()
        for f in t.get("kernel_sources", []):
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        if not t.get("kernel_sources") or t.get("kernel_sha256") != h.hexdigest():
            return None
        return t.get("per_launch_bytes", {}).get(key, {}).get(f"{tile_y}x{waves}")
    except (OSError, ValueError):
        return None


KERNEL_SOURCES = ["paper_2201_04560_amd/csrc/lbm_step.hip", "paper_2201_04560_amd/csrc/lbm_device.hpp",
                  "paper_2201_04560_amd/csrc/lbm_kernels.hpp"]
PROFILE_NODES = {"vaporisation512": 512 * 512, "vaporisation512x4": 4 * 512 * 512,
                 "pool4096": 4096 * 4096}


def write_traffic(pmc_dir, copy_mib):
    """Build profiles/traffic.json from rocprofv3 --pmc runs of the profile
    mode: one directory per counter, named pmc_<case>_<prec>_<TY>x<W>_<CTR>
    (CTR FETCH_SIZE or WRITE_SIZE), each holding run_counter_collection.csv.
    Each counter is scaled by what it reads for the largest device copy of
    the same run (copy_mib MiB read and written) and averaged over the
    step-kernel dispatches."""
    import csv
    import glob

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    per = {}
    for f in sorted(glob.glob(os.path.join(pmc_dir, "pmc_*", "run_counter_collection.csv"))):
        parts = os.path.basename(os.path.dirname(f))[4:].split("_")
        case, cfg, ctr = "_".join(parts[:2]), parts[2], "_".join(parts[3:])
        with open(f) as fh:
            rows = list(csv.DictReader(fh))
        march = [float(r["Counter_Value"]) for r in rows if "lbm_march" in r["Kernel_Name"]]
        copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"]]
        if not march or not copies:
            raise SystemExit(f"{f}: needs step-kernel dispatches and the calibration copy "
                             "(run the profile case with --copy-mib > 0)")
        big = max(int(r["Grid_Size"]) for r in copies)
        cal = [float(r["Counter_Value"]) for r in copies if int(r["Grid_Size"]) == big]
        per.setdefault(case, {}).setdefault(cfg, {})[ctr] = dict(
            kib=sum(march) / len(march), scale=copy_mib * 1024.0 / (sum(cal) / len(cal)),
            n=len(march))
    out = {"kernel_sha256": h.hexdigest(), "kernel_sources": KERNEL_SOURCES,
           "calibration": f"each counter scaled by its KiB per dispatch of a {copy_mib} MiB "
                          "device copy (that many KiB read and written)",
           "per_launch_bytes": {}, "detail": {}}
    for case, cfgs in sorted(per.items()):
        alg = alg_bytes_per_node(case.endswith("fp32")) * PROFILE_NODES[case.split("_")[0]]
        for cfg, c in sorted(cfgs.items()):
            rd = c["FETCH_SIZE"]["kib"] * c["FETCH_SIZE"]["scale"] * 1024
            wr = c["WRITE_SIZE"]["kib"] * c["WRITE_SIZE"]["scale"] * 1024
            out["per_launch_bytes"].setdefault(case, {})[cfg] = int(round(rd + wr))
            out["detail"].setdefault(case, {})[cfg] = {
                "read_bytes": int(round(rd)), "write_bytes": int(round(wr)),
                "algorithmic_bytes": alg, "ratio": round((rd + wr) / alg, 4),
                "fetch_kib_raw": round(c["FETCH_SIZE"]["kib"], 1),
                "write_kib_raw": round(c["WRITE_SIZE"]["kib"], 1),
                "fetch_scale": round(c["FETCH_SIZE"]["scale"], 4),
                "write_scale": round(c["WRITE_SIZE"]["scale"], 4),
                "dispatches": c["FETCH_SIZE"]["n"]}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    return out


def copy_bandwidth(mib=2048, reps=5):
    """Measured device-to-device copy bandwidth (GB/s, bytes read + written),
    the practical ceiling next to the 8 TB/s data-sheet figure."""
    import torch

    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    bw = reps * 2 * n * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return round(bw, 1)


def with_copy_fraction(rl, copy_gbs):
    """Roofline record plus the fraction of the measured copy bandwidth."""
    if copy_gbs:
        rl["copy_GBps"] = copy_gbs
        rl["frac_of_copy"] = round(rl["achieved"] / copy_gbs, 4)
    return rl


def host_cpu():
    """Host CPU model and the logical CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count() or 0
    return model, os.cpu_count() or 0, avail


def cpu_baseline(case, budget_s=15.0):
    """The float64 oracle on the host: the calling thread pinned to one core
    (os.sched_setaffinity on this thread; the process has already started
    the GPU runtime, so it is not re-launched under taskset) and BLAS thread
    pools limited to one thread, a bounded number of steps."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:
        threadpool_limits = None
    from oracle.step import Params, Sim

    nx, ny, kw, bnd, rho, T = case
    keys = ["a", "sigma", "kappa", "rho_l", "rho_v", "thermal", "cv", "lambda_l", "lambda_v",
            "t_side_val", "s_rho", "s_e", "s_zeta", "s_j", "s_q"]
    p = Params(nx=nx, ny=ny, t_side_dirichlet=True, t_bottom_kind=bnd["t_bottom_kind"],
               t_bottom_val=bnd["t_bottom_val"], t_top_kind=bnd["t_top_kind"],
               t_top_val=bnd["t_top_val"], **{k: kw[k] for k in keys})
    import contextlib

    model, ncpu, avail = host_cpu()
    prev = None
    core = None
    try:
        prev = os.sched_getaffinity(0)
        core = min(prev)
        os.sched_setaffinity(0, {core})
    except (AttributeError, OSError):
        prev = None
    lim = threadpool_limits(limits=1) if threadpool_limits else contextlib.nullcontext()
    try:
        with lim:
            s = Sim(p)
            s.init_fields(rho, None, None, T)
            t0 = time.perf_counter()
            s.step(2)
            per = (time.perf_counter() - t0) / 2
            n = max(3, int(budget_s / per))
            t0 = time.perf_counter()
            s.step(n)
            dt = time.perf_counter() - t0
    finally:
        if prev is not None:
            os.sched_setaffinity(0, prev)
    pinned = f"pinned to logical CPU {core}" if core is not None else "not pinned"
    return {"value": round(nx * ny * n / dt / 1e6, 4), "unit": "MLUPS", "cores": 1,
            "kind": "oracle",
            "sample": f"{nx}x{ny} droplet vaporisation (seed 0), {n} float64 oracle steps after 2 "
                      f"untimed, {dt:.1f} s on one host core ({pinned}, BLAS threads limited to 1)",
            "host_cpu_model": model, "host_nproc": ncpu, "host_cpus_available": avail}


def ladder_case(k, seed, precision, steps0):
    """Mesh k of the pool-boiling refinement ladder (128x256 base, dx = 2^-k)
    with its seeded initial fields: liquid below 1400/2048 of the height,
    tanh interface and nucleation half-disk scaled with the mesh."""
    import workloads as wl
    from paper_2201_04560_amd.ladder import pool_level

    L = pool_level(k, steps0=steps0, precision=precision)
    lv, nx, ny = L["level"], L["nx"], L["ny"]
    rho, T = wl.pool(nx, ny, ny * 1400.0 / 2048.0, 2.3 * 2 ** k, lv["rho_l"], lv["rho_v"], lv["T"],
                     seed_radius=6.0 * 2 ** k, seed=100 * k + seed)
    return L, rho, T


def ladder_bench(steps0, levels=(0, 1, 2, 3), seeds=(0, 1, 2, 3), tile_cache=None):
    """16 grids (4 meshes x 4 seeds), mesh k advanced by steps0 4^k steps
    (the same physical time), four ways: float32 shifted storage in one
    batched, graph-replayed launch per step (strip height and waves per
    strip tuned per mesh on its seeds' batched launch); float32 one grid at a
    time (the batching gain at equal precision); the plain float64 step one
    grid at a time; and, on the finest mesh, a float64 batch started from the
    float64 initial state perturbed by one ulp, whose drift from the float64
    run is the trajectory's own sensitivity (nucleation) against which the
    float32 deviation is read."""
    import torch

    from paper_2201_04560_amd import Batch, Lattice
    from paper_2201_04560_amd.ladder import TileCache

    cache = TileCache(tile_cache)
    dev = device_key()
    specs = [(k, sd) for k in levels for sd in seeds]

    def build(precision, only=None, perturb=False):
        lats, steps = [], []
        for k, sd in specs:
            if only is not None and k != only:
                continue
            L, rho, T = ladder_case(k, sd, precision, steps0)
            if perturb:
                rho = np.nextafter(rho, np.inf)
            lat = Lattice(L["params"])
            lat.set_boundary(**L["boundary"])
            lat.init_fields(rho, None, None, T)
            lats.append(lat)
            steps.append(L["steps"])
        return lats, steps

    def make(k):
        return build(1, only=k)[0]

    def timed_batch(lats, steps):
        b = Batch(lats)
        b.run([2] * len(lats))  # warm-up: graph instantiation path and caches
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        rec = b.last_time()
        b.close()
        return wall, rec

    def timed_plain(lats, steps):
        for lat in lats:
            lat.step(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for lat, n in zip(lats, steps):
            lat.step(n)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    tiles = {k: cache.tune_batch(lambda k=k: make(k), device=dev, waves=(1, 2), with_waves=True)
             for k in levels}
    lats32, steps = build(1)
    for (k, sd), lat in zip(specs, lats32):
        lat.tile_y, lat.strip_waves = tiles[k]
    log(f"bench: ladder tiles {tiles}, steps {sorted(set(steps))}")
    t32, (ms32, launches, graphs) = timed_batch(lats32, steps)
    lats32p, _ = build(1)
    t32p = timed_plain(lats32p, steps)
    lats64, _ = build(0)
    t64 = timed_plain(lats64, steps)
    lu = sum(l.nx * l.ny * n for l, n in zip(lats32, steps))
    per_level = {}
    for (k, sd), a, c, ap in zip(specs, lats32, lats64, lats32p):
        r32, _, _, T32 = a.fields()
        r64, _, _, T64 = c.fields()
        e = per_level.setdefault(k, {"grid": f"{a.nx}x{a.ny}", "steps": steps[specs.index((k, sd))],
                                     "tile_y": tiles[k][0], "strip_waves": tiles[k][1],
                                     "rho_max_rel": 0.0, "T_max_rel": 0.0, "kappa": None,
                                     "fp32_batched_vs_per_grid_rho_max_rel": 0.0})
        e["rho_max_rel"] = max(e["rho_max_rel"], rel_err(r32, r64))
        e["T_max_rel"] = max(e["T_max_rel"], rel_err(T32, T64))
        # same arithmetic; with gravity the order of the mean-density partial
        # sums follows the strip height, which differs between the two runs
        e["fp32_batched_vs_per_grid_rho_max_rel"] = max(e["fp32_batched_vs_per_grid_rho_max_rel"],
                                                        rel_err(r32, ap.fields()[0]))
    for k in per_level:
        from paper_2201_04560_amd.ladder import pool_level

        lv = pool_level(k, steps0=steps0)["level"]
        per_level[k].update(a=lv["a"], sigma=round(lv["sigma"], 6), kappa=round(lv["kappa"], 6),
                            gy=lv["gy"])
    for lat in lats32 + lats32p:
        lat.close()
    torch.cuda.empty_cache()
    # float64 trajectory sensitivity on the finest mesh (batched float64 is
    # the same arithmetic as the plain float64 step)
    kf = max(levels)
    latsp, stp = build(0, only=kf, perturb=True)
    timed_batch(latsp, stp)
    ref = [c for (k, sd), c in zip(specs, lats64) if k == kf]
    chaos = {"mesh": per_level[kf]["grid"], "steps": stp[0], "rho_max_rel": 0.0, "T_max_rel": 0.0,
             "perturbation": "initial density moved up by one ulp at every node"}
    for a, c in zip(latsp, ref):
        ra, _, _, Ta = a.fields()
        rc, _, _, Tc = c.fields()
        chaos["rho_max_rel"] = max(chaos["rho_max_rel"], rel_err(ra, rc))
        chaos["T_max_rel"] = max(chaos["T_max_rel"], rel_err(Ta, Tc))
    for lat in latsp + lats64:
        lat.close()
    torch.cuda.empty_cache()
    return {"grids": len(specs), "steps0": steps0, "lattice_updates": lu,
            "fp32_batched": {"wall_s": round(t32, 4), "device_ms": round(ms32, 3),
                             "MLUPS": round(lu / t32 / 1e6, 1), "step_launches": launches,
                             "graph_launches": graphs},
            "fp32_per_grid": {"wall_s": round(t32p, 4), "MLUPS": round(lu / t32p / 1e6, 1),
                              "kernel_launches": sum(steps)},
            "fp64_plain_per_grid": {"wall_s": round(t64, 4), "MLUPS": round(lu / t64 / 1e6, 1),
                                    "kernel_launches": sum(steps)},
            "speedup": round(t64 / t32, 3),
            "speedup_batching_fp32": round(t32p / t32, 3),
            "speedup_precision_per_grid": round(t64 / t32p, 3),
            "levels": {str(k): v for k, v in per_level.items()},
            "fp64_trajectory_sensitivity": chaos,
            "accuracy": "max relative rho / T difference, float32 batched vs float64 plain, "
                        "per mesh over its 4 seeds, after the full schedule"}


def adjoint_case(n=256, seed=0):
    """Droplet vaporisation on n x n (radius 60 n / 512, as the 512^2
    workload) whose bottom ring row is the heater profile (0.95 T_c)."""
    import paper_2201_04560_amd as pp
    import workloads as wl

    a = 2.0 / 49.0
    Tc = pp.pr_critical_temperature(a)
    Tsat, Tout = 0.86 * Tc, 0.95 * Tc
    rv, rl, _ = pp.pr_maxwell(a, Tsat)
    rho, T = wl.droplet(n, n, 60.0 * n / 512, 4.6 / 5.0, rl, rv, Tsat, Tout, seed=seed)
    kw = dict(a=a, sigma=0.1, kappa=0.1, rho_l=rl, rho_v=rv, thermal=1, cv=6.0, lambda_l=2.0 / 3.0,
              lambda_v=2.0 / 3.0, t_side_dirichlet=1, t_side_val=Tout, rho_ref=rv)
    kw.update(wl.DROPLET_RATES)
    bnd = dict(t_bottom_kind=np.full(n, 1, np.int32), t_bottom_val=np.full(n, Tout),
               t_top_kind=np.full(n, 1, np.int32), t_top_val=np.full(n, Tout))
    return n, kw, bnd, rho, T


def adjoint_bench(nsteps=500, ckpt=50, n=256, fd_entries=8, h=1e-4):
    """Heater-profile gradient of the evaporated mass: cost of the adjoint
    against the plain forward, check against central differences."""
    import torch

    from paper_2201_04560_amd import HeaterProblem, make_params

    n, kw, bnd, rho, T = adjoint_case(n)
    out = {"workload": f"droplet vaporisation {n}x{n}, {nsteps} steps, checkpoint every {ckpt}, "
                       f"gradient of the evaporated liquid mass w.r.t. the {n}-entry bottom heater "
                       "profile"}
    grads = {}
    for name, prec in (("fp32", 1), ("fp64", 0)):
        pr = HeaterProblem(make_params(n, n, precision=prec, **kw), bnd, rho, T, nsteps, ckpt)
        tb = bnd["t_bottom_val"]
        pr.run(tb)  # warm-up (module load, first-touch)
        pr.adjoint.backward()
        torch.cuda.synchronize()
        # each timing the best of three runs (single runs of the 500-step
        # forward varied by 5 %)
        t_plain = 1e300
        for _ in range(3):
            t0 = time.perf_counter()
            pr.lattice.set_boundary(**bnd)
            pr.lattice.init_fields(rho, None, None, T)
            pr.lattice.step(nsteps)
            pr.lattice.sync()
            t_plain = min(t_plain, time.perf_counter() - t0)
        f_ms = b_ms = 1e300
        for _ in range(3):
            J = pr.run(tb)
            g = pr.adjoint.backward()
            f1, b1 = pr.adjoint.timing()
            f_ms, b_ms = min(f_ms, f1), min(b_ms, b1)
        grads[name] = g
        out[name] = {"J": J, "plain_forward_ms": round(t_plain * 1e3, 3),
                     "checkpointed_forward_ms": round(f_ms, 3), "backward_ms": round(b_ms, 3),
                     "backward_over_forward": round(b_ms / (t_plain * 1e3), 2),
                     "gradient_over_forward": round((f_ms + b_ms) / (t_plain * 1e3), 2),
                     "speedup_vs_central_fd": round(2 * n * t_plain * 1e3 / (f_ms + b_ms), 1)}
        if name == "fp64" and fd_entries > 0:
            ent = np.linspace(16, n - 17, fd_entries).astype(int)
            errs = []
            for x in ent:
                tp, tm = tb.copy(), tb.copy()
                tp[x] += h
                tm[x] -= h
                fd = (pr.run(tp) - pr.run(tm)) / (2 * h)
                errs.append(abs(fd - g[x]) / np.abs(g).max())
            out["fd_check"] = {"entries": ent.tolist(), "h": h, "forward": "float64 library step",
                               "max_abs_diff_over_max_grad": float(max(errs))}
        pr.adjoint.close()
        pr.lattice.close()
        torch.cuda.empty_cache()
    out["fp32_vs_fp64_grad_rel"] = float(np.abs(grads["fp32"] - grads["fp64"]).max() /
                                         np.abs(grads["fp64"]).max())
    return out


def droplet_stats(rho, rho_l, rho_v):
    """Equivalent radius of the liquid area, liquid density at the centre and
    vapour density in the far corners."""
    ny, nx = rho.shape
    mid = 0.5 * (rho_l + rho_v)
    R = float(np.sqrt((rho > mid).sum() / np.pi))
    y, x = np.mgrid[0:ny, 0:nx]
    r = np.hypot(x - nx / 2 + 0.5, y - ny / 2 + 0.5)
    return {"R_eq": R, "rho_centre": float(rho[r < 0.5 * R].mean()),
            "rho_far": float(rho[r > 0.45 * min(nx, ny) + R / 2].mean())}


def pool_heat_flux(precision, steps, every, tune):
    """Pool boiling 1024 wide x 2048 tall (liquid below 1400, heater 128 wide
    at 0.95 T_c, the rest of the bottom adiabatic; mesh 3 of the refinement
    ladder over a 128 x 256 base with g = -3e-5 there): the wall heat flux of
    Eq. pool-heat-flux and the heater's own mean flux every `every` steps."""
    import torch

    from paper_2201_04560_amd import Lattice, make_params

    nx, ny, kw, bnd, rho, T = pool_case(1024, 2048, level=3)
    lat = Lattice(make_params(nx, ny, precision=precision, **kw))
    lat.set_boundary(**bnd)
    lat.init_fields(rho, None, None, T)
    if tune is not None:
        tune.tune(lat, device=device_key())
    q, qh = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps // every):
        lat.step(every)
        n = lat.norms()
        q.append(n["q_bottom"])
        qh.append(n["q_heater"])
    dt = time.perf_counter() - t0
    r = lat.fields()[0]
    lat.close()
    torch.cuda.empty_cache()
    # Nusselt number of the heater (reading C18): the heater's mean flux made
    # dimensionless with its length W_h (the held bottom nodes) and the
    # liquid conduction scale lambda_l (T_h - T_sat); positive into the fluid
    tb = np.broadcast_to(np.asarray(bnd["t_bottom_val"], dtype=np.float64), (nx,))
    t_h, t_sat = float(tb.max()), float(np.min(bnd["t_top_val"]))
    w_h = int(n["n_heater"])
    nu_scale = -w_h / (kw["lambda_l"] * (t_h - t_sat))
    return np.array(q), np.array(qh), r, nx * ny * steps / dt / 1e6, dict(kw, nu_scale=nu_scale, w_h=w_h)


def accuracy_bench(args, tune):
    """Float32 shifted storage against the float64 step on the 1024 x 2048
    pool: wall and heater heat-flux histories and the heater Nusselt number."""
    steps, every = args.pool_steps, max(args.pool_steps // 10, 1)
    q32, h32, p32, m32, _ = pool_heat_flux(1, steps, every, tune)
    q64, h64, p64, m64, k64 = pool_heat_flux(0, steps, every, tune)
    nu32, nu64 = h32 * k64["nu_scale"], h64 * k64["nu_scale"]
    return {"pool1024x2048": {
        "steps": steps, "q_every": every, "heater_nodes": k64["w_h"],
        "q_wall_fp32": q32.tolist(), "q_wall_fp64": q64.tolist(),
        "q_wall_max_rel_diff": float(np.abs(q32 - q64).max() / np.abs(q64).max()),
        "q_heater_fp32": h32.tolist(), "q_heater_fp64": h64.tolist(),
        "nusselt_heater_fp32": np.round(nu32, 6).tolist(), "nusselt_heater_fp64": np.round(nu64, 6).tolist(),
        "nusselt_max_rel_diff": float(np.abs(nu32 - nu64).max() / np.abs(nu64).max()),
        "rho_max_rel": rel_err(p32, p64),
        "MLUPS_fp32_with_norms": round(m32, 1), "MLUPS_fp64_with_norms": round(m64, 1)}}


def optional_section(fn, *a, **kw):
    """A report section beside the metric: a library error (e.g. a state
    leaving the EOS domain) is recorded in the JSON instead of ending the run."""
    from paper_2201_04560_amd import LbmError

    try:
        return fn(*a, **kw)
    except LbmError as e:
        log(f"bench: section {fn.__name__} failed: {e}")
        return {"error": str(e)}


def rel_err(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--accuracy-steps", type=int, default=20000,
                    help="length of the float32-vs-float64 comparison on the four seeds (the "
                         "configuration's 20000 steps)")
    ap.add_argument("--sizing-steps", type=int, default=200)
    ap.add_argument("--no-sizing", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["fp32", "fp64", "both"], default="both")
    ap.add_argument("--profile-case", choices=["vaporisation512", "vaporisation512x4", "pool4096",
                                               "adjoint256"], default=None,
                    help="profiling run: only this case (precision from --only), --steps steps, "
                         "plus a device copy of --copy-mib MiB (counter calibration); no JSON. "
                         "vaporisation512x4: the four seeds in the batched launch timed by the "
                         "metric; adjoint256: the 256^2 x 500-step heater gradient in both "
                         "precisions")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--tile-y", type=int, default=0)
    ap.add_argument("--launch", choices=["auto", "graph", "direct"], default="auto",
                    help="batched step: graph-replayed or direct launches (auto: the faster over "
                         "200 steps)")
    ap.add_argument("--strip-waves", type=int, default=0,
                    help="waves per strip with --tile-y (0: the library's choice)")
    ap.add_argument("--traffic-from", default=None, metavar="DIR",
                    help="no GPU work: write profiles/traffic.json from the rocprofv3 --pmc "
                         "directories DIR/pmc_<case>_<prec>_<TY>x<W>_<FETCH_SIZE|WRITE_SIZE> "
                         "of --profile-case runs (calibration copy of --copy-mib MiB)")
    ap.add_argument("--ladder-steps0", type=int, default=800,
                    help="steps of the coarsest ladder mesh (mesh k runs steps0 * 4^k)")
    ap.add_argument("--no-ladder", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--refinement-study", action="store_true",
                    help="also run the Sec. 4.1 droplet refinement (meshes 128..432, float64, "
                         "about 100 s of GPU time)")
    ap.add_argument("--pool-refinement-study", action="store_true",
                    help="also run the Sec. 4.3 pool refinement (meshes 160..540, 40000 base "
                         "steps, rho_wh 0.38, T_h 1.2 T_c, float64, about 40 s of GPU time)")
    ap.add_argument("--contact-angle-study", action="store_true",
                    help="also run the Sec. 4.3 contact-angle tests: the G_w search of the "
                         "modified-psi model (meshes 160..540) and the psi-based refinement "
                         "(meshes 160..810), float64, about 130 s of GPU time")
    ap.add_argument("--stefan-study", action="store_true",
                    help="also run the Sec. 4.2 1-D boiling refinement (columns of 160..2560 "
                         "nodes, both parameter sets, 40000 base steps, float64, about 4 min "
                         "of GPU time)")
    ap.add_argument("--pool-steps", type=int, default=50000,
                    help="steps of the 1024 x 2048 pool in the float32 accuracy check (the "
                         "configuration's 50,000 by default, about 10 s of GPU time)")
    ap.add_argument("--tile-cache", default=None, help="JSON cache of autotuned strip heights")
    ap.add_argument("--no-autotune", action="store_true",
                    help="library default strip heights instead of the autotuner")
    args = ap.parse_args()
    if args.traffic_from:
        for case, cfgs in write_traffic(args.traffic_from, args.copy_mib)["detail"].items():
            for cfg, d in cfgs.items():
                log(f"traffic: {case} {cfg} {(d['read_bytes'] + d['write_bytes']) / 1e6:.2f} MB "
                    f"per launch, {d['ratio']}x algorithmic")
        return
    if args.gpus != 1:
        print(f"bench.py: the step runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU slab decomposition is designed but not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    from paper_2201_04560_amd import LBM_FP32_SHIFTED, LBM_FP64
    from paper_2201_04560_amd.ladder import TileCache

    tune = None if (args.tile_y or args.no_autotune) else TileCache(args.tile_cache)

    if args.profile_case == "adjoint256":
        r = adjoint_bench(fd_entries=0)
        for name in ("fp32", "fp64"):
            log(f"profile: adjoint256 {name} backward {r[name]['backward_ms']} ms, checkpointed forward "
                f"{r[name]['checkpointed_forward_ms']} ms, plain forward {r[name]['plain_forward_ms']} ms")
        return
    if args.profile_case:
        for name, prec in (("fp32", LBM_FP32_SHIFTED), ("fp64", LBM_FP64)):
            if args.only not in (name, "both"):
                continue
            if args.profile_case == "vaporisation512x4":
                ty, w = (args.tile_y, args.strip_waves) if args.tile_y else tune_vap_batch(tune, prec)
                ug = (args.launch == "graph") if args.launch != "auto" else pick_launch_mode(prec, ty, w)
                r = run_vap_batch(prec, args.warmup, args.steps, ty, w, want_fields=False, use_graph=ug)
            else:
                pcase = vaporisation_case() if args.profile_case == "vaporisation512" else pool_case()
                r = run_lattice(pcase, prec, args.warmup, args.steps, want_fields=False,
                                tile_y=args.tile_y, tune=tune, strip_waves=args.strip_waves)
            log(f"profile: {args.profile_case} {name} kernel {r['kernel_ms_avg'] * 1e3:.2f} us "
                f"avg over {r['launches']} launches, tile_y {r['tile_y']}, waves {r['strip_waves']}")
        if args.copy_mib > 0:
            n = args.copy_mib * (1 << 20) // 4
            src = torch.ones(n, dtype=torch.float32, device="cuda")
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            log(f"profile: copy kernel {args.copy_mib} MiB read + {args.copy_mib} MiB written, 3 times")
        return

    case = vaporisation_case()
    nx, ny = case[0], case[1]
    nodes = len(SEEDS) * nx * ny
    res = {}
    tiles = {}
    for name, prec in (("fp32", LBM_FP32_SHIFTED), ("fp64", LBM_FP64)):
        if args.only not in (name, "both"):
            continue
        if name == "fp32":
            ty, w = (args.tile_y, args.strip_waves) if args.tile_y else tune_vap_batch(tune, prec)
            tiles[name] = (ty, w)
            ug = (args.launch == "graph") if args.launch != "auto" else pick_launch_mode(prec, ty, w)
            log(f"bench: fp32 4 x {nx}x{ny} vaporisation batch, tile_y {ty}, waves {w}, "
                f"{'graph-replayed' if ug else 'direct'} launches, warmup {args.warmup}, steps {args.steps}")
            res[name] = run_vap_batch(prec, args.warmup, args.steps, ty, w, use_graph=ug)
        else:
            log(f"bench: fp64 plain step, 4 x {nx}x{ny} one lattice after another, warmup "
                f"{args.warmup}, steps {args.steps}")
            res[name] = run_vap_plain(prec, args.warmup, args.steps, tile_y=args.tile_y,
                                      waves=args.strip_waves)
        r = res[name]
        log(f"bench: {name} {args.steps * nodes / r['wall_s'] / 1e6:.0f} MLUPS, kernel "
            f"{r['kernel_ms_avg'] * 1e3:.2f} us avg over {r['launches']} launches, "
            f"tile_y {r['tile_y']}, waves {r['strip_waves']}")

    main_name = "fp32" if "fp32" in res else "fp64"
    m = res[main_name]
    value = args.steps * nodes / m["wall_s"] / 1e6
    per_launch_nodes = nodes if main_name == "fp32" else nx * ny
    traffic_key = "vaporisation512x4_fp32" if main_name == "fp32" else "vaporisation512_fp64"
    out = {
        "metric": "MLUPS + % HBM roofline, FP32 fused vs FP64 plain step, at stated rho/T error",
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["wall_s"] * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if main_name == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "droplet vaporisation 512x512, seeds 0-3 (+-0.5 interface jitter), "
                               "PR a=2/49 b=2/21, r=60 at 0.86 Tc in vapour held at 0.95 Tc, "
                               "sigma=kappa=0.1, cv=6, lambda=2/3, no gravity; a step advances the "
                               "four seeds by one time step",
                   "nx": nx, "ny": ny, "lattices": len(SEEDS),
                   "storage": "f32 shifted populations (f - w rho_v) + f32 T; f64 EOS/psi, wall "
                              "closure and reductions" if main_name == "fp32" else "f64",
                   "launch": ("one batched multi-lattice launch per step, " +
                              ("graph-replayed" if m.get("use_graph") else "launched directly") +
                              (" (the faster of the two over 200 steps)" if args.launch == "auto" else ""))
                             if main_name == "fp32" else "one launch per lattice and step",
                   "steps_total": args.warmup + args.steps,
                   "tile_y": m["tile_y"], "strip_waves": m["strip_waves"]},
        "roofline": roofline(main_name == "fp32", per_launch_nodes, m["kernel_ms_avg"],
                             measured_traffic(traffic_key, m["tile_y"], m["strip_waves"])),
    }
    copy_gbs = copy_bandwidth()
    log(f"bench: device copy {copy_gbs} GB/s")
    with_copy_fraction(out["roofline"], copy_gbs)
    if main_name == "fp32":
        out["batch_bitwise_vs_solo"] = batch_bitwise_vs_solo(m, LBM_FP32_SHIFTED,
                                                             args.warmup + args.steps)
    if "fp32" in res and "fp64" in res:
        f32, f64 = res["fp32"], res["fp64"]
        out["fp64_plain"] = {
            "value": round(args.steps * nodes / f64["wall_s"] / 1e6, 1), "unit": "MLUPS",
            "tile_y": f64["tile_y"], "strip_waves": f64["strip_waves"],
            "ms_per_step": round(f64["wall_s"] * 1e3 / args.steps, 5),
            "launch": "one launch per lattice and step, the four lattices one after another",
            "roofline": with_copy_fraction(
                roofline(False, nx * ny, f64["kernel_ms_avg"],
                         measured_traffic("vaporisation512_fp64", f64["tile_y"], f64["strip_waves"])),
                copy_gbs),
        }
        out["speedup_fp32_vs_fp64"] = round(f64["wall_s"] / f32["wall_s"], 3)
        if not args.no_accuracy:
            log(f"bench: float32 vs float64 accuracy, 4 seeds x {args.accuracy_steps} steps")
            out["fp32_error_vs_fp64"] = optional_section(accuracy_20k, args.accuracy_steps, tune)
    # the single lattice (seed 0) as in the plain per-lattice runs, for reference
    single = {}
    for name, prec in (("fp32", LBM_FP32_SHIFTED), ("fp64", LBM_FP64)):
        if args.only not in (name, "both"):
            continue
        r = run_lattice(case, prec, args.warmup, args.steps, want_fields=False, tile_y=args.tile_y,
                        tune=tune, strip_waves=args.strip_waves)
        single[name] = {"value": round(args.steps * nx * ny / r["wall_s"] / 1e6, 1), "unit": "MLUPS",
                        "tile_y": r["tile_y"], "strip_waves": r["strip_waves"],
                        "roofline": with_copy_fraction(
                            roofline(name == "fp32", nx * ny, r["kernel_ms_avg"],
                                     measured_traffic(f"vaporisation512_{name}", r["tile_y"],
                                                      r["strip_waves"])), copy_gbs)}
    out["single_lattice_seed0"] = single
    if "fp32" in res and "fp64" in res and not args.no_accuracy:
        log("bench: pool heat flux and heater Nusselt number, float32 vs float64")
        out["fp32_accuracy"] = optional_section(accuracy_bench, args, tune)
    if not args.no_sizing:
        pc = pool_case()
        sz = {}
        for name, prec in (("fp32", LBM_FP32_SHIFTED), ("fp64", LBM_FP64)):
            if args.only not in (name, "both"):
                continue
            log(f"bench: sizing {name} {pc[0]}x{pc[1]} pool, {args.sizing_steps} steps")
            r = run_lattice(pc, prec, 20, args.sizing_steps, want_fields=False, tune=tune)
            n2 = pc[0] * pc[1]
            sz[name] = {"value": round(args.sizing_steps * n2 / r["wall_s"] / 1e6, 1),
                        "unit": "MLUPS",
                        "tile_y": r["tile_y"], "strip_waves": r["strip_waves"],
                        "roofline": with_copy_fraction(
                            roofline(name == "fp32", n2, r["kernel_ms_avg"],
                                     measured_traffic(f"pool4096_{name}", r["tile_y"],
                                                      r["strip_waves"])),
                            copy_gbs)}
        out["hbm_sized_run"] = {"workload": "pool boiling 4096x4096 (walls, heater, gravity, "
                                            "energy equation; mesh 5 of the refinement procedure "
                                            "over a 128x128 base), 1.3 GB f32 / 2.7 GB f64 state",
                                **sz}
    if not args.no_ladder:
        log(f"bench: refinement ladder, steps0 {args.ladder_steps0}")
        out["ladder"] = optional_section(ladder_bench, args.ladder_steps0, tile_cache=args.tile_cache)
    if not args.no_adjoint:
        log("bench: adjoint 256x256, 500 steps")
        out["adjoint"] = optional_section(adjoint_bench)
    if args.refinement_study:
        from paper_2201_04560_amd.ladder import droplet_refinement

        log("bench: droplet refinement study 128/192/288/432")
        t0 = time.perf_counter()
        rs = droplet_refinement((128, 192, 288, 432), L0=128, samples=200, sample0=2048,
                                progress=lambda k, n: k % 20 == 0 and log(f"bench:   sample {k}/{n}"))
        R = rs.pop("R")
        rs["R_every_20_samples"] = np.round(R[:, ::20], 4).tolist()
        rs["wall_s"] = round(time.perf_counter() - t0, 1)
        out["refinement_study"] = rs
    if args.pool_refinement_study:
        from paper_2201_04560_amd.ladder import pool_refinement

        log("bench: pool refinement study 160/240/360/540")
        t0 = time.perf_counter()
        ps = pool_refinement(rho_wh=0.38, Th_r=1.2,
                             progress=lambda k, n, what: k % 20 == 0 and log(f"bench:   {what} sample {k}/{n}"))
        for k in ("d_rho", "d_T"):
            ps[k] = np.round(np.asarray(ps[k])[:, ::8], 5).tolist()
        ps["wall_s"] = round(time.perf_counter() - t0, 1)
        out["pool_refinement_study"] = ps
    if args.contact_angle_study:
        from paper_2201_04560_amd.ladder import contact_angle_refinement, gw_search

        log("bench: contact-angle study (G_w search 160..540, psi-based refinement 160..810)")
        t0 = time.perf_counter()
        cs = {"gw_search": gw_search(progress=lambda k, n: log(f"bench:   G_w mesh {k}/{n}")),
              "psi_based": contact_angle_refinement(
                  progress=lambda k, n: log(f"bench:   psi-based check {k}/{n}"))}
        cs["wall_s"] = round(time.perf_counter() - t0, 1)
        out["contact_angle_study"] = cs
    if args.stefan_study:
        from paper_2201_04560_amd.ladder import stefan_refinement

        log("bench: Stefan refinement study 160..2560")
        t0 = time.perf_counter()
        ss = stefan_refinement(progress=lambda k, n: log(f"bench:   sample {k}/{n}"))
        for d in ss["sets"].values():
            d["s"] = np.round(np.asarray(d["s"])[:, ::10], 3).tolist()
            d["reference"] = np.round(np.asarray(d["reference"])[::10], 3).tolist()
        ss["t"] = ss["t"][::10]
        ss["wall_s"] = round(time.perf_counter() - t0, 1)
        out["stefan_study"] = ss
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
