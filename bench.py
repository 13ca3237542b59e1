#!/usr/bin/env python3
"""Throughput of the coupled D2Q9 + D2Q5 lattice Boltzmann step on one MI355X.

One benchmark step is one coupled time step (collide + stream of both
lattices, boundary links, valve schedule, FP64 boundary-flux accumulation,
and every `--monitor-every` steps the FP64 mass / compound / velocity /
Peclet reduction) over the whole synthetic lattice, with the state resident
in HBM. The default workload is the largest single-GPU configuration: the
8192 x 4096 gradient generator with FP16-shifted population storage, FP32
collision arithmetic and FP64 reductions (channel Peclet 500, valves
toggling every 2000 steps).

The timed region is exactly --steps steps after --warmup untimed ones (and
at most 3 more that start the timed steps on the two-step pass's parity),
bracketed by HIP events on the lattice's stream. Inside it, the library
records an event pair around every launch of the dominant kernel, whose
mean duration gives the roofline figures.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "coupled NSE+CDE MLUPS and % HBM roofline on 1 MI355X; FP32/FP16 vs FP64 error"
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2}
CSRC = os.path.join(ROOT, "paper_1307_4703_amd", "csrc")
# sources of the dominant kernel (the two-step pass); the counters in
# profiles/traffic.json hold for the hash of these files
KERNEL_SRC = [os.path.join(CSRC, f)
              for f in ("gg_device.h", "gg_node.h", "gg_fused.hip", "gg_cde.hip")]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bytes_per_update(storage):
    # in-place AA: every one of the 9 + 5 populations read once and written
    # once per fluid-node update, plus the 1-byte link code
    return 14 * 2 * STORAGE_BYTES[storage] + 1


def workload(name):
    from paper_1307_4703_amd import workloads as W
    table = {
        "gg2048_f32": lambda: W.gradient_generator(storage="f32"),
        "gg2048_f16": lambda: W.gradient_generator(storage="f16"),
        "gg2048_f64": lambda: W.gradient_generator(storage="f64"),
        "gg8192_f16": lambda: W.gradient_generator(scale=4.0, storage="f16"),
        "gg8192_f16_pe2000": lambda: W.gradient_generator(scale=4.0, storage="f16", peclet=2000.0),
        "gg8192_f32": lambda: W.gradient_generator(scale=4.0, storage="f32"),
        "allfluid8192_f32": lambda: W.all_fluid_channel(storage="f32"),
        "allfluid8192_f16": lambda: W.all_fluid_channel(storage="f16"),
        "allfluid8192_f64": lambda: W.all_fluid_channel(storage="f64"),
        # one GPU's slab of the all-fluid 8192 x 4096 lattice split over 8
        # GPUs along y (its two y faces walls here, halo rows there)
        "shard8192x512_f32": lambda: W.all_fluid_channel(ny=512, storage="f32"),
        "straight_f64": lambda: W.straight_channel(),
    }
    if name not in table:
        raise SystemExit(f"unknown workload {name}; choose from {sorted(table)}")
    return table[name]()


# launch form per workload ((fuse, rows) of gg_set_two_step), as the
# autotuner picks it on this GPU; --tune re-runs the autotuner
FORMS = {"gg2048_f32": (5, 6), "gg2048_f16": (4, 6), "gg8192_f16": (3, 6),
         "gg8192_f16_pe2000": (3, 6), "gg8192_f32": (5, 6), "allfluid8192_f32": (5, 6),
         "allfluid8192_f16": (3, 6), "shard8192x512_f32": (5, 6),
         "allfluid8192_f64": (5, 6), "gg2048_f64": (5, 6), "straight_f64": (4, 6)}
# the adjoint leg's lattice (2048 x 1024 FP32): the one-kernel two-step
# form, whose taped recomputation passes are one kernel as well (the
# four-step pass has no taped form; its lattices recompute in the two
# kernels of fuse 3: the forward sweep gains, 0.138 against 0.164 s over
# 20000 steps on this GPU, the whole gradient loses, 0.588-0.592 against
# 0.569-0.580 s)
ADJOINT_FORM = (4, 6)


def kernel_hash():
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(wl_name):
    """HBM bytes per step launch from committed rocprofv3 counter runs, or
    None when they are missing or were taken on another kernel source
    (wl_name "cde:<workload>" for the compound-only step)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = data.get("workloads", {}).get(wl_name)
    if not ent or data.get("kernel_sha") != kernel_hash():
        return None
    return ent.get("bytes_per_launch")


def align_steps(t):
    """Untimed steps that bring step count t to a multiple of 4, where a run
    of two-step passes starts (each pass from an even step, pairs of passes
    ending in the first plane set)."""
    return (-t) % 4


def monitor_interval(steps, every):
    """Timed steps between FP64 monitor reductions: at most `every`, and a
    divisor of `steps` (between every / 2 and every) where there is one,
    so that the last reduction falls on the last timed step."""
    if steps <= 0:
        return 0
    if steps <= every:
        return steps
    for m in range(every, max(1, every // 2) - 1, -1):
        if steps % m == 0:
            return m
    return every


def time_lattice(name, steps, warmup, tile, chunk, form=None, monitor_every=1024,
                 graph_steps=None):
    """One workload: `warmup` untimed steps (plus at most 3 that align the
    step count to the pass's parity, and one graph chunk that captures the
    graph), then exactly `steps` timed steps of gg_step_profile — graph
    replays of `chunk` steps (at most the timed steps, rounded down to a
    multiple of 4) and plain launches for the rest — with the FP64 monitor
    reduction after every `monitor_every` of them (at least one, after the
    last step). The timed region is bracketed by HIP events on the lattice's
    stream (torch's current stream); gg_step_profile also records an event
    pair on that stream around every graph replay and every plain launch of
    the dominant kernel. Then `graph_steps` steps replayed from graphs of
    `chunk` steps, for comparison."""
    import torch
    from paper_1307_4703_amd import Lattice
    from paper_1307_4703_amd import tune as T
    wl = workload(name)
    lat = Lattice.from_workload(wl)
    chunk_t = 0
    try:
        nf = lat.info()["n_fluid"]
        if form == "tune":
            res = T.tune_lattice(lat, steps=64 if nf > 1e7 else 256, graph_chunk=chunk,
                                 use_cache=False)
            form = {"tile": res["tile"], "fuse": res["fuse"], "rows": res["rows"]}
        else:
            if form is None:
                fuse, rows = FORMS.get(name, (3, 6))
                form = {"fuse": fuse, "rows": rows}
            form = {"tile": list(tile), **form}
        lat.set_two_step(form["fuse"], form["rows"])
        form["layout"] = lat.layout
        # graph chunk of the timed region: whole replays inside it (a
        # multiple of 4 steps, of 8 with the four-step pass)
        q = 8 if form["fuse"] == 5 else 4
        chunk_t = min(chunk, steps // q * q) if chunk > 0 else 0
        lat.set_launch(form["tile"][0], form["tile"][1], chunk_t)
        log(f"{wl.name}: {wl.nx}x{wl.ny}, {nf} fluid nodes, storage {wl.storage}, "
            f"form {form}; warmup {warmup}")
        lat.step(warmup)
        extra_warm = align_steps(lat.info()["t"])
        lat.step(extra_warm)
        if chunk_t > 0:  # the graph is captured (and replayed once) here
            lat.step(chunk_t)
            extra_warm += chunk_t
        mon = monitor_interval(steps, monitor_every)
        lat.set_monitor(mon)
        lat.sync()
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        log(f"timed region: {steps} steps from t = {lat.info()['t']}, "
            f"monitor every {mon}")
        t0 = time.perf_counter()
        ev0.record(stream)
        prof = lat.step_profile(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ev_ms = ev0.elapsed_time(ev1)
        diag = lat.monitor(check_finite=False) if mon else lat.diagnostics(check_finite=False)
        lat.set_monitor(0)
        graph = None
        if graph_steps:
            k = max(4, graph_steps // 4 * 4)
            lat.set_launch(tile[0], tile[1], chunk)
            lat.step(align_steps(lat.info()["t"]))
            lat.step(max(chunk, 4))  # graphs captured
            lat.sync()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            lat.step(k)
            e1.record(stream)
            torch.cuda.synchronize()
            gms = e0.elapsed_time(e1)
            graph = {"steps": k, "graph_chunk": chunk, "ms_per_step": round(gms / k, 6),
                     "mlups": round(nf * k / (gms * 1e-3) / 1e6, 1)}
    finally:
        lat.close()
    return {"wl": wl, "nf": nf, "wall_s": wall, "event_ms": ev_ms, "form": form,
            "graph_chunk": chunk_t,
            "prof": prof, "diag": diag, "warmup_run": warmup + extra_warm, "steps": steps,
            "monitor_every": mon, "graph_replayed": graph}


def roofline(r, storage, traffic):
    """Dominant kernel: the interior-tile kernel of the two-step (or
    four-step) pass, or the single-step kernel when no pass ran. A launch of
    the pass advances each fluid node of its tiles by two (four) updates,
    so its algorithmic bytes are 2 (4) x (fluid nodes of its tiles) x the
    bytes per coupled update (14 populations read and written + the 1-byte
    link code); achieved = those bytes / the kernel's mean event-measured
    launch duration. Because the pass makes one trip through memory for
    two (four) updates, this figure can exceed the HBM peak; the counter bytes
    (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated) per launch, when
    present for the current kernel source, give the HBM fraction."""
    p = r["prof"]
    bpu = bytes_per_update(storage)
    passes = p["n_pass"] + p["graph_passes"]
    spp = p.get("steps_per_pass", 2)
    if passes > 0:
        # plain launches timed one by one; graph replays as a whole, divided
        # by the passes they hold (the boundary tiles' kernel runs beside)
        ms = (p["ms_pass"] + p["ms_graph"]) / passes
        units = spp * p["pass_fluid"]
        kind = ("four-step pass (interior tiles)" if spp == 4 else
                "two-step pass (interior tiles)" if p["fuse"] != 4 else "two-step pass")
        n_launch = passes
    else:
        n_launch = p["n_single"][0] + p["n_single"][1] + p["graph_singles"]
        ms = (p["ms_single"][0] + p["ms_single"][1] + p["ms_graph"]) / max(1, n_launch)
        units = r["nf"]
        kind = "single step"
    alg = units * bpu
    ach = alg / (ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": traffic,
           "kernel": kind, "launches_timed": n_launch,
           "launches_in_graph_replays": p["graph_passes"] if passes > 0 else p["graph_singles"],
           "kernel_ms": round(ms, 5),
           "updates_per_launch": units, "bytes_per_update": bpu,
           "algorithmic_bytes_per_launch": alg}
    if traffic:
        out["traffic_gbs"] = round(traffic / (ms * 1e-3) / 1e9, 1)
        out["traffic_frac"] = round(traffic / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
        out["traffic_per_algorithmic_single_trip"] = round(traffic / (alg / spp if passes else alg), 4)
    # whole-step throughput (all kernels of the step) priced at the bytes of
    # one coupled update
    out["step_rate_frac"] = round(r["nf"] * bpu * 1e-9 / (r["event_ms"] * 1e-3 / max(1, r.get("steps", 1)))
                                  / PEAK_HBM_GBS, 4) if r.get("steps") else None
    return out


def copy_bandwidth(nbytes=2 << 30, reps=20):
    import ctypes
    import torch
    from paper_1307_4703_amd import _abi as A
    a = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    ms = ctypes.c_double()
    stream = torch.cuda.current_stream().cuda_stream
    A.call("gg_stream_copy", ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(a.data_ptr()),
           nbytes, reps, ctypes.c_void_p(stream), ctypes.byref(ms))
    del a, b
    return 2.0 * nbytes / (ms.value * 1e-3) / 1e9


# Bytes per fluid node and time step of the adjoint with checkpoints (FP32
# storage): the forward pass (113), its recomputation segment by segment
# (113) with the tape of g and u written (7 x 4 = 28), and the adjoint step
# (FP64 lambda read and written, 2 x 5 x 8 = 80, and the tape read, 28).
ADJOINT_BYTES_F32 = 113 + 113 + 28 + 80 + 28
# one adjoint step: FP64 lambda read and written, the tape read, the link code
ADJOINT_STEP_BYTES_F32 = 80 + 28 + 1


def adjoint_bench(steps=20000, chunk=64):
    """The 2048 x 1024 FP32 gradient generator's chamber-misfit gradient
    (loss window, target ramp and source patch of chamber_misfit_setup)
    over `steps` steps with sqrt(N) checkpoints, against `steps` plain
    forward steps of the same lattice; wall-clock (gg_adjoint returns after
    the gradients are on the host)."""
    import torch
    from paper_1307_4703_amd import Lattice
    from paper_1307_4703_amd import workloads as W
    wl = workload("gg2048_f32")
    weight, target, r_box = W.chamber_misfit_setup(wl)
    lat = Lattice.from_workload(wl)
    try:
        lat.set_launch(64, 4, chunk)
        lat.set_two_step(*ADJOINT_FORM)
        lat.adjoint(64, weight, target, r_box=r_box)  # kernels loaded, graphs captured
        lat.init(**(wl.init or {}))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = lat.adjoint(steps, weight, target, r_box=r_box)
        t1 = time.perf_counter()
        lat.init(**(wl.init or {}))
        lat.sync()
        t2 = time.perf_counter()
        lat.step(steps)
        lat.sync()
        t3 = time.perf_counter()
        nf = lat.info()["n_fluid"]
    finally:
        lat.close()
    sec, fwd = t1 - t0, t3 - t2
    return {"workload": wl.name, "storage": "f32", "steps": steps, "n_fluid": nf,
            "ckpt_every": g["ckpt_every"], "n_checkpoints": g["n_checkpoints"],
            "seconds": round(sec, 4), "forward_seconds": round(fwd, 4),
            "ratio_to_forward": round(sec / fwd, 2),
            "gradient_mlups": round(nf * steps / sec / 1e6, 1),
            "bytes_per_node_step_model": ADJOINT_BYTES_F32,
            "model_gbs": round(nf * steps * ADJOINT_BYTES_F32 / sec / 1e9, 1),
            "loss": g["loss"], "d_D": g["d_D"]}


def batch_bench(steps=2000, seq_steps=400, n=64, seed=4703, chunk=64):
    """64 seeded gradient generators of uneven size (FP32): aggregate
    fluid-node updates per second of one batched, graph-captured launch per
    step (launch form from the library's autotuner) against stepping the
    instances one after the other with the same kernels."""
    import torch
    from paper_1307_4703_amd import Batch, Lattice, workloads as W
    wls = W.batch_instances(n, seed)
    log(f"batch: creating {n} lattices")
    lats = [Lattice.from_workload(wl, storage="f32") for wl in wls]
    nf = sum(l.info()["n_fluid"] for l in lats)
    # the library's autotuner picks the launch form (gg_batch_create with
    # GG_AUTOTUNE, the members left as they were)
    t0 = time.perf_counter()
    b = Batch(lats, tile=None, graph_chunk=chunk)
    tune_s = time.perf_counter() - t0
    f = b.form()
    best = {"tile": [f["tile_x"], f["tile_y"]], "persist": f["persist"], "fuse": f["fuse"],
            "rows": f["rows"]}
    log(f"batch: tuned tile {best['tile']} persist {best['persist']} "
        f"fuse {best['fuse']} rows {best['rows']} ({tune_s:.2f} s)")
    b.step(64)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    b.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    t_b = e0.elapsed_time(e1) * 1e-3
    b.close()
    for lat in lats:  # the same kernels, one lattice after the other
        lat.set_launch(best["tile"][0], best["tile"][1], chunk)
        lat.set_two_step(best["fuse"], best["rows"])
        lat.step(64)
    torch.cuda.synchronize()
    e0.record(stream)
    for lat in lats:
        lat.step(seq_steps)
    e1.record(stream)
    torch.cuda.synchronize()
    t_s = e0.elapsed_time(e1) * 1e-3
    for lat in lats:
        lat.close()
    mb = nf * steps / t_b / 1e6
    ms = nf * seq_steps / t_s / 1e6
    return {"n_instances": n, "seed": seed, "n_fluid_total": nf, "tile": best["tile"],
            "persist": best["persist"], "fuse": best["fuse"], "rows": best["rows"],
            "autotune_seconds": round(tune_s, 3),
            "steps": steps, "ms_per_step": round(t_b / steps * 1e3, 5),
            "batched_mlups": round(mb, 1), "sequential_mlups": round(ms, 1),
            "speedup": round(mb / ms, 3),
            "achieved_gbs": round(nf * bytes_per_update("f32") * steps / t_b / 1e9, 1)}


def cde_bytes_per_update(storage):
    # compound-only step: the 5 compound populations read once and written
    # once, the two components of the frozen velocity field read (FP64 for
    # FP64 storage, FP32 otherwise), the 1-byte link code
    return 5 * 2 * STORAGE_BYTES[storage] + 2 * (8 if storage == "f64" else 4) + 1


def cde_bench(name, steps, flow_steps, rows, chunk=64, layout="planes"):
    """The compound alone on a frozen velocity field (the paper's decoupled
    path): the flow developed for flow_steps coupled steps, its velocity
    captured into a field slot, then graph-replayed compound-only steps
    (two-step passes over tiles of `rows` rows, four-step passes over tiles
    of -rows rows, or single steps with rows 0)
    timed with HIP events on the lattice's stream, the populations in the
    given layout (gg_set_layout)."""
    import torch
    from paper_1307_4703_amd import Lattice
    wl = workload(name)
    lat = Lattice.from_workload(wl)
    lat.set_launch(64, 4, chunk)
    nf = lat.info()["n_fluid"]
    lat.step(flow_steps)
    lat.set_velocity_field(0)
    lat.set_layout(layout)  # (planes: the compound alone reads g only)
    lat_layout = lat.layout
    lat.set_cde_launch(rows)
    lat.cde_step(4 * max(chunk, 4))
    lat.sync()
    log(f"compound only, {wl.name}: {steps} steps (rows {rows}) on the field after "
        f"{flow_steps} coupled steps")
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    lat.cde_step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    d = lat.diagnostics(check_finite=False)
    lat.close()
    bpu = cde_bytes_per_update(wl.storage)
    spl = 4 if rows < 0 else (2 if rows else 1)  # steps per launch
    launch_ms = ms * spl
    ach = nf * bpu / (launch_ms * 1e-3) / 1e9
    return {"workload": wl.name, "storage": wl.storage, "n_fluid": nf, "steps": steps,
            "launch_form": {"rows": rows, "steps_per_launch": spl, "layout": lat_layout},
            "mlups": round(nf / (ms * 1e-3) / 1e6, 1),
            "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4),
                         "traffic": load_traffic("cde:" + name),
                         "algorithmic_bytes_per_launch": nf * bpu,
                         "kernel_ms": round(launch_ms, 5),
                         "update_rate_frac_of_single_step_roofline":
                             round(nf * bpu * spl / (launch_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)},
            "n_nonfinite": d["n_nonfinite"]}


# (workload, timed steps, coupled steps that develop the flow first, rows of
# the two-step tiles, minus the rows of the four-step tiles, or 0 for single
# steps, as measured fastest on this GPU)
CDE_LEG = (("gg2048_f32", 4096, 2000, 14), ("allfluid8192_f32", 512, 64, -6),
           ("gg8192_f16", 1024, 512, 0))


def cpu_baseline(name, budget_s=15.0, single_budget_s=4.0):
    """The FP64 oracle, as it stands, on the host cores: a bounded number of
    steps of the same workload from its initial state, on all cores and on
    one."""
    import numpy as np
    import oracle
    wl = workload(name)
    o = oracle.Oracle(wl.mask, tau_f=wl.tau_f, D=wl.D, w0=wl.w0, rho0=wl.rho0,
                      k_decay=wl.k_decay, periodic=wl.periodic, segments=wl.segments,
                      schedule=wl.schedule, t_origin=wl.t_origin)
    if wl.init:
        o.init(**wl.init)
    nf = int(np.count_nonzero(wl.mask == 0))
    cores = oracle.threads()
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter() - t0
    n = int(max(1, min(500, budget_s / max(t1, 1e-6))))
    log(f"cpu baseline: oracle {n} steps on {cores} threads (one step took {t1:.3f} s)")
    t0 = time.perf_counter()
    o.step(n)
    dt = time.perf_counter() - t0
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        o.step(1)
        t1s = time.perf_counter() - t0
        n1 = int(max(1, min(100, single_budget_s / max(t1s, 1e-6))))
        t0 = time.perf_counter()
        o.step(n1)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(nf * n / dt / 1e6, 2), "unit": "MLUPS", "cores": cores,
            "kind": "oracle",
            "sample": f"{n} FP64 oracle steps of {wl.name} ({nf} fluid nodes) from rest",
            "single_thread_value": round(nf * n1 / dt1 / 1e6, 2),
            "single_thread_sample": f"{n1} further steps on one thread",
            "cpu_model": model, "nproc": os.cpu_count()}


CTYPE = {"f64": "double", "f32": "float", "f16": "__half"}


def counters_leg(leg, tile, chunk_unused=0):
    """One leg of the counter runs (rocprofv3 --pmc runs the whole process):
    plain launches only (no graph replays), the calibration copy first, then
    the leg's kernels. Writes the manifest gpurun_out/counters/counters_<leg>.json
    naming, per workload, the dominant kernel (a part of its name) and its
    grid size, which the digest matches against the counter rows."""
    import torch
    from paper_1307_4703_amd import Batch, Lattice
    from paper_1307_4703_amd import workloads as W
    copy_bandwidth(nbytes=256 << 20, reps=2)
    manifest = {}
    if leg == "lattices":
        for name in ("gg8192_f16",) + tuple(n for n, _ in SECONDARY):
            wl = workload(name)
            lat = Lattice.from_workload(wl)
            lat.set_launch(tile[0], tile[1], 0)
            fuse, rows = FORMS.get(name, (3, 6))
            lat.set_two_step(fuse, rows)
            lat.step(4)
            p = lat.step_profile(16)
            lat.close()
            seg = "true" if p["fuse"] == 4 else "false"
            spp = p["steps_per_pass"]
            # rows + 2 wavefronts per tile, rows + 6 in the four-step pass
            waves = p["rows"] + (6 if spp == 4 else 2)
            grid = 8 * ((p["pass_tiles"] + 7) // 8) * waves * 64
            kern = "k_tile4" if spp == 4 else "k_tile2"
            manifest[name] = {"kernel": f"{kern}<{CTYPE[wl.storage]}, {seg}, {p['rows']},",
                              "grid": grid, "units": spp * p["pass_fluid"],
                              "bytes_per_update": bytes_per_update(wl.storage)}
            log(f"counters: {name} {manifest[name]}")
    elif leg == "batch":
        wls = W.batch_instances(64, 4703)
        lats = [Lattice.from_workload(wl, storage="f32") for wl in wls]
        # the form the library's autotuner picks for this batch on this GPU
        # (four-step passes, the boundary tiles apart): both kernels of
        # each pass, their bytes summed per pass
        b = Batch(lats, tile=(64, 4), graph_chunk=0, fuse=5, rows=6)
        b.step(16)
        torch.cuda.synchronize()
        b.close()
        nf = sum(l.info()["n_fluid"] for l in lats)
        manifest["batch64"] = {"kernel": "k_tile4<float,", "grid": None, "sum_kernels": True,
                               "units": 4 * nf, "bytes_per_update": bytes_per_update("f32")}
    elif leg == "adjoint":
        wl = workload("gg2048_f32")
        weight, target, r_box = W.chamber_misfit_setup(wl)
        lat = Lattice.from_workload(wl)
        lat.set_launch(64, 4, 0)
        lat.set_two_step(*ADJOINT_FORM)
        lat.adjoint(400, weight, target, r_box=r_box, ckpt_every=20)
        nf = lat.info()["n_fluid"]
        lat.close()
        # (the lattice steps in passes, so the adjoint steps go in pairs: two
        # adjoint steps per launch)
        manifest["adjoint:k_adjoint2"] = {"kernel": "k_adjoint2<float, 6>", "grid": None,
                                          "units": 2 * nf,
                                          "bytes_per_update": ADJOINT_STEP_BYTES_F32}
        manifest["adjoint:taped_pass"] = {"kernel": "k_tile2<float, true, 6, false, true, true>",
                                          "grid": None, "units": 2 * nf,
                                          "bytes_per_update": bytes_per_update("f32") / 2 + 28}
    elif leg == "cde":
        for name, steps, flow, rows in CDE_LEG:
            r = cde_bench(name, 16, 4, rows, 0)
            ct = CTYPE[r["storage"]]
            if rows < 0:
                # (the only four-step compound kernel of the leg)
                kern, grid = f"k_cde_tile4<{ct}, {-rows},", None
            elif rows:
                # the compound-only pass walks the tile list of the one-kernel
                # coupled pass of the same height
                lat = Lattice.from_workload(workload(name))
                lat.set_launch(tile[0], tile[1], 0)
                lat.set_two_step(4, rows)
                lat.step(4)
                p = lat.step_profile(2)
                lat.close()
                kern = f"k_cde_tile2<{ct}, {rows},"
                grid = 8 * ((p["pass_tiles"] + 7) // 8) * (rows + 2) * 64
            else:
                kern, grid = f"k_cde<{ct},", None
            # one trip of the compound's bytes per launch (a pass moves them
            # once for its two or four steps)
            manifest["cde:" + name] = {"kernel": kern, "grid": grid, "units": r["n_fluid"],
                                       "bytes_per_update": cde_bytes_per_update(r["storage"])}
    else:
        raise SystemExit(f"unknown counter leg {leg}")
    out_dir = os.path.join(ROOT, "gpurun_out", "counters")
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, f"counters_{leg}.json"), "w") as fh:
        json.dump(manifest, fh, indent=1)
    print(json.dumps(manifest), flush=True)


def digest_counters(prof_dir, out_path):
    """Turn the counter runs of each leg (rocprofv3 --pmc FETCH_SIZE, then
    --pmc WRITE_SIZE, KiB per dispatch, under prof_dir/<leg>_fetch and
    prof_dir/<leg>_write, with the leg's manifest counters_<leg>.json) into
    HBM bytes per launch of each workload's dominant kernel, scaled per leg
    by what the same counters read for the plain copy kernel of known size;
    writes ``out_path`` (JSON)."""
    import csv
    import glob
    from collections import defaultdict

    def per_dispatch(path, counter):
        acc = defaultdict(list)
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] == counter:
                    acc[(row["Kernel_Name"], int(row["Grid_Size"]))].append(float(row["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in acc.items()}

    data = {"kernel_sha": kernel_hash(), "source": [os.path.relpath(p, ROOT) for p in KERNEL_SRC],
            "legs": {}, "workloads": {}}
    for man_path in sorted(glob.glob(os.path.join(prof_dir, "counters_*.json"))):
        leg = os.path.basename(man_path)[len("counters_"):-len(".json")]
        with open(man_path) as fh:
            manifest = json.load(fh)
        fcsv = glob.glob(os.path.join(prof_dir, f"{leg}_fetch", "*counter_collection.csv"))
        wcsv = glob.glob(os.path.join(prof_dir, f"{leg}_write", "*counter_collection.csv"))
        if not fcsv or not wcsv:
            continue
        fetch = per_dispatch(fcsv[0], "FETCH_SIZE")
        write = per_dispatch(wcsv[0], "WRITE_SIZE")
        copy = [k for k in fetch if "k_copy" in k[0]]
        if len(copy) != 1:
            raise SystemExit(f"{leg}: expected exactly one copy-kernel grid")
        ck = copy[0]
        n_copy = ck[1] * 16  # one 16-byte vector per lane, read and written
        fs, ws = n_copy / 1024.0 / fetch[ck], n_copy / 1024.0 / write[ck]
        data["legs"][leg] = {"fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
                             "calibration": {"kernel": "gg::k_copy", "bytes_read": n_copy,
                                             "bytes_written": n_copy,
                                             "FETCH_SIZE_KiB": fetch[ck],
                                             "WRITE_SIZE_KiB": write[ck]}}
        for name, m in manifest.items():
            keys = [k for k in fetch if m["kernel"] in k[0] and (m["grid"] is None or k[1] == m["grid"])]
            if not keys:
                raise SystemExit(f"{leg}: no kernel {m['kernel']!r} grid {m['grid']} ({name})")
            # per launch of the kernel (averaged over its grids), or, with
            # sum_kernels, per pass: the mean of each matching kernel summed
            # (the pass launches each of them once)
            div = 1 if m.get("sum_kernels") else len(keys)
            fb = sum(fetch[k] for k in keys) / div * 1024 * fs
            wb = sum(write.get(k, 0.0) for k in keys) / div * 1024 * ws
            alg = m["units"] * m["bytes_per_update"]
            data["workloads"][name] = {
                "kernel": m["kernel"], "grid_size": m["grid"], "leg": leg,
                "fetch_bytes_per_launch": round(fb), "write_bytes_per_launch": round(wb),
                "bytes_per_launch": round(fb + wb),
                "algorithmic_bytes_per_launch": round(alg),
                "ratio_to_algorithmic": round((fb + wb) / alg, 4)}
    with open(out_path, "w") as fh:
        json.dump(data, fh, indent=1)
    return data


def lattice_entry(r, traffic):
    """Secondary-lattice record: rate, roofline of the dominant kernel."""
    e = roofline(r, r["wl"].storage, traffic)
    e["mlups"] = round(r["nf"] * r["steps"] / (r["event_ms"] * 1e-3) / 1e6, 1)
    e["workload"] = r["wl"].name
    e["storage"] = r["wl"].storage
    e["n_fluid"] = r["nf"]
    e["steps"] = r["steps"]
    e["launch_form"] = r["form"]
    if r["graph_replayed"]:
        e["graph_replayed"] = r["graph_replayed"]
    return e


# secondary lattices of the default run: (workload, timed steps)
SECONDARY = (("gg2048_f32", 4000), ("allfluid8192_f32", 1000), ("allfluid8192_f16", 1000),
             ("gg8192_f32", 2000), ("shard8192x512_f32", 2000), ("allfluid8192_f64", 400),
             ("gg2048_f64", 2000))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=400)
    ap.add_argument("--workload", default="gg8192_f16")
    ap.add_argument("--tile", default="64x4")
    ap.add_argument("--chunk", type=int, default=64,
                    help="graph chunk of the graph-replayed comparison and of the batch "
                         "and adjoint legs (0: plain launches everywhere)")
    ap.add_argument("--monitor-every", type=int, default=1024,
                    help="FP64 diagnostics reduction every this many timed steps")
    ap.add_argument("--fuse", type=int, default=0,
                    help="launch form (1 single steps, 2-4 two-step passes); 0: the "
                         "workload's default form")
    ap.add_argument("--tune", action="store_true", help="autotune the launch form")
    ap.add_argument("--rows", type=int, default=6, help="rows of the two-step strips or tiles")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-instances leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint (gradient) leg")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the FP32/FP16-vs-FP64 error leg")
    ap.add_argument("--precision-steps", type=int, default=20000)
    ap.add_argument("--no-extra", action="store_true",
                    help="headline only: no secondary lattices, copy bandwidth, compound-only, "
                         "batch, adjoint, precision or experiment legs")
    ap.add_argument("--experiments", action="store_true",
                    help="also run the step-profile and boundary-kind experiments")
    ap.add_argument("--cde-only", action="store_true",
                    help="time only the compound-only step on frozen velocity fields")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="time only the adjoint (gradient) leg")
    ap.add_argument("--batch-only", action="store_true", help="time only the batched leg")
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--adjoint-steps", type=int, default=20000)
    ap.add_argument("--cde-steps", type=int, default=0,
                    help="timed compound-only steps per lattice (0: the defaults)")
    ap.add_argument("--cde-layout", choices=["planes", "paired"], default="planes",
                    help="population layout of the compound-only leg")
    ap.add_argument("--counters", metavar="LEG",
                    choices=["lattices", "batch", "adjoint", "cde"],
                    help="no benchmark: run one leg with plain launches for rocprofv3 --pmc "
                         "(the manifest goes to gpurun_out/counters/counters_LEG.json)")
    ap.add_argument("--digest", metavar="DIR",
                    help="no run: digest rocprofv3 counter CSVs and manifests under DIR "
                         "into profiles/traffic.json")
    args = ap.parse_args(argv)
    if args.digest:
        d = digest_counters(args.digest, os.path.join(ROOT, "profiles", "traffic.json"))
        print(json.dumps(d["workloads"]))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the library does not shard a lattice across GPUs)", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be positive and --warmup non-negative", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    tile = tuple(int(v) for v in args.tile.split("x"))
    cde_leg = [(n, args.cde_steps or k, f, r) for n, k, f, r in CDE_LEG]
    if args.cde_only:
        print(json.dumps({name: cde_bench(name, steps, flow, rows, args.chunk, args.cde_layout)
                          for name, steps, flow, rows in cde_leg}), flush=True)
        return
    if args.adjoint_only:
        print(json.dumps(adjoint_bench(args.adjoint_steps, args.chunk)), flush=True)
        return
    if args.batch_only:
        print(json.dumps(batch_bench(args.batch_steps, chunk=args.chunk)), flush=True)
        return
    if args.counters:
        counters_leg(args.counters, tile)
        return

    form = "tune" if args.tune else ({"fuse": args.fuse, "rows": args.rows} if args.fuse else None)
    r = time_lattice(args.workload, args.steps, args.warmup, tile, args.chunk, form,
                     args.monitor_every, graph_steps=None if args.no_extra else max(args.steps, 1000))
    wl, nf, p = r["wl"], r["nf"], r["prof"]
    d = r["diag"]
    out = {
        "metric": METRIC,
        "value": round(nf * args.steps / (r["event_ms"] * 1e-3) / 1e6, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["event_ms"] / args.steps, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if wl.storage == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "nx": wl.nx, "ny": wl.ny, "n_fluid": nf,
                   "storage": {"f16": "FP16-shifted (f - w rho0, g - w C_s)", "f32": "FP32",
                               "f64": "FP64"}[wl.storage],
                   "collision_arithmetic": "f64" if wl.storage == "f64" else "f32",
                   "reductions": "f64",
                   "peclet": getattr(wl, "peclet", None), "D": wl.D, "tau_f": wl.tau_f,
                   "valve_half_period": wl.schedule[0].duration if wl.schedule else None,
                   "launch_form": r["form"],
                   "launches": {"pass_kernel": p["n_pass"] + p["graph_passes"],
                                "steps_per_pass": p["steps_per_pass"],
                                "pass_kernel_in_graph_replays": p["graph_passes"],
                                "two_step_pass_beside_four_step": p["n_pass2"],
                                "graph_replays": p["n_graph"],
                                "single_even": p["n_single"][0],
                                "single_odd": p["n_single"][1],
                                "single_in_graph_replays": p["graph_singles"]},
                   "graph_chunk": r["graph_chunk"],
                   "warmup_steps_run": r["warmup_run"],
                   "monitor_every": r["monitor_every"], "monitor_reductions": p["n_monitor"],
                   "bytes_per_update": bytes_per_update(wl.storage),
                   "wall_clock_mlups": round(nf * args.steps / r["wall_s"] / 1e6, 1),
                   "lattice_mlups": round(wl.nx * wl.ny * args.steps / (r["event_ms"] * 1e-3) / 1e6, 1),
                   "parallelism": "single GPU"},
        "roofline": roofline(r, wl.storage, load_traffic(args.workload)),
        "diagnostics": {"t": d["t"], "mass": d["mass"], "solute": d["solute"],
                        "n_nonfinite": d["n_nonfinite"], "max_u": d["max_u"],
                        "max_u_chamber": d["max_u_region"],
                        "max_cell_peclet_chamber": d["max_pe_region"]},
    }
    if r["graph_replayed"]:
        out["graph_replayed"] = r["graph_replayed"]
    if not args.no_extra:
        out["copy_bandwidth_gbs"] = round(copy_bandwidth(), 1)
        log(f"plain copy: {out['copy_bandwidth_gbs']} GB/s")
        extra = {}
        for name, steps in SECONDARY:
            if name == args.workload:
                continue
            r2 = time_lattice(name, steps, 100, tile, args.chunk, form, args.monitor_every,
                              graph_steps=steps)
            extra[name] = lattice_entry(r2, load_traffic(name))
        out["other_lattices"] = extra
        out["compound_only_frozen_velocity"] = {
            name: cde_bench(name, steps, flow, rows, args.chunk)
            for name, steps, flow, rows in cde_leg}
        if not args.no_batch:
            out["batched_64_instances"] = batch_bench(args.batch_steps, chunk=args.chunk)
        if not args.no_adjoint:
            log(f"adjoint: chamber-misfit gradient over {args.adjoint_steps} steps, 2048x1024 FP32")
            out["adjoint_gradient"] = adjoint_bench(args.adjoint_steps, args.chunk)
        if not args.no_precision:
            from paper_1307_4703_amd import experiments
            from paper_1307_4703_amd import workloads as W
            log(f"reduced-precision storage against FP64: 8192x4096, Pe 500 and 2000, "
                f"{args.precision_steps} steps")
            out["precision_vs_fp64"] = {
                "gg8192_pe500": experiments.precision_report(
                    W.gradient_generator(scale=4.0, storage="f16", peclet=500.0), ("f16", "f32"),
                    steps=args.precision_steps),
                "gg8192_pe2000": experiments.precision_report(
                    W.gradient_generator(scale=4.0, storage="f16", peclet=2000.0), ("f16",),
                    steps=args.precision_steps)}
        if args.experiments:
            from paper_1307_4703_amd import experiments
            log("step-profile test (Table 3), four cases, FP32")
            out["step_profile_table3"] = experiments.step_profile_summary(storage="f32")
            log("boundary kinds: velocity inlet / outflow links against the pressure boundary")
            out["boundary_kinds"] = experiments.boundary_comparison()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
        out["cpu_baseline"]["gpu_over_cpu"] = round(out["value"] / out["cpu_baseline"]["value"], 1)
    print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main()
