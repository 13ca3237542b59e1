#!/usr/bin/env python3
"""Throughput of the coupled D2Q9 + D2Q5 lattice Boltzmann step on one MI355X.

One benchmark step is one coupled time step (collide + stream of both
lattices, boundary links, valve schedule, FP64 boundary-flux accumulation)
over the whole synthetic lattice, with the state resident in HBM. The
default workload is the 2048 x 1024 gradient generator in FP32 storage
(channel Peclet 500, valves toggling every 2000 steps).

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
FORMS = {"gg2048_f32": (4, 6), "gg2048_f16": (4, 6), "gg8192_f16": (3, 6),
         "gg8192_f16_pe2000": (3, 6), "gg8192_f32": (3, 6), "allfluid8192_f32": (3, 14),
         "allfluid8192_f16": (3, 6), "shard8192x512_f32": (3, 6),
         "allfluid8192_f64": (3, 14), "gg2048_f64": (3, 14), "straight_f64": (4, 6)}


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


def time_lattice(name, steps, warmup, tile, chunk, form=None):
    """Graph-replayed steps timed with HIP events on the lattice's stream
    (torch's current stream), after the autotuner picked the launch form
    (single steps or a two-step pass); plus per-kernel timings."""
    import torch
    from paper_1307_4703_amd import Lattice
    from paper_1307_4703_amd import tune as T
    wl = workload(name)
    lat = Lattice.from_workload(wl)
    lat.set_launch(tile[0], tile[1], chunk)
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
    log(f"{wl.name}: {wl.nx}x{wl.ny}, {nf} fluid nodes, storage {wl.storage}, "
        f"form {form}, graph chunk {chunk}; warmup {warmup}")
    lat.step(warmup)
    lat.sync()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    log(f"timed region: {steps} steps")
    t0 = time.perf_counter()
    ev0.record(stream)
    lat.step(steps)
    ev1.record(stream)
    lat.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    n_k = min(steps, 200 if nf > 1e7 else 1000)
    extra = {}
    if form["fuse"] >= 2:
        extra["ms_pass_plain_launches"] = lat.step2_timed(max(1, n_k // 4))
    fuse = form["fuse"]
    lat.set_two_step(1)  # single-step kernels, for the breakdown
    ms_even, ms_odd = lat.step_timed(n_k)
    diag = lat.diagnostics(check_finite=False)
    lat.close()
    spl = 2 if fuse >= 2 else 1  # steps per launch of the dominant kernel
    return {"wl": wl, "nf": nf, "wall_s": wall, "event_ms": ev_ms, "form": form,
            "steps_per_launch": spl, "launch_ms": ev_ms / steps * spl,
            "ms_even": ms_even, "ms_odd": ms_odd, "diag": diag, **extra}


def roofline(r, storage, traffic):
    """Dominant kernel: the two-step pass (each population read and written
    once per launch, two steps) or the single step; algorithmic bytes per
    launch = fluid nodes x (14 x 2 x storage bytes + 1 link byte)."""
    bpl = r["nf"] * bytes_per_update(storage)
    ach = bpl / (r["launch_ms"] * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": traffic,
           "algorithmic_bytes_per_launch": bpl, "steps_per_launch": r["steps_per_launch"],
           "kernel_ms": round(r["launch_ms"], 5),
           "single_step_kernel_ms_even_odd": [round(r["ms_even"], 5), round(r["ms_odd"], 5)],
           # the rate in updates, priced at the single-step bytes per update
           "update_rate_frac_of_single_step_roofline":
               round(r["nf"] * bytes_per_update(storage) * r["steps_per_launch"] /
                     (r["launch_ms"] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    if "ms_pass_plain_launches" in r:
        out["kernel_ms_pass_plain_launches"] = round(r["ms_pass_plain_launches"], 5)
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


def adjoint_bench(steps=20000):
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
        lat.set_launch(64, 4, 64)
        lat.set_two_step(*FORMS["gg2048_f32"])
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


def batch_bench(steps=2000, seq_steps=400, n=64, seed=4703, tune_steps=32):
    """64 seeded gradient generators of uneven size (FP32): aggregate
    fluid-node updates per second of one batched, graph-captured launch per
    step (launch shape from the autotuner) against stepping the instances
    one after the other with the same kernels."""
    import torch
    from paper_1307_4703_amd import Batch, Lattice, tune, workloads as W
    wls = W.batch_instances(n, seed)
    log(f"batch: creating {n} lattices")
    lats = [Lattice.from_workload(wl, storage="f32") for wl in wls]
    nf = sum(l.info()["n_fluid"] for l in lats)
    best = tune.tune_batch(lats, steps=tune_steps, use_cache=False)
    log(f"batch: tuned tile {best['tile']} persist {best['persist']} "
        f"fuse {best['fuse']} rows {best['rows']}")
    b = Batch(lats, tile=tuple(best["tile"]), persist=best["persist"], graph_chunk=64,
              fuse=best["fuse"], rows=best["rows"])
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
        lat.set_launch(best["tile"][0], best["tile"][1], 64)
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
            "steps": steps, "ms_per_step": round(t_b / steps * 1e3, 5),
            "batched_mlups": round(mb, 1), "sequential_mlups": round(ms, 1),
            "speedup": round(mb / ms, 3),
            "achieved_gbs": round(nf * bytes_per_update("f32") * steps / t_b / 1e9, 1)}


def cde_bytes_per_update(storage):
    # compound-only step: the 5 compound populations read once and written
    # once, the two components of the frozen velocity field read (FP64 for
    # FP64 storage, FP32 otherwise), the 1-byte link code
    return 5 * 2 * STORAGE_BYTES[storage] + 2 * (8 if storage == "f64" else 4) + 1


def cde_bench(name, steps, flow_steps, rows, chunk=64):
    """The compound alone on a frozen velocity field (the paper's decoupled
    path): the flow developed for flow_steps coupled steps, its velocity
    captured into a field slot, then graph-replayed compound-only steps
    (two-step passes over tiles of `rows` rows, or single steps with rows 0)
    timed with HIP events on the lattice's stream."""
    import torch
    from paper_1307_4703_amd import Lattice
    wl = workload(name)
    lat = Lattice.from_workload(wl)
    lat.set_launch(64, 4, chunk)
    nf = lat.info()["n_fluid"]
    lat.step(flow_steps)
    lat.set_velocity_field(0)
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
    spl = 2 if rows else 1  # steps per launch
    launch_ms = ms * spl
    ach = nf * bpu / (launch_ms * 1e-3) / 1e9
    return {"workload": wl.name, "storage": wl.storage, "n_fluid": nf, "steps": steps,
            "launch_form": {"rows": rows, "steps_per_launch": spl},
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
# the two-step tiles or 0 for single steps, as measured fastest on this GPU)
CDE_LEG = (("gg2048_f32", 4096, 2000, 14), ("allfluid8192_f32", 512, 64, 14),
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


def digest_counters(prof_dir, grids, out_path):
    """Turn two rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE, KiB per
    dispatch) into HBM bytes per step launch for the workloads named in
    ``grids`` ({"grid size/kernel name part": workload}; the bytes of all
    matching kernels are averaged), scaled by what the same counters read
    for the plain copy kernel of known size; writes ``out_path`` (JSON)."""
    import csv
    from collections import defaultdict

    def per_dispatch(path, counter):
        acc = defaultdict(list)
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] == counter:
                    acc[(row["Kernel_Name"], int(row["Grid_Size"]))].append(float(row["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in acc.items()}

    fetch = per_dispatch(os.path.join(prof_dir, "pmc_fetch", "fetch_counter_collection.csv"),
                         "FETCH_SIZE")
    write = per_dispatch(os.path.join(prof_dir, "pmc_write", "write_counter_collection.csv"),
                         "WRITE_SIZE")
    copy = [k for k in fetch if "k_copy" in k[0]]
    if len(copy) != 1:
        raise SystemExit("expected exactly one copy-kernel grid in the counter runs")
    ck = copy[0]
    n_copy = ck[1] * 16  # one 16-byte vector per lane, read and written
    fs, ws = n_copy / 1024.0 / fetch[ck], n_copy / 1024.0 / write[ck]
    data = {"kernel_sha": kernel_hash(), "source": [os.path.relpath(p, ROOT) for p in KERNEL_SRC],
            "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
            "calibration": {"kernel": "gg::k_copy", "bytes_read": n_copy, "bytes_written": n_copy,
                            "FETCH_SIZE_KiB": fetch[ck], "WRITE_SIZE_KiB": write[ck]},
            "workloads": {}}
    for key, name in grids.items():
        grid, _, kname = key.partition("/")
        grid = int(grid)
        steps = {k: v for k, v in fetch.items() if k[1] == grid and kname in k[0]}
        if not steps:
            raise SystemExit(f"no kernel {kname!r} with grid size {grid} ({name})")
        par = {}
        for k in steps:
            m = re.search(r"k_\w+(<[^>]*>)?", k[0])
            tag = m.group(0) if m else k[0]
            par[tag] = {"fetch_bytes": round(fetch[k] * 1024 * fs),
                        "write_bytes": round(write.get(k, 0.0) * 1024 * ws)}
        tot = [v["fetch_bytes"] + v["write_bytes"] for v in par.values()]
        bpl = round(sum(tot) / len(tot))
        cde = name.startswith("cde:")
        wl = workload(name[4:] if cde else name)
        import numpy as np
        bpu = cde_bytes_per_update(wl.storage) if cde else bytes_per_update(wl.storage)
        alg = int(np.count_nonzero(wl.mask == 0)) * bpu
        data["workloads"][name] = {"bytes_per_launch": bpl, "algorithmic_bytes_per_launch": alg,
                                   "ratio_to_algorithmic": round(bpl / alg, 4),
                                   "per_kernel": par, "grid_size": grid, "kernel": kname}
    with open(out_path, "w") as fh:
        json.dump(data, fh, indent=1)
    return data


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--workload", default="gg2048_f32")
    ap.add_argument("--tile", default="64x4")
    ap.add_argument("--chunk", type=int, default=64)
    ap.add_argument("--fuse", type=int, default=0,
                    help="launch form (1 single steps, 2-4 two-step passes); 0: the "
                         "workload's default form")
    ap.add_argument("--tune", action="store_true", help="autotune the launch form")
    ap.add_argument("--rows", type=int, default=6, help="rows of the two-step strips or tiles")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-instances leg")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the out-of-cache and FP16 lattices and the copy bandwidth")
    ap.add_argument("--no-experiments", action="store_true",
                    help="skip the step-profile, boundary-kind and precision legs")
    ap.add_argument("--cde-only", action="store_true",
                    help="time only the compound-only step on frozen velocity fields")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="time only the adjoint (gradient) leg")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint (gradient) leg (counter runs: rocprofv3 --pmc "
                         "ended the process with a segmentation fault inside it)")
    ap.add_argument("--cde-steps", type=int, default=0,
                    help="timed compound-only steps per lattice (0: the defaults)")
    ap.add_argument("--digest", metavar="DIR",
                    help="no run: digest rocprofv3 counter CSVs under DIR into profiles/traffic.json")
    ap.add_argument("--grids", default="",
                    help="with --digest: grid/kernel=workload pairs, separated by ';' "
                         "(kernel: a part of the kernel name, e.g. k_tile2<float)")
    args = ap.parse_args()
    if args.digest:
        grids = dict(kv.split("=") for kv in args.grids.split(";") if kv)
        d = digest_counters(args.digest, grids, os.path.join(ROOT, "profiles", "traffic.json"))
        print(json.dumps(d["workloads"]))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the library does not shard a lattice across GPUs)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    tile = tuple(int(v) for v in args.tile.split("x"))
    cde_leg = [(n, args.cde_steps or k, f, r) for n, k, f, r in CDE_LEG]
    if args.cde_only:
        print(json.dumps({name: cde_bench(name, steps, flow, rows, args.chunk)
                          for name, steps, flow, rows in cde_leg}), flush=True)
        return
    if args.adjoint_only:
        print(json.dumps(adjoint_bench()), flush=True)
        return

    form = "tune" if args.tune else ({"fuse": args.fuse, "rows": args.rows} if args.fuse else None)
    r = time_lattice(args.workload, args.steps, args.warmup, tile, args.chunk, form)
    wl, nf = r["wl"], r["nf"]
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
                   "storage": wl.storage, "D": wl.D, "tau_f": wl.tau_f,
                   "valve_half_period": wl.schedule[0].duration if wl.schedule else None,
                   "launch_form": r["form"], "graph_chunk": args.chunk,
                   "bytes_per_update_single_step": bytes_per_update(wl.storage),
                   "wall_clock_mlups": round(nf * args.steps / r["wall_s"] / 1e6, 1),
                   "lattice_mlups": round(wl.nx * wl.ny * args.steps / (r["event_ms"] * 1e-3) / 1e6, 1),
                   "parallelism": "single GPU"},
        "roofline": roofline(r, wl.storage, load_traffic(args.workload)),
        "diagnostics": {"t": r["diag"]["t"], "mass": r["diag"]["mass"],
                        "n_nonfinite": r["diag"]["n_nonfinite"],
                        "max_u_chamber": r["diag"]["max_u_region"],
                        "max_cell_peclet_chamber": r["diag"]["max_pe_region"]},
    }
    if not args.no_extra:
        out["copy_bandwidth_gbs"] = round(copy_bandwidth(), 1)
        log(f"plain copy: {out['copy_bandwidth_gbs']} GB/s")
        extra = {}
        for name, steps in (("allfluid8192_f32", 1000), ("allfluid8192_f16", 1000),
                            ("gg8192_f16", 2000), ("shard8192x512_f32", 2000),
                            ("allfluid8192_f64", 400), ("gg2048_f64", 4000)):
            if name == args.workload:
                continue
            r2 = time_lattice(name, steps, 100, tile, args.chunk, form)
            e = roofline(r2, r2["wl"].storage, load_traffic(name))
            e["mlups"] = round(r2["nf"] * steps / (r2["event_ms"] * 1e-3) / 1e6, 1)
            e["workload"] = r2["wl"].name
            e["storage"] = r2["wl"].storage
            extra[name] = e
        out["roofline_other_lattices"] = extra
        out["compound_only_frozen_velocity"] = {
            name: cde_bench(name, steps, flow, rows, args.chunk)
            for name, steps, flow, rows in cde_leg}
        if not args.no_batch:
            out["batched_64_instances"] = batch_bench()
        if not args.no_adjoint:
            log("adjoint: chamber-misfit gradient over 20000 steps, 2048x1024 FP32")
            out["adjoint_gradient"] = adjoint_bench()
    if not args.no_extra and not args.no_experiments:
        from paper_1307_4703_amd import experiments
        log("step-profile test (Table 3), four cases, FP32")
        out["step_profile_table3"] = experiments.step_profile_summary(storage="f32")
        log("boundary kinds: velocity inlet / outflow links against the pressure boundary")
        out["boundary_kinds"] = experiments.boundary_comparison()
        log("reduced-precision storage against FP64: 8192x4096 (Pe 500, 2000) and 2048x1024")
        from paper_1307_4703_amd import workloads as W
        out["precision_vs_fp64"] = {
            "gg8192_pe500": experiments.precision_report(
                W.gradient_generator(scale=4.0, storage="f16", peclet=500.0), ("f16", "f32")),
            "gg8192_pe2000": experiments.precision_report(
                W.gradient_generator(scale=4.0, storage="f16", peclet=2000.0), ("f16",)),
            "gg2048_pe500": experiments.precision_report(W.gradient_generator(), ("f32", "f16"))}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
