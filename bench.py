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
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "coupled NSE+CDE MLUPS and % HBM roofline on 1 MI355X; FP32/FP16 vs FP64 error"
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2}
KERNEL_SRC = os.path.join(ROOT, "paper_1307_4703_amd", "csrc", "gg_kernels.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bytes_per_update(storage):
    # in-place AA: every one of the 9 + 5 populations read once and written
    # once per fluid-node update, plus the 1-byte link code
    return 14 * 2 * STORAGE_BYTES[storage] + 1


def workload(name):
    from paper_1307_4703_amd import workloads as W
    if name == "gg2048_f32":
        return W.gradient_generator(storage="f32")
    if name == "gg2048_f16":
        return W.gradient_generator(storage="f16")
    if name == "gg8192_f16":
        return W.gradient_generator(scale=4.0, storage="f16")
    if name == "gg8192_f32":
        return W.gradient_generator(scale=4.0, storage="f32")
    if name == "allfluid8192_f32":
        return W.all_fluid_channel(storage="f32")
    if name == "allfluid8192_f16":
        return W.all_fluid_channel(storage="f16")
    if name == "straight_f64":
        return W.straight_channel()
    raise SystemExit(f"unknown workload {name}")


def kernel_hash():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def load_traffic(wl_name):
    """HBM bytes per step launch from committed rocprofv3 counter runs, or
    None when they are missing or were taken on another kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = data.get(wl_name)
    if not ent or ent.get("kernel_sha") != kernel_hash():
        return None
    return ent.get("bytes_per_launch")


def make_lattice(name, tile, chunk):
    from paper_1307_4703_amd import Lattice
    wl = workload(name)
    lat = Lattice.from_workload(wl)
    lat.set_launch(tile[0], tile[1], chunk)
    return wl, lat


def time_lattice(name, steps, warmup, tile, chunk):
    import torch
    wl, lat = make_lattice(name, tile, chunk)
    nf = lat.info()["n_fluid"]
    log(f"{wl.name}: {wl.nx}x{wl.ny}, {nf} fluid nodes, storage {wl.storage}, "
        f"tile {tile}, graph chunk {chunk}; warmup {warmup}")
    lat.step(warmup)
    lat.sync()
    torch.cuda.synchronize()
    log(f"timed region: {steps} steps")
    t0 = time.perf_counter()
    lat.step(steps)
    lat.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_k = min(steps, 2000)
    log(f"per-kernel event timing over {n_k} step launches")
    kms = lat.step_timed(n_k)
    diag = lat.diagnostics()
    lat.close()
    return wl, nf, dt, kms, diag


def copy_bandwidth(nbytes=2 << 30, reps=20):
    import ctypes
    import torch
    from paper_1307_4703_amd import _abi as A
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    ms = ctypes.c_double()
    stream = torch.cuda.current_stream().cuda_stream
    A.call("gg_stream_copy", ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(a.data_ptr()),
           nbytes, reps, ctypes.c_void_p(stream), ctypes.byref(ms))
    return 2.0 * nbytes / (ms.value * 1e-3) / 1e9, ms.value


def cpu_baseline(name, budget_s=15.0):
    """The FP64 oracle, as it stands, on the host cores: a bounded number of
    steps of the same workload from its initial state."""
    import numpy as np
    import oracle
    wl = workload(name)
    o = oracle.Oracle(wl.mask, tau_f=wl.tau_f, D=wl.D, w0=wl.w0, rho0=wl.rho0,
                      k_decay=wl.k_decay, periodic=wl.periodic, segments=wl.segments,
                      schedule=wl.schedule, t_origin=wl.t_origin)
    if wl.init:
        o.init(**wl.init)
    nf = int(np.count_nonzero(wl.mask == 0))
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter() - t0
    n = int(max(1, min(500, budget_s / max(t1, 1e-6))))
    log(f"cpu baseline: oracle {n} steps (one step took {t1:.3f} s)")
    t0 = time.perf_counter()
    o.step(n)
    dt = time.perf_counter() - t0
    return {"value": nf * n / dt / 1e6, "unit": "MLUPS", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{n} FP64 oracle steps of {wl.name} ({nf} fluid nodes) from its initial state"}


def roofline(nf, storage, kms, traffic):
    bpl = nf * bytes_per_update(storage)
    ach = bpl / (kms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(ach / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": bpl,
            "kernel_ms": round(kms, 5)}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--workload", default="gg2048_f32")
    ap.add_argument("--tile", default="64x4")
    ap.add_argument("--chunk", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the out-of-cache roofline lattice and the copy bandwidth")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the lattice is not sharded across GPUs in this build)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    tile = tuple(int(v) for v in args.tile.split("x"))

    wl, nf, dt, kms, diag = time_lattice(args.workload, args.steps, args.warmup, tile, args.chunk)
    mlups = nf * args.steps / dt / 1e6
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if wl.storage == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "nx": wl.nx, "ny": wl.ny, "n_fluid": nf,
                   "storage": wl.storage, "D": wl.D, "tau_f": wl.tau_f,
                   "schedule_half_period": wl.schedule[0].duration if wl.schedule else None,
                   "tile": args.tile, "graph_chunk": args.chunk,
                   "bytes_per_update": bytes_per_update(wl.storage),
                   "lattice_updates_per_s": round(wl.nx * wl.ny * args.steps / dt / 1e6, 1),
                   "parallelism": "single GPU"},
        "roofline": roofline(nf, wl.storage, kms, load_traffic(args.workload)),
        "mass_drift_check": {"t": diag["t"], "mass": diag["mass"],
                             "max_u_chamber": diag["max_u_region"],
                             "max_cell_peclet_chamber": diag["max_pe_region"]},
    }
    if not args.no_extra:
        try:
            bw, cms = copy_bandwidth()
            out["copy_bandwidth_gbs"] = round(bw, 1)
            log(f"plain copy: {bw:.0f} GB/s")
        except Exception as e:  # report, do not hide
            out["copy_bandwidth_gbs"] = f"failed: {e}"
        if args.workload.startswith("gg2048"):
            st = args.workload.split("_")[1]
            name = f"allfluid8192_{st}"
            wl2, nf2, dt2, kms2, _ = time_lattice(name, 1000, 100, tile, args.chunk)
            r2 = roofline(nf2, wl2.storage, kms2, load_traffic(name))
            r2["workload"] = wl2.name
            r2["mlups"] = round(nf2 * 1000 / dt2 / 1e6, 1)
            out["roofline_out_of_cache"] = r2
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
