"""Launch-shape autotuner for single lattices and batches.

Candidates are tile shapes (tile_x x tile_y nodes per work-group) of the
single steps, the forms of the two-step pass (walking strips, row-parallel
tiles with the boundary rules in a kernel of their own or in the one
kernel) and the four-step pass, for batches persistent grid sizes, and for the compound-only step
the row count of its two-step tiles. Each candidate is timed
on the GPU with HIP events over a few graph-replayed steps (the lattices
advance while being tuned, so tune before the run or on a copy). Results are cached in a JSON
file keyed by the device name, storage type and the lattices' shapes and
fluid counts.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

from ._abi import GGError

TILES: Tuple[Tuple[int, int], ...] = ((64, 4), (32, 8), (64, 2), (128, 2), (128, 1),
                                      (64, 8), (128, 4), (256, 1), (32, 4), (16, 8))
PERSIST: Tuple[int, ...] = (0, 2048, 4096)
# (fuse, rows) of gg_set_two_step; fuse 1 is the single-step path
TWO_STEP: Tuple[Tuple[int, int], ...] = ((3, 6), (3, 14), (4, 6), (4, 14), (5, 6), (2, 8),
                                         (2, 16))


def cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "paper_1307_4703_amd", "tune.json")


def _key(lattices: Sequence, kind: str) -> str:
    import torch
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    desc = [(l.nx, l.ny, l.storage, l.info()["n_fluid"]) for l in lattices]
    h = hashlib.sha256(json.dumps([dev, kind, desc]).encode()).hexdigest()[:20]
    return f"{kind}:{h}"


def _load(path: str) -> Dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path: str, key: str, value) -> None:
    data = _load(path)
    data[key] = value
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1)
    os.replace(tmp, path)


def _time(fn, steps: int) -> float:
    import torch
    stream = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    fn(4)  # capture graphs, warm caches
    torch.cuda.synchronize()
    a.record(stream)
    fn(steps)
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def tune_lattice(lat, steps: int = 64, tiles: Iterable[Tuple[int, int]] = TILES,
                 two_step: Iterable[Tuple[int, int]] = TWO_STEP, graph_chunk: int = 64,
                 use_cache: bool = True, path: Optional[str] = None) -> Dict:
    """Pick the single-step tile shape with the shortest step time, then the
    fastest of single steps and the two-step forms; applies both. steps
    should be a multiple of 4 (two-step passes come in pairs)."""
    path = path or cache_path()
    key = _key([lat], "lattice2")
    if use_cache:
        hit = _load(path).get(key)
        if hit:
            lat.set_launch(hit["tile"][0], hit["tile"][1], graph_chunk)
            lat.set_two_step(hit["fuse"], hit["rows"])
            return hit
    results: List[Dict] = []
    lat.set_two_step(1)
    for t in tiles:
        lat.set_launch(t[0], t[1], graph_chunk)
        results.append({"tile": list(t), "fuse": 1, "rows": 0,
                        "ms_per_step": _time(lat.step, steps)})
    best = min(results, key=lambda r: r["ms_per_step"])
    lat.set_launch(best["tile"][0], best["tile"][1], graph_chunk)
    for fuse, rows in two_step:
        try:
            lat.set_two_step(fuse, rows)
        except GGError:  # a form this lattice refuses (walking strips, see gg_set_two_step)
            continue
        results.append({"tile": best["tile"], "fuse": fuse, "rows": rows,
                        "ms_per_step": _time(lat.step, steps)})
    best = min(results, key=lambda r: r["ms_per_step"])
    lat.set_launch(best["tile"][0], best["tile"][1], graph_chunk)
    lat.set_two_step(best["fuse"], best["rows"] or 6)
    out = {"tile": best["tile"], "fuse": best["fuse"], "rows": best["rows"] or 6,
           "ms_per_step": best["ms_per_step"], "all": results}
    _store(path, key, out)
    return out


def tune_batch(lattices: Sequence, steps: int = 32, tiles: Iterable[Tuple[int, int]] = TILES,
               persist: Iterable[int] = PERSIST,
               two_step: Iterable[Tuple[int, int]] = ((4, 6), (4, 14), (3, 6), (3, 14)),
               graph_chunk: int = 64, use_cache: bool = True,
               path: Optional[str] = None) -> Dict:
    """Pick the launch form of a batch: single steps with a tile shape and a
    persistent grid size, or a two-step form (with the best tile shape for
    the single steps that align the parity). steps: a multiple of 4."""
    from .lattice import Batch
    path = path or cache_path()
    key = _key(lattices, "batch2")
    if use_cache:
        hit = _load(path).get(key)
        if hit:
            return hit
    results: List[Dict] = []
    for t in tiles:
        for p in persist:
            b = Batch(lattices, tile=t, persist=p, graph_chunk=graph_chunk)
            results.append({"tile": list(t), "persist": p, "fuse": 1, "rows": 6,
                            "ms_per_step": _time(b.step, steps)})
            b.close()
    single = min(results, key=lambda r: r["ms_per_step"])
    for fuse, rows in two_step:
        b = Batch(lattices, tile=tuple(single["tile"]), persist=single["persist"],
                  graph_chunk=graph_chunk, fuse=fuse, rows=rows)
        results.append({"tile": single["tile"], "persist": single["persist"], "fuse": fuse,
                        "rows": rows, "ms_per_step": _time(b.step, steps)})
        b.close()
    best = min(results, key=lambda r: r["ms_per_step"])
    out = {k: best[k] for k in ("tile", "persist", "fuse", "rows", "ms_per_step")}
    out["all"] = results
    _store(path, key, out)
    return out


def tune_cde(lat, steps: int = 256, rows: Iterable[int] = (0, 6, 14, -6, -10),
             use_cache: bool = True,
             path: Optional[str] = None) -> Dict:
    """Pick the launch form of the compound-only step (two-step passes over
    tiles of 6 or 14 rows, four-step passes over 58-column tiles of 6 or 10
    rows (rows -6, -10), or single steps) with the shortest step time and
    apply it. Needs a velocity field for every phase; advances the compound
    (steps should be a multiple of 8)."""
    path = path or cache_path()
    key = _key([lat], "cde4")
    if use_cache:
        hit = _load(path).get(key)
        if hit:
            lat.set_cde_launch(hit["rows"])
            return hit
    results: List[Dict] = []
    for r in rows:
        lat.set_cde_launch(r)
        results.append({"rows": r, "ms_per_step": _time(lat.cde_step, steps)})
    best = min(results, key=lambda x: x["ms_per_step"])
    lat.set_cde_launch(best["rows"])
    out = {"rows": best["rows"], "ms_per_step": best["ms_per_step"], "all": results}
    _store(path, key, out)
    return out
