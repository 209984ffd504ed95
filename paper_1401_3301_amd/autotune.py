"""Autotuner for the batched assembly.

Times ``fem_batch_numeric`` for each candidate -- the vertex-pair kernel with
a given layout (rows per vertex block of the 3D and of the 2D meshes, tasks
of 64 pairs per wavefront; the layouts are rebuilt for each) in one launch
over both dimensions or one launch per dimension, or the
persistent row-gather kernel with a given number of threads per workgroup
and workgroups per compute unit -- with HIP events on the current stream and
keeps the fastest.  The candidates differ only in how the work is scheduled,
never in the values (every CSR entry is summed in ascending element number
with the same expressions), so any choice gives bitwise-identical output.
Results are cached in a JSON file keyed by GPU architecture, operator and a
size signature of the batch.
"""
from __future__ import annotations

import json
import os
import statistics

import torch

from . import femasm

PAIR_ROWS_3D = {"scalar": (48, 64, 72), "elas": (48, 56, 64)}


def candidates(op: str):
    kind = "elas" if op == "ELAS" else "scalar"
    layouts = [(r3, 128, s) for r3 in PAIR_ROWS_3D[kind] for s in (1, 2)]
    layouts.append((PAIR_ROWS_3D[kind][1], 96, 2))
    # per layout: one launch over both dimensions, or one per dimension
    pair = [(k,) + lay for lay in layouts for k in ("pair", "pair_split")]
    return pair + [("rowgather", bt, w) for bt, w in ((256, 1), (256, 2), (128, 4))]


def _key(params):
    return params[0] + ":" + "x".join(str(x) for x in params[1:])


def default_cache_path() -> str:
    return os.environ.get("FEMASM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "femasm_autotune.json"))


def batch_key(batch: femasm.Batch, op: str) -> str:
    arch = torch.cuda.get_device_properties(batch.device).gcnArchName.split(":")[0]
    nel = sum(batch.nme)
    bucket = 1 << max(0, int(nel).bit_length() - 1)
    d2 = sum(1 for d in batch.d if d == 2)
    return f"{arch}|{op}|n{len(batch)}|d2:{d2}|el~{bucket}"


def _time(batch, op, q_cat, w_cat, out, reps):
    stream = torch.cuda.current_stream()
    for _ in range(2):
        batch.numeric(op, q_cat, w_cat, out=out)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        batch.numeric(op, q_cat, w_cat, out=out)
        b.record(stream)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def tune(batch: femasm.Batch, op: str, q_cat, w_cat=None, reps: int = 5,
         cache_path: str | None = None, force: bool = False):
    """Pick and apply the fastest (kernel, block_threads, wg_per_cu) for this
    batch and operator.  Returns (params, {params: ms})."""
    cache_path = cache_path or default_cache_path()
    key = batch_key(batch, op)
    cache = {}
    if os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    if not force and key in cache and tuple(cache[key]["params"]) in candidates(op):
        params = tuple(cache[key]["params"])
        batch.configure(params, op)
        return params, cache[key].get("times", {})
    nnz = batch.offsets(op).nnz[-1]
    out = torch.empty(max(nnz, 1), dtype=torch.float64, device=batch.device)
    times = {}
    for cand in candidates(op):
        try:
            batch.configure(cand, op)
        except femasm.FemError:
            continue
        times[_key(cand)] = _time(batch, op, q_cat, w_cat, out, reps)
    best = min(times, key=times.get)
    kern, rest = best.split(":")   # e.g. "pair_split:64x128x2"
    params = (kern,) + tuple(int(x) for x in rest.split("x"))
    batch.configure(params, op)
    cache[key] = {"params": list(params), "times": times}
    os.makedirs(os.path.dirname(cache_path) or ".", exist_ok=True)
    tmp = cache_path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, cache_path)
    return params, times
