"""Tile- and launch-shape autotuner for the batched Gauss-Newton step.

The batched kernels are persistent loops over the (pair, block) work items of all pairs.
Two kinds of shape decide how well the uneven work is balanced and how much each compute
unit overlaps: the brick tile of the brick passes (16 x 4 x cells_z cells, cells_z 4 or 2:
half-depth bricks double the work items, which helps batches of small pairs), and how many
workgroups per compute unit each kind of pass gets (brick passes, node passes, vector
passes).  The tuner times whole batched steps on scratch copies of the displacement fields
(hipEvents on the current stream): first the tile with the default launch shapes, then the
three launch shapes in turn (coordinate descent over a small candidate set).  It caches the
winners in a JSON file keyed by the batch's shapes, storage, step sizes and the GPU
architecture, so that later batches of the same kind reuse them without timing.
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Optional, Sequence

import torch

from .disco import Batch, Disco, Params

# key of the brick tile (cells per brick along z) in a choice; the pass kinds are 0..2
TILE = 3
# 0: one workgroup per work item; n > 0: a persistent grid of n workgroups per compute unit
CANDIDATES = {Batch.PASS_BRICK: (0, 1, 2, 3, 4), Batch.PASS_NODE: (0, 2, 4, 8, 16), Batch.PASS_VEC: (0, 2, 4, 8, 16),
              TILE: (4, 2)}
DEFAULT = {Batch.PASS_BRICK: 4, Batch.PASS_NODE: 8, Batch.PASS_VEC: 8, TILE: 4}


def batch_key(ctxs: Sequence[Disco], params: Sequence[Params]) -> str:
    arch = torch.cuda.get_device_properties(ctxs[0].device).gcnArchName.split(":")[0]
    shapes = sorted(f"{c.shape[0]}x{c.shape[1]}x{c.shape[2]}" for c in ctxs)
    counts: Dict[str, int] = {}
    for s in shapes:
        counts[s] = counts.get(s, 0) + 1
    shp = ",".join(f"{k}*{v}" for k, v in sorted(counts.items()))
    st = "fp16" if ctxs[0].storage else "fp32"
    p = params[0]
    # "tiles": the entry holds a brick tile as well as launch shapes
    return f"{arch}|{st}|{shp}|pcg{p.pcg_iters}|ls{p.ls_max}|tiles"


def _time_steps(batch: Batch, reps: int) -> float:
    batch.gn_step()  # warm
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        batch.gn_step()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(ctxs: Sequence[Disco], params: Sequence[Params], us: Sequence[torch.Tensor], reps: int = 2,
         cache: Optional[str] = None, log=None) -> Dict[int, int]:
    """Best brick tile (key TILE) and workgroups-per-CU for each pass kind (keys 0..2);
    reads/writes `cache` (JSON) if given.  The displacement fields `us` are not modified
    (the timing runs on copies)."""
    key = batch_key(ctxs, params)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if key in table:
            return {int(k): int(v) for k, v in table[key].items()}
    scratch = [u.clone() for u in us]
    batch = Batch(ctxs)
    batch.prepare(params, scratch)
    best = dict(DEFAULT)
    apply(batch, best)
    for kind in (TILE, Batch.PASS_BRICK, Batch.PASS_NODE, Batch.PASS_VEC):
        timings: List = []
        for w in CANDIDATES[kind]:
            apply(batch, {kind: w})
            for u, a in zip(scratch, us):
                u.copy_(a)
            ms = _time_steps(batch, reps)
            timings.append((ms, w))
            if log:
                log(f"[autotune] {'tile cells_z' if kind == TILE else f'pass {kind} wg/CU'} {w}: {ms:.3f} ms/step")
        best[kind] = min(timings)[1]
        apply(batch, {kind: best[kind]})
    batch.close()
    if cache:
        table = {}
        if os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        table[key] = {str(k): v for k, v in best.items()}
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return best


def apply(batch: Batch, choice: Dict[int, int]):
    """Set the tile (a prepared batch is prepared again) and the launch shapes of a choice."""
    for k, w in choice.items():
        if k == TILE:
            batch.set_tile(w)
        else:
            batch.set_launch(k, w)
