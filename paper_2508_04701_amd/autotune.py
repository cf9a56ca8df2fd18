"""Autotuner: per size bucket, the tuning record with the lowest measured
device time among candidates that all return identical results (any
difference is a race and raises). Batched plans are tuned natively by
rel_autotune (tune_batch_plans here): the candidates vary the global
group-table replicas, the LDS group table (off, 1024 or 4096 slots: the
workgroup's LDS shape, which sets how many workgroups share a CU), the
group-table load factor, the fan-out of an instance over the persistent
workgroups (fact tiles per work item), the block shape (one or two
workgroups per CU) and the spilled-row records (none, or 16 or 256
partitions); rel_autotune_lookup reads a record back (lookup here).
For the standalone group-by (tune_groupby) the candidates vary the partition
fan-out (single pass, automatic, 2048 to 16384 partitions) and the first
scatter's LDS table. Records persist as JSON keyed by (GPU architecture,
operation, size bucket) and are applied per plan, also to each instance of a
batch.

A bucket is the magnitude (in steps of 4x) of the fact rows, the largest dim
and the group bound: plans within a bucket share the behaviour the knobs trade off
(how many rows reach the group table, whether the groups fit the LDS
table, how many hot lines the global atomics meet).
"""

from __future__ import annotations

import json
import math
import os

import numpy as np
import torch

from . import rel

CANDIDATES = [
    {},
    {"replicas": 1},
    {"replicas": 8},
    {"replicas": 32},
    {"replicas": 64},
    {"lds_slots": -1, "replicas": 32},
    {"load_factor": 0.3},
    {"load_factor": 0.3, "replicas": 32},
    {"lds_slots": 1024},
    {"lds_slots": 4096},
]

# rel_groupby_agg: partitions of the radix-partitioned aggregation (-1: one
# pass over the global table; 0: from the group bound) and the first
# scatter's LDS table.
GROUPBY_CANDIDATES = [
    {},
    {"fanout": -1},
    {"fanout": 2048},
    {"fanout": 8192},
    {"fanout": 16384},
    {"lds_slots": -1},
]

FIELDS = ("load_factor", "lds_slots", "replicas", "chunk_tiles", "dim_lds_bytes", "grid", "fanout")


def arch() -> str:
    if not torch.cuda.is_available():
        return "none"
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _mag(x: int) -> int:
    return 0 if x <= 1 else int(math.ceil(math.log2(x)))


def bucket(n_fact: int, n_dim: int, max_groups: int) -> str:
    """Magnitudes in steps of 4x: f/d/g name the even exponent at or below
    the ceiling log2 of each size."""
    step = lambda x: 2 * (_mag(x) // 2)  # noqa: E731
    return f"f{step(n_fact)}-d{step(n_dim)}-g{step(max_groups)}"


def cache_key(op: str, b: str, gpu: str | None = None) -> str:
    return f"{gpu or arch()}/{op}/{b}"


class Cache:
    """Tuning records: {key: {"tuning": {field: value}, "ms": best time,
    "candidates": {candidate: ms}}}."""

    def __init__(self, path: str | None = None):
        self.path = path
        self.records = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.records = json.load(f)

    def get(self, key: str):
        r = self.records.get(key)
        return None if r is None else r["tuning"]

    def put(self, key: str, record: dict):
        self.records[key] = record

    def save(self, path: str | None = None):
        path = path or self.path
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.records, f, indent=1, sort_keys=True)
        os.replace(tmp, path)


def to_tuning(fields: dict | None) -> rel.Tuning | None:
    if not fields:
        return None
    unknown = set(fields) - set(FIELDS)
    if unknown:
        raise ValueError(f"unknown tuning fields {sorted(unknown)}")
    return rel.tuning(**fields)


def _canon(keys, aggs):
    hk = [k.cpu().numpy().astype(np.int64) for k in keys]
    ha = [a.cpu().numpy().view(np.int64) for a in aggs]
    if hk:
        order = np.lexsort(hk[::-1])
        hk = [k[order] for k in hk]
        ha = [a[order] for a in ha]
    return hk + ha


def tune_plan(make, candidates=CANDIDATES, reps: int = 3) -> dict:
    """make(tuning) -> rel.PreparedPipeline. Times every candidate (after one
    warm launch) with events on the current stream and checks that all return
    the same groups. Returns {"tuning", "ms", "candidates"}."""
    stream = torch.cuda.current_stream()
    times, ref = {}, None
    for cand in candidates:
        plan = make(to_tuning(cand))
        plan.launch()
        got = _canon(*plan.result())
        if ref is None:
            ref = got
        elif len(got) != len(ref) or not all(np.array_equal(a, b) for a, b in zip(got, ref)):
            raise RuntimeError(f"tuning candidate {cand} changed the result: a race")
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(reps):
            plan.launch()
        stop.record(stream)
        stop.synchronize()
        times[json.dumps(cand, sort_keys=True)] = start.elapsed_time(stop) / reps
        del plan
    best = min(times, key=times.get)
    return {"tuning": json.loads(best), "ms": times[best], "candidates": times}


class GroupByCall:
    """rel_groupby_agg on fixed inputs with its own workspace and outputs, in
    the launch()/result() form that tune_plan times."""

    def __init__(self, keys, vals, aggs, max_groups: int, t=None):
        self.keys, self.vals, self.aggs, self.max_groups, self.t = keys, vals, aggs, max_groups, t
        dev = (keys or vals)[0].device
        n = (keys or vals)[0].numel()
        self.ws = rel.workspace(rel.groupby_ws([k.dtype for k in keys], aggs, n, max_groups, t), dev)
        cap = max(1, min(max_groups, n))
        self.out_keys, self.out_aggs = rel._out_tensors([k.dtype for k in keys], aggs, cap, dev)
        self.count = torch.zeros(1, dtype=torch.int64, device=dev)

    def launch(self):
        rel.groupby_agg_async(self.keys, self.vals, self.aggs, self.out_keys, self.out_aggs,
                              self.count, self.max_groups, self.ws, t=self.t)

    def result(self):
        n = int(self.count.item())
        if n < 0 or n > self.out_aggs[0].numel():
            raise RuntimeError(f"group-by produced {n} groups for a bound of {self.max_groups}")
        return [k[:n] for k in self.out_keys], [a[:n] for a in self.out_aggs]


def tune_groupby(keys, vals, aggs, max_groups: int, candidates=GROUPBY_CANDIDATES,
                 reps: int = 3) -> dict:
    """tune_plan over rel_groupby_agg records for these inputs."""
    return tune_plan(lambda t: GroupByCall(keys, vals, aggs, max_groups, t), candidates, reps)


def plan_bucket(n_fact: int, dim_rows: list, max_groups: int) -> str:
    return bucket(n_fact, max(dim_rows) if dim_rows else 0, max_groups)


def tuning_for(cache: Cache, op: str, n_fact: int, dim_rows: list, max_groups: int):
    """The cached record of the plan's bucket as a rel.Tuning (None: defaults)."""
    return to_tuning(cache.get(cache_key(op, plan_bucket(n_fact, dim_rows, max_groups))))


# ----------------------------------------------------------- batched plans

def tune_batch_plans(plans, cache_path: str) -> None:
    """rel_autotune over the plans (rel.Plan, one representative per size
    bucket): times every candidate as a one-plan batch on the GPU and stores
    the fastest record of each bucket in the JSON file at cache_path."""
    descs = (rel.PipelineDesc * len(plans))(*[p.desc for p in plans])
    rel._check(rel.lib().rel_autotune(descs, len(plans), cache_path.encode()))


def lookup(cache_path: str, plan) -> rel.Tuning | None:
    """The record rel_autotune stored for the plan's bucket (None: none)."""
    t = rel.Tuning()
    found = rel.ctypes.c_int(0)
    rel._check(rel.lib().rel_autotune_lookup(cache_path.encode(), rel.ctypes.byref(plan.desc),
                                             rel.ctypes.byref(t), rel.ctypes.byref(found)))
    return t if found.value else None
