"""Helpers shared by the GPU parity tests: device transfer and canonical
comparison against the oracle (filter output is compared as is; join pairs
sorted by (probe row, build row); groups sorted by key tuple)."""

from __future__ import annotations

import sys

import numpy as np
import torch


def announce(*parts):
    """Names the case about to run on the GPU, flushed before the GPU step."""
    print("[case]", *parts, flush=True)
    sys.stdout.flush()


def dev(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rowids(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def canon_pairs(ob: np.ndarray, op: np.ndarray):
    order = np.lexsort((ob, op))
    return ob[order], op[order]


def assert_pairs(got, want, what=""):
    gb, gp = canon_pairs(rowids(got[0]), rowids(got[1]))
    wb, wp = want
    assert len(gb) == len(wb), f"{what}: {len(gb)} pairs, oracle {len(wb)}"
    assert np.array_equal(gp, wp), f"{what}: probe ids differ"
    assert np.array_equal(gb, wb), f"{what}: build ids differ"


def canon_groups(keys, aggs):
    """Device group outputs -> host arrays sorted by key tuple (keys widened
    to int64, aggregates as int64 bit patterns)."""
    hk = [k.cpu().numpy().astype(np.int64) for k in keys]
    ha = [a.cpu().numpy().view(np.int64) for a in aggs]
    if hk:
        order = np.lexsort(hk[::-1])
        hk = [k[order] for k in hk]
        ha = [a[order] for a in ha]
    return hk, ha


def assert_groups(got, want, aggs, what=""):
    gk, ga = canon_groups(*got)
    wk, wa = want
    ng = len(wa[0])
    assert len(ga[0]) == ng, f"{what}: {len(ga[0])} groups, oracle {ng}"
    for k in range(len(wk)):
        assert np.array_equal(gk[k], wk[k]), f"{what}: key {k} differs"
    for a, (op, _) in enumerate(aggs):
        w = np.asarray(wa[a])
        w = w.view(np.int64) if w.dtype == np.float64 else w.astype(np.int64)
        if not np.array_equal(ga[a], w):
            bad = np.flatnonzero(ga[a] != w)[:5]
            raise AssertionError(f"{what}: {op} differs at groups {bad.tolist()}: "
                                 f"got {ga[a][bad].tolist()} oracle {w[bad].tolist()}")
