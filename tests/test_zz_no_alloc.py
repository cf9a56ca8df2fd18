"""rel_filter_noalloc (tile states in the library's static device scratch)
against rel_filter (caller's workspace) through the C-ABI: two calls in a
row on the same GPU, the second over fewer rows, so that state left by the
first call must not leak into the second."""

import numpy as np
import pytest
import torch

from gpu_helpers import announce
from paper_2508_04701_amd import datagen, rel

pytestmark = pytest.mark.gpu


def run_both(cols, preds):
    n = cols[0].numel()
    a = torch.full((max(1, n),), -1, dtype=torch.int32, device="cuda")
    b = torch.full((max(1, n),), -1, dtype=torch.int32, device="cuda")
    ca = torch.zeros(1, dtype=torch.int64, device="cuda")
    cb = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    ws = rel.workspace(rel.filter_ws(n))
    rel.filter_async(cols, preds, a, ca, ws)
    rel.filter_noalloc_async(cols, preds, b, cb)
    torch.cuda.synchronize()
    k = int(ca.item())
    assert int(cb.item()) == k
    assert torch.equal(a[:k], b[:k])
    return k


@pytest.mark.parametrize("sizes", [(3_000_017, 100_003), (50_000_000, 8193)])
def test_filter_noalloc_matches_filter_twice(sizes):
    for i, n in enumerate(sizes):
        announce("filter_noalloc", n, "call", i)
        date = torch.from_numpy(datagen.uniform(datagen.SEED0 + 9, 12 + i, 0, 2557, n,
                                                np.int32)).cuda()
        price = torch.from_numpy(datagen.uniform(datagen.SEED0 + 9, 13 + i, 100, 10_000_000, n,
                                                 np.int64)).cuda()
        k = run_both([date, price], [(0, "lt", 767), (1, "ge", 5_000_000)])
        assert 0 < k < n


def test_filter_noalloc_empty_then_nonempty():
    announce("filter_noalloc empty then 5000 rows")
    empty = torch.empty(0, dtype=torch.int32, device="cuda")
    assert run_both([empty], [(0, "lt", 10)]) == 0
    x = torch.arange(5000, dtype=torch.int32, device="cuda")
    assert run_both([x], [(0, "range", 100, 4000)]) == 3900
