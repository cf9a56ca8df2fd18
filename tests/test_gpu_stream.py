"""rel_stream_read, the streaming-read ceiling kernel: every byte read once.
Checked against the XOR of the buffer's zero-padded little-endian 64-bit
words computed on the host, over sizes around the 16-byte load width, a
grid-stride step and several full sweeps."""

import numpy as np
import pytest
import torch

from gpu_helpers import announce
from paper_2508_04701_amd import rel

pytestmark = pytest.mark.gpu


def host_xor(b: np.ndarray) -> int:
    pad = (-len(b)) % 8
    w = np.concatenate([b, np.zeros(pad, np.uint8)]).view(np.uint64)
    return int(np.bitwise_xor.reduce(w)) if len(w) else 0


@pytest.mark.parametrize("n", [0, 1, 7, 8, 15, 16, 17, 31, 4095, 4096 * 256 * 4 + 24,
                               1_000_003, 64 << 20])
def test_stream_read_xor(n):
    announce("stream_read", n)
    rng = np.random.default_rng(n)
    b = rng.integers(0, 256, size=n, dtype=np.uint8)
    t = torch.from_numpy(b).cuda()
    assert rel.stream_read(t) == host_xor(b)


def test_stream_read_rejects_misaligned():
    t = torch.zeros(64, dtype=torch.uint8, device="cuda")
    d = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(rel.RelError):
        rel.stream_read_async(t[1:], d)
