"""The rate probes that bench.py times for its measured peaks do exactly the
work they claim: the copy probe copies, and the VALU probe's chains end at
the values a plain Python loop gives."""
import numpy as np
import pytest
import torch

import paper_2604_27058_amd as pk

pytestmark = pytest.mark.gpu


def test_copy_probe_copies():
    n = (1 << 20) + 48  # a ragged tail of 16-byte elements beyond the grid
    src = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    pk.probe(0, dst, src, n, 7)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)


def test_read_probe_reads():
    grid, n = 5, (1 << 20) + 32
    src = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros(grid * 256 * 16, dtype=torch.uint8, device="cuda")
    pk.probe(2, dst, src, n, grid)
    torch.cuda.synchronize()
    words = src.cpu().numpy().view(np.uint32).reshape(-1, 4)
    out = dst.cpu().numpy().view(np.uint32).reshape(-1, 4)
    T = grid * 256
    for t in (0, 1, T - 1):
        ref = np.bitwise_xor.reduce(words[t::T], axis=0)
        assert np.array_equal(out[t], ref), t


def test_valu_probe_chains():
    grid, iters = 3, 37
    dst = torch.zeros(grid * 256, dtype=torch.int32, device="cuda")
    pk.probe(1, dst, None, iters, grid)
    torch.cuda.synchronize()
    out = dst.cpu().numpy().view(np.uint32)
    c = 0x9E3779B9
    for g in (0, 1, 255, 256, grid * 256 - 1):
        acc = 0
        for j in range(8):
            a = g * 8 + j
            for _ in range(iters):
                a = ((a ^ c) + c) & 0xFFFFFFFF
            acc ^= a
        assert int(out[g]) == acc, g


def test_probe_rejects_bad_arguments():
    # sized for one workgroup's outputs, so that no call here could write
    # beyond it even if it were accepted
    x = torch.zeros(256 * 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(pk.ClifftError):
        pk.probe(0, x, x, 63, 1)
    with pytest.raises(pk.ClifftError):
        pk.probe(2, x, x, 17, 1)
    with pytest.raises(pk.ClifftError):
        pk.probe(3, x, x, 16, 1)
