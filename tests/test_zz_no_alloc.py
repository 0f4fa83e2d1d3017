"""The no-allocation stateless split (rafi_multisplit_noalloc) against the
allocating one (rafi_multisplit), bit-exact, on two calls in a row: the
second smaller, so it runs on the scratch buffer the first one left."""
import numpy as np
import pytest
import torch

from gpu_util import announce, device
from paper_2605_30294_amd import rafi

pytestmark = pytest.mark.gpu


def _case(n, D, words, seed):
    rng = np.random.default_rng(seed)
    dest = rng.integers(0, D, n).astype(np.int32)
    dest[rng.random(n) < 0.05] = -1           # done
    dest[rng.random(n) < 0.01] = D + 7        # invalid: dropped and counted
    items = rng.integers(0, 2**31, (n, words)).astype(np.int32)
    return items, dest


def _check_pair(n, D, words, seed):
    dev = device()
    announce(f"no-alloc split n={n} D={D} S={4 * words}")
    items_h, dest_h = _case(n, D, words, seed)
    items = torch.from_numpy(items_h).to(dev)
    dest = torch.from_numpy(dest_h).to(dev)
    ref_out, ref_off, ref_sum = rafi.multisplit(items, dest, D)
    out = torch.full_like(items, -3)
    off = torch.full((D + 1,), -3, dtype=torch.int64, device=dev)
    summ = torch.full((4,), -3, dtype=torch.int64, device=dev)
    rafi.multisplit_noalloc(items, dest, D, out, off, summ)
    torch.cuda.synchronize()
    total = int(ref_off[-1])
    assert np.array_equal(off.cpu().numpy(), ref_off.cpu().numpy())
    assert np.array_equal(summ.cpu().numpy(), ref_sum.cpu().numpy())
    assert np.array_equal(out[:total].cpu().numpy(), ref_out[:total].cpu().numpy())
    s = summ.cpu().numpy()
    assert s[0] == total and s[0] + s[1] + s[2] == n and s[2] > 0


def test_noalloc_split_matches_allocating_split_twice():
    # first: 3M x 32-byte items over 1024 destinations (many tiles, ragged tail)
    _check_pair(3_000_001, 1024, 8, seed=71)
    # second, smaller: 70K x 16-byte items over 64 destinations
    _check_pair(70_001, 64, 4, seed=72)


def test_noalloc_split_rejects_too_large():
    dev = device()
    items = torch.zeros((16, 8), dtype=torch.int32, device=dev)
    dest = torch.zeros(16, dtype=torch.int32, device=dev)
    out = torch.empty_like(items)
    off = torch.empty(4097, dtype=torch.int64, device=dev)
    summ = torch.empty(4, dtype=torch.int64, device=dev)
    L = rafi.lib()
    # 2^26 slots over 4096 destinations need a 63 MB count table: refused before any access
    rc = L.rafi_multisplit_noalloc(rafi._dptr(items), rafi._dptr(dest), 1 << 26, 32, 4096, rafi._dptr(out),
                                   rafi._dptr(off), rafi._dptr(summ), None)
    assert rc == rafi.ERR_TOO_LARGE
