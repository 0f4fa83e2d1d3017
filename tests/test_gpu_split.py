"""GPU parity of the forward step (stable multi-split) against the oracle.

Bit-exact on the permuted items, the per-destination offsets and the
done/bad counts, over small and ragged sizes, many item sizes and domain
counts, the 64M-item x 32-byte uniform and Zipf workloads, and through the
context's round API (debug poison, bad destinations).
"""
import numpy as np
import pytest
import torch

from gpu_util import announce, device
from paper_2605_30294_amd import rafi
from paper_2605_30294_amd import workloads as W

pytestmark = pytest.mark.gpu


def _run_split(orc, n, D, words, seed, dist="mixed"):
    dev = device()
    rng = np.random.default_rng(seed)
    if dist == "mixed":
        dest = rng.integers(-2, D + 1, n).astype(np.int32)        # done, bad and valid
    elif dist == "cyclic":
        dest = (np.arange(n) % D).astype(np.int32)                # every destination in every chunk
    else:
        dest = W.split_dest(n, D, dist, seed=seed)
    items = rng.integers(0, 2**32, (n, words), dtype=np.uint64).astype(np.uint32)
    announce(f"split n={n} D={D} S={4 * words} dist={dist}")
    out, offsets, summary = rafi.multisplit(torch.from_numpy(items.view(np.int32)).to(dev),
                                            torch.from_numpy(dest).to(dev), D)
    torch.cuda.synchronize()
    e_out, e_counts, e_off, e_done, e_bad = orc.multisplit(items, dest, D)
    total = int(e_off[-1])
    s = summary.cpu().numpy()
    assert s[0] == total and s[1] == e_done and s[2] == e_bad
    assert np.array_equal(offsets.cpu().numpy().astype(np.uint64), e_off)
    assert np.array_equal(out[:total].cpu().numpy().view(np.uint32), e_out)


@pytest.mark.parametrize("n,D,words", [
    (0, 4, 4), (1, 1, 4), (3, 2, 1), (1000, 8, 4), (5000, 64, 8), (1023, 3, 11), (4097, 1024, 8),
    (70001, 1024, 4), (100_000, 8192, 2), (65536 + 17, 17, 64), (250_000, 64, 3), (33_333, 5, 6),
    (200_000, 1, 8), (131_072, 2048, 12),
])
def test_split_matches_oracle(orc, n, D, words):
    _run_split(orc, n, D, words, seed=n * 7 + D)


@pytest.mark.parametrize("dist", ["uniform", "zipf"])
def test_split_full_size(orc, dist):
    """The 64M x 32-byte microbenchmark, 1024 destinations."""
    dev = device()
    n, D = 1 << 26, 1024
    dest = W.split_dest(n, D, dist)
    items = W.split_items(n)
    announce(f"split full size {dist}")
    d_items = torch.from_numpy(items.view(np.int32)).to(dev)
    d_dest = torch.from_numpy(dest).to(dev)
    out, offsets, summary = rafi.multisplit(d_items, d_dest, D)
    out2, offsets2, _ = rafi.multisplit(d_items, d_dest, D)      # determinism
    torch.cuda.synchronize()
    assert torch.equal(out, out2) and torch.equal(offsets, offsets2)
    e_out, e_counts, e_off, e_done, e_bad = orc.multisplit(items, dest, D)
    assert np.array_equal(offsets.cpu().numpy().astype(np.uint64), e_off)
    assert int(summary[0]) == n and int(summary[1]) == 0 and int(summary[2]) == 0
    assert np.array_equal(out.cpu().numpy().view(np.uint32), e_out)


def test_context_round_and_error_paths(orc):
    dev = device()
    D, S, cap = 16, 16, 10_000
    ctx = rafi.Context(D, S, cap, debug=True)
    ctx.begin(5000)
    # bulk emission from device arrays stands in for a generator kernel
    rng = np.random.default_rng(3)
    items = rng.integers(0, 2**31, (5000, 4)).astype(np.int32)
    dest = rng.integers(-1, D, 5000).astype(np.int32)
    dest[4000:] = rafi.RAFI_POISON                   # slots a "kernel" never wrote
    t_items = torch.from_numpy(items).to(dev)
    t_dest = torch.from_numpy(dest[:4000]).to(dev)
    ctx.emit_bulk(t_items[:4000], t_dest)             # slots 4000.. stay poisoned
    counts, total, rc = ctx.round(allow=(rafi.RAFI_OK, rafi.ERR_BAD_DEST))
    assert rc == rafi.ERR_BAD_DEST                    # 1000 poisoned slots counted as bad
    e_out, e_counts, e_off, e_done, e_bad = orc.multisplit(items, dest, D)
    assert total == int(e_off[-1]) and np.array_equal(counts, e_counts)
    q, offs = ctx.copy_queue()
    assert np.array_equal(q.cpu().numpy().view(np.int32).reshape(-1, 4), e_out.reshape(-1, 4))
    assert np.array_equal(offs, e_off)
    st = ctx.stats()
    assert st["bad_dest"] == 1000 and st["done"] == e_done and st["rounds"] == 1
    ctx.close()


@pytest.mark.parametrize("variant", list(range(1, 16)))
@pytest.mark.parametrize("n,D,words", [(300_001, 1024, 8), (200_003, 64, 4), (77_777, 1000, 8), (150_000, 7, 4)])
def test_split_shapes_identical(orc, variant, n, D, words):
    """Every workgroup shape of the staged scatter gives the oracle's bytes."""
    try:
        rafi.split_set_variant(variant)
        _run_split(orc, n, D, words, seed=variant * 1000 + n)
    finally:
        rafi.split_set_variant(0)


@pytest.mark.parametrize("variant", [0, 12, 14, 15])
@pytest.mark.parametrize("n,D,words,dist", [
    (1_000_003, 64, 8, "mixed"), (2_500_000, 1024, 8, "mixed"), (600_000, 1024, 4, "mixed"),
    (4_096_000, 1024, 8, "cyclic"), (3_072_005, 1024, 4, "cyclic"), (2_000_000, 1000, 8, "zipf")])
def test_split_line_aligned_shapes(orc, variant, n, D, words, dist):
    """Sizes where one workgroup of the line-aligned shapes spans several
    histogram tiles, and cyclic destinations, which leave more unfinished
    lines after a chunk than the stage keeps (those are written at once)."""
    try:
        rafi.split_set_variant(variant)
        _run_split(orc, n, D, words, seed=variant * 1000 + n + 1, dist=dist)
    finally:
        rafi.split_set_variant(0)


def _run_ctx_split(orc, n, D, words, seed, dist="mixed"):
    """The same split through a context's round (item buffers padded by the
    library, so the raw-staged shape also takes lengths that are not whole
    16-byte pieces)."""
    dev = device()
    rng = np.random.default_rng(seed)
    if dist == "mixed":
        dest = rng.integers(-1, D, n).astype(np.int32)
    elif dist == "cyclic":
        dest = (np.arange(n) % D).astype(np.int32)
    else:
        dest = W.split_dest(n, D, dist, seed=seed)
    items = rng.integers(0, 2**32, (n, words), dtype=np.uint64).astype(np.uint32)
    announce(f"context split n={n} D={D} S={4 * words} dist={dist}")
    ctx = rafi.Context(D, 4 * words, n)
    try:
        ctx.begin(n)
        ctx.emit_bulk(torch.from_numpy(items.view(np.int32)).to(dev), torch.from_numpy(dest).to(dev))
        counts, total, rc = ctx.round()
        q, offs = ctx.copy_queue()
        e_out, e_counts, e_off, e_done, e_bad = orc.multisplit(items, dest, D)
        assert total == int(e_off[-1]) and np.array_equal(counts, e_counts)
        assert np.array_equal(offs, e_off)
        assert np.array_equal(q.cpu().numpy().view(np.uint32).reshape(-1), e_out.reshape(-1))
    finally:
        ctx.close()


@pytest.mark.parametrize("variant", [0, 16])
@pytest.mark.parametrize("n,D,words,dist", [
    (1_000_000, 1024, 11, "mixed"), (1_000_003, 1024, 11, "mixed"), (600_000, 64, 10, "zipf"),
    (524_288, 1000, 6, "cyclic"), (300_000, 1024, 3, "mixed"), (2_000_000, 1024, 11, "cyclic"),
    (70_000, 16, 11, "mixed")])
def test_split_raw_staged_shape(orc, variant, n, D, words, dist):
    """Item sizes that are not a multiple of 16 bytes (12, 24, 40, 44 bytes):
    the raw-staged shape (chunk bytes in LDS in load order, 4-byte words
    out), automatic or forced, through the stateless split (which keeps the
    staged shapes when the array is not a whole number of 16-byte pieces)
    and through a context."""
    try:
        rafi.split_set_variant(variant)
        _run_split(orc, n, D, words, seed=variant * 1000 + n + 2, dist=dist)
        _run_ctx_split(orc, n, D, words, seed=variant * 1000 + n + 3, dist=dist)
    finally:
        rafi.split_set_variant(0)


@pytest.mark.parametrize("n,D,words", [
    (16_777_216, 64, 4), (16_777_220, 64, 4),      # 16-byte items: shape 4 up to 2^28 bytes
    (8_388_608, 128, 8), (8_388_612, 128, 8),      # 32-byte items: shape 2 up to 2^28 bytes
    (1_525_201, 64, 11), (1_525_204, 64, 11),      # 44-byte items: plain scatter up to 2^26 bytes
    (1_398_101, 64, 12), (1_398_104, 64, 12),      # 48-byte items
])
def test_split_automatic_shape_boundaries(orc, n, D, words):
    """The automatic scatter shape for few destinations changes with the
    array's size (small staged shapes or the plain per-thread scatter up
    to a bound, the usual choice above): both sides of each bound, through
    the stateless split, against the oracle."""
    _run_split(orc, n, D, words, seed=n + D + 7, dist="mixed")


@pytest.mark.parametrize("variant", [0, 17])
@pytest.mark.parametrize("n,D,words,dist", [
    (2_097_152, 1024, 11, "mixed"), (2_500_003, 1024, 11, "mixed"), (3_000_000, 1000, 10, "zipf"),
    (4_194_308, 64, 6, "cyclic"), (2_200_001, 1024, 3, "mixed"), (2_100_000, 1, 11, "mixed")])
def test_split_lockstep_shape(orc, variant, n, D, words, dist):
    """Large splits of items that are not whole 16-byte pieces: the lockstep
    schedule (tiles of 32 chunks of 2048 slots, each chunk's run bases from
    its tile's column plus the histogram pass's per-chunk prefixes, 256
    persistent workgroups), automatic or forced. Through the stateless split
    (which falls back to the staged shapes, on the lockstep plan's table,
    when the array is not a whole number of 16-byte pieces) and a context;
    ragged last chunks and tiles; 1 to 1024 destinations."""
    try:
        rafi.split_set_variant(variant)
        _run_split(orc, n, D, words, seed=variant * 1000 + n + 4, dist=dist)
        _run_ctx_split(orc, n, D, words, seed=variant * 1000 + n + 5, dist=dist)
    finally:
        rafi.split_set_variant(0)


def test_split_lockstep_workspace_fallback(orc):
    """A workspace sized while another scatter shape was selected lacks the
    lockstep plan's chunk prefixes: the stateless split then plans without
    them instead of failing, with the same result."""
    dev = device()
    n, D, words = 2_097_152, 1024, 11
    try:
        rafi.split_set_variant(16)
        small = rafi.multisplit_workspace(n, D, 4 * words)
    finally:
        rafi.split_set_variant(0)
    assert rafi.multisplit_workspace(n, D, 4 * words) > small
    rng = np.random.default_rng(11)
    dest = rng.integers(-1, D, n).astype(np.int32)
    items = rng.integers(0, 2**32, (n, words), dtype=np.uint64).astype(np.uint32)
    announce("split lockstep workspace fallback")
    d_items = torch.from_numpy(items.view(np.int32)).to(dev)
    d_dest = torch.from_numpy(dest).to(dev)
    out = torch.empty_like(d_items)
    offsets = torch.empty(D + 1, dtype=torch.int64, device=dev)
    summary = torch.empty(4, dtype=torch.int64, device=dev)
    ws = torch.empty(small, dtype=torch.uint8, device=dev)
    rc = rafi.lib().rafi_multisplit(rafi._dptr(d_items), rafi._dptr(d_dest), n, 4 * words, D, rafi._dptr(out),
                                    rafi._dptr(offsets), rafi._dptr(summary), rafi._dptr(ws), small, None)
    assert rc == 0
    torch.cuda.synchronize()
    e_out, e_counts, e_off, e_done, e_bad = orc.multisplit(items, dest, D)
    total = int(e_off[-1])
    assert np.array_equal(offsets.cpu().numpy().astype(np.uint64), e_off)
    assert int(summary[0]) == total and int(summary[1]) == e_done
    assert np.array_equal(out[:total].cpu().numpy().view(np.uint32), e_out)


@pytest.mark.parametrize("dist", ["uniform", "zipf"])
def test_split_full_size_44_bytes(orc, dist):
    """The microbenchmark at the paper's 44-byte ray size: 64M items, 1024
    destinations (the lockstep schedule)."""
    dev = device()
    n, D = 1 << 26, 1024
    dest = W.split_dest(n, D, dist)
    items = W.split_items(n, 11)
    announce(f"split full size 44 B {dist}")
    out, offsets, summary = rafi.multisplit(torch.from_numpy(items.view(np.int32)).to(dev),
                                            torch.from_numpy(dest).to(dev), D)
    torch.cuda.synchronize()
    e_out, e_counts, e_off, e_done, e_bad = orc.multisplit(items, dest, D)
    assert np.array_equal(offsets.cpu().numpy().astype(np.uint64), e_off)
    assert int(summary[0]) == n and int(summary[1]) == 0 and int(summary[2]) == 0
    assert np.array_equal(out.cpu().numpy().view(np.uint32), e_out)
