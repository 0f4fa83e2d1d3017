"""Pins for the oracle's forward step (stable split by destination).

The forward step of Sec. 4.2.1-4.2.2 (sort by the key (dest << 32 | i), gather,
tally begin/end, Alltoall of counts, Alltoallv of items) is checked here
against things other than the oracle itself:
  * numpy's stable argsort on the destinations;
  * a simulation of R ranks doing exactly the paper's sort-key / tally /
    Alltoall / Alltoallv sequence, whose receive buffers must equal the
    single-array split byte for byte;
  * invariants and special cases (D = 1, all done, empty input).
"""
import numpy as np
import pytest

from paper_2605_30294_amd import workloads as W


def _expected_by_argsort(items, dest, D):
    valid = (dest >= 0) & (dest < D)
    order = np.argsort(dest[valid], kind="stable")
    return items[valid][order], np.bincount(dest[valid], minlength=D)


@pytest.mark.parametrize("n,D,seed", [(0, 4, 0), (1, 1, 1), (37, 3, 2), (1000, 17, 3),
                                      (5000, 1024, 4), (4096, 64, 5)])
def test_split_matches_stable_argsort(orc, n, D, seed):
    rng = np.random.default_rng(seed)
    dest = rng.integers(-3, D + 2, n).astype(np.int32)   # includes done (-1) and bad values
    items = rng.integers(0, 2**32, (n, 8), dtype=np.uint64).astype(np.uint32)
    out, counts, offsets, nd, nb = orc.multisplit(items, dest, D)
    exp_out, exp_counts = _expected_by_argsort(items, dest, D)
    assert np.array_equal(out, exp_out)
    assert np.array_equal(counts, exp_counts.astype(np.uint64))
    assert offsets[0] == 0 and np.array_equal(np.diff(offsets.astype(np.int64)), counts.astype(np.int64))
    assert nd == int((dest == -1).sum())
    assert nb == int(((dest < -1) | (dest >= D)).sum())
    assert int(counts.sum()) + nd + nb == n


def test_split_invariants_zipf(orc):
    n, D = 200_000, 1024
    dest = W.split_dest(n, D, "zipf")
    items = W.split_items(n)
    out, counts, offsets, nd, nb = orc.multisplit(items, dest, D)
    assert nd == 0 and nb == 0 and int(offsets[-1]) == n
    # output is a permutation of the input (ids are word 0)
    ids = out[:, 0].astype(np.int64)
    assert np.array_equal(np.sort(ids), np.arange(n))
    # within each bucket the source index increases (stability) and the
    # destination of every item matches its bucket
    for e in [0, 1, 2, 511, 1023]:
        seg = ids[int(offsets[e]):int(offsets[e + 1])]
        assert np.all(np.diff(seg) > 0)
        assert np.all(dest[seg] == e)
    # the truncated Zipf head holds ~17.9% of the items
    assert abs(counts[0] / n - 1.0 / np.sum(np.arange(1, D + 1) ** -1.1)) < 0.01


def test_split_special_cases(orc):
    rng = np.random.default_rng(7)
    items = rng.integers(0, 2**31, (500, 4)).astype(np.int32)
    # D = 1: order-preserving compaction of the kept items
    dest = np.where(rng.random(500) < 0.3, -1, 0).astype(np.int32)
    out, counts, offsets, nd, nb = orc.multisplit(items, dest, 1)
    assert np.array_equal(out, items[dest == 0])
    # everything done: total 0
    out, counts, offsets, nd, nb = orc.multisplit(items, np.full(500, -1, np.int32), 8)
    assert int(offsets[-1]) == 0 and nd == 500 and counts.sum() == 0
    # everything into one bucket keeps the order
    out, counts, offsets, nd, nb = orc.multisplit(items, np.full(500, 5, np.int32), 8)
    assert np.array_equal(out, items) and int(offsets[5]) == 0 and int(offsets[6]) == 500
    # empty buckets get zero counts and the running offset
    assert list(offsets[:6]) == [0] * 6 and list(offsets[6:]) == [500] * 3


def _paper_exchange(items, dest, R):
    """R ranks hold contiguous slices of the emitted slots. Each rank builds
    the 64-bit keys (dest << 32 | i), radix-sorts them, gathers, finds the
    begin/end of every destination run by comparing neighbours, fills gaps,
    exchanges counts (Alltoall) and items (Alltoallv, receive buffers in
    source-rank order)."""
    n = len(dest)
    bounds = np.linspace(0, n, R + 1).astype(np.int64)
    send = []
    for r in range(R):
        d = dest[bounds[r]:bounds[r + 1]]
        it = items[bounds[r]:bounds[r + 1]]
        keep = d >= 0                               # only emitted (forwarded) items
        d, it = d[keep], it[keep]
        key = (d.astype(np.uint64) << np.uint64(32)) | np.arange(len(d), dtype=np.uint64)
        key = np.sort(key)                          # keys are unique: any sort is the radix sort's result
        idx = (key & np.uint64(0xFFFFFFFF)).astype(np.int64)
        sd = (key >> np.uint64(32)).astype(np.int64)
        sorted_items = it[idx]
        begin = np.full(R, -1, np.int64)
        end = np.full(R, -1, np.int64)
        for i in range(len(sd)):
            if i == 0 or sd[i] != sd[i - 1]:
                begin[sd[i]] = i
            if i == len(sd) - 1 or sd[i] != sd[i + 1]:
                end[sd[i]] = i + 1
        cnt = np.where(begin < 0, 0, end - begin)
        off = np.where(begin < 0, 0, begin)
        send.append((sorted_items, cnt, off))
    recv = []
    for dst in range(R):                            # Alltoallv: sources in rank order
        parts = [s[0][s[2][dst]:s[2][dst] + s[1][dst]] for s in send]
        recv.append(np.concatenate(parts) if parts else items[:0])
    return recv


@pytest.mark.parametrize("R,n,seed", [(2, 100, 0), (4, 3000, 1), (8, 20000, 2), (5, 7, 3)])
def test_split_equals_paper_alltoallv(orc, R, n, seed):
    rng = np.random.default_rng(seed)
    dest = rng.integers(-1, R, n).astype(np.int32)
    items = rng.integers(0, 2**32, (n, 11), dtype=np.uint64).astype(np.uint32)   # 44-byte items
    recv = _paper_exchange(items, dest, R)
    out, counts, offsets, nd, nb = orc.multisplit(items, dest, R)
    for e in range(R):
        assert np.array_equal(out[int(offsets[e]):int(offsets[e + 1])], recv[e])
