"""A CPU replay of the source stream of the pair-once near-field kernel.

The kernel stages a segment's records (at most 64, one per lane) and takes
their source points as one stream, 64 per step.  A lane finds the record of
its flat index f = 64 st + lane from the records' inclusive ends: a ballot
counts the records ending at or before the step's first index, a second the
records ending inside the step, and a uniform walk over the latter adds one
for each end at or before f.  The replay checks, for record sizes of the
kinds the tree produces (equal within one, leaves of 17 to 64 points) and
for arbitrary ones (empty records, single points, a segment shorter than 64
records), that this gives the record that holds f, that the source position
and the source-sum position the kernel forms from it are the record's own,
and that the walk stays within the 64 lanes.

This is test infrastructure: it models the kernel's indexing only and holds
none of the method's arithmetic.
"""
import numpy as np
import pytest


def stream_records(sizes):
    """Per step and lane: the kernel's record index (None past the stream)."""
    sizes = list(sizes) + [0] * (64 - len(sizes))  # lanes past the segment: empty records
    rend = np.cumsum(sizes)  # lane r: one past the last flat index of record r
    nflat = int(rend[63])
    out = []
    for st in range((nflat + 63) // 64):
        r_lo = int(np.count_nonzero(rend <= 64 * st))
        r_hi = int(np.count_nonzero(rend <= 64 * st + 63))
        assert 0 <= r_lo <= r_hi <= 64
        row = []
        for lane in range(64):
            f = 64 * st + lane
            r = r_lo
            for i in range(r_lo, r_hi):  # uniform walk: i < 64
                r += 1 if f >= rend[i] else 0
            row.append(r if f < nflat else None)
        out.append(row)
    return out, rend, nflat


def check(sizes):
    steps, rend, nflat = stream_records(sizes)
    pre = np.concatenate([[0], rend[:-1]])
    seen = set()
    for st, row in enumerate(steps):
        for lane, r in enumerate(row):
            f = 64 * st + lane
            if r is None:
                assert f >= nflat
                continue
            assert 0 <= r < len(sizes)  # a real record
            assert pre[r] <= f < rend[r]  # ... the one holding f
            jj = f - pre[r]  # point of the source leaf, and its source-sum slot
            assert 0 <= jj < sizes[r] <= 64
            seen.add((r, jj))
    # every point of every record is streamed exactly once
    assert seen == {(r, j) for r, m in enumerate(sizes) for j in range(m)}
    assert len(steps) == (sum(sizes) + 63) // 64


@pytest.mark.parametrize("m", [17, 24, 32, 33, 38, 39, 40, 48, 50, 63, 64])
def test_tree_like_segments(m):
    rng = np.random.default_rng(m)
    for nrec in (1, 2, 7, 25, 63, 64):
        sizes = [m - int(rng.integers(0, 2)) if m > 17 else m for _ in range(nrec)]
        check(sizes)


def test_arbitrary_sizes():
    rng = np.random.default_rng(7)
    for _ in range(300):
        nrec = int(rng.integers(1, 65))
        sizes = [int(v) for v in rng.integers(0, 65, nrec)]
        if sum(sizes) == 0:
            sizes[0] = 1
        check(sizes)


def test_degenerate_segments():
    check([1])
    check([64])
    check([1] * 64)
    check([64] * 64)
    check([0, 0, 5, 0, 64, 0, 1])
