"""Coverage counts for parity inputs, computed with the oracle only.

A parity test is only as strong as the values its input sends through each
stage.  These helpers count, for a given input, how many output rows take
their value through the stages that only long-range inputs reach, so a test
can assert minimum counts and an input cannot silently degenerate into
EMPTY rows.  They mirror the kernels' tiling only to decide which stage a
dependency crosses (partitions of T elements, union blocks of UB
partitions); the values themselves come from the oracle.
"""
import numpy as np

import oracle

T = 1024  # elements per partition
UB = 256  # partitions per union block
BIG = np.float32(3e38)  # a finite box that contains every other box


def nonempty(out):
    return (out[:, 0] < out[:, 2]) & (out[:, 1] < out[:, 3])


def far_context_rows(kind, box, out, first_parts, min_dist):
    """Non-EMPTY rows at least `min_dist` partitions after the first
    `first_parts` partitions whose value changes when the clips of those
    partitions stop cutting anything: their clip context carries a value
    from that far back, which only the pointer jumping over partitions
    brings in (2^r partitions per round r)."""
    lim = min(first_parts * T, len(kind))
    b2 = box.copy()
    clips = np.flatnonzero(kind[:lim] == 1)
    b2[clips] = [-BIG, -BIG, BIG, BIG]
    _, _, out2, st = oracle.bbox(kind, b2)
    assert st == 0
    start = (first_parts + min_dist) * T
    ch = (out[start:].view(np.uint32) != out2[start:].view(np.uint32)).any(1) & nonempty(out[start:])
    return int(ch.sum())


def mid_block_unions(kind, box, match, out):
    """(count, levels) of blend rows whose pair leaves at least one whole
    union block strictly between the blocks of its open and close
    partitions, and whose value changes when the leaves of such a block are
    made EMPTY: the block-level range union (sparse table over blocks)
    delivers part of their value.  `levels` is the set of sparse-table levels
    (log2 of the number of whole blocks between) those pairs use."""
    n = len(kind)
    nblk = (n + T * UB - 1) // (T * UB)
    closes = np.flatnonzero((kind == 4) & (match >= 0))
    opens = match[closes].astype(np.int64)
    a = opens // T + 1
    bend = closes // T - 1
    ba, bb = a // UB, bend // UB
    count, levels = 0, set()
    for blk in range(1, nblk - 1):
        sel = (ba < blk) & (blk < bb)
        if not sel.any():
            continue
        b2 = box.copy()
        lo, hi = blk * T * UB, min((blk + 1) * T * UB, n)
        leaves = lo + np.flatnonzero(kind[lo:hi] == 0)
        b2[leaves] = 0.0  # zero area: EMPTY, out of every union
        _, _, out2, st = oracle.bbox(kind, b2)
        assert st == 0
        c = closes[sel]
        ch = (out[c].view(np.uint32) != out2[c].view(np.uint32)).any(1) & nonempty(out[c])
        count += int(ch.sum())
        nb = (bb[sel] - ba[sel] - 1)[ch]
        levels.update(int(x).bit_length() - 1 for x in np.unique(nb))
    return count, levels


def cross_partition_routes(kind, box, min_parts=1):
    """Gradient routes (row, coordinate) -> source element whose source lies
    at least `min_parts` partitions away from the row, and how many of those
    rows are blend rows."""
    src, st = oracle.sources(kind, box)
    assert st == 0
    rows = np.repeat(np.arange(len(kind)), 4).reshape(-1, 4)
    ok = src >= 0
    far = ok & (np.abs(rows // T - np.where(ok, src, 0) // T) >= min_parts)
    blend = far & np.isin(kind, (3, 4))[:, None]
    return int(far.sum()), int(blend.sum()), int(ok.sum())
