"""Per-chunk results from one oracle run over chunks laid end to end.

An occurrence found in the concatenation belongs to chunk k when it starts in
chunk k and ends inside it; those are exactly chunk k's own occurrences, so
the per-chunk results need only one (multi-threaded) oracle call.
"""

import numpy as np


def split_by_chunk(off, ids, pattern_lengths, offsets, sizes):
    """(chunk of each kept record, offset in its chunk, id) for records wholly inside a chunk."""
    off = np.asarray(off, dtype=np.int64)
    ids = np.asarray(ids, dtype=np.int64)
    lens = np.asarray(pattern_lengths, dtype=np.int64)
    starts = np.asarray(offsets, dtype=np.int64)
    ends = starts + np.asarray(sizes, dtype=np.int64)
    k = np.searchsorted(starts, off, side="right") - 1
    inside = (k >= 0) & (off + lens[ids] <= ends[np.maximum(k, 0)])
    return k[inside], off[inside] - starts[k[inside]], ids[inside]
