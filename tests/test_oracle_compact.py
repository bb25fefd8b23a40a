"""Pin of the oracle's point-cloud compaction on a hand-built record array: the
defined records, unchanged, in raster order."""
import numpy as np

from oracle import oracle


def test_compaction_by_hand():
    H, W = 3, 4
    rec = np.zeros((H, W, 8), np.float32)
    for v in range(H):
        for u in range(W):
            rec[v, u, :6] = [u, v, 10 * v + u, 0, 0, -1]
    flags = np.zeros((H, W), np.uint32)
    defined = [(0, 1), (1, 0), (1, 3), (2, 2)]          # (v, u)
    for v, u in defined:
        flags[v, u] = 1 | 2
    flags[0, 0] = 2                                     # labelled, not defined
    rec[..., 7] = flags.view(np.float32)
    out = oracle.compact_points(rec)
    assert out.shape == (4, 8)
    assert [(int(r[1]), int(r[0])) for r in out] == defined
    assert np.array_equal(out.view(np.uint32)[:, 7], np.full(4, 3, np.uint32))
    assert oracle.compact_points(np.zeros((2, 2, 8), np.float32)).shape == (0, 8)
