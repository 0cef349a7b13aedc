"""Input generators that are not matrices of the method itself: the multi-source BFS frontier matrices of
the square x tall-skinny workload, checked against a plain breadth-first search."""
import numpy as np

import synth


def _bfs_dist(A, s):
    dist = np.full(A.nrows, -1)
    dist[s] = 0
    front, d = [s], 0
    while front:
        d += 1
        nxt = []
        for u in front:
            for w in A.col[A.rp[u]:A.rp[u + 1]]:
                if dist[w] < 0:
                    dist[w] = d
                    nxt.append(int(w))
        front = nxt
    return dist


def test_frontier_columns_are_bfs_level_sets():
    A = synth.workload_stencil27(5, 2, 3)[0]
    dist = np.array([_bfs_dist(A, s) for s in range(A.nrows)])   # all-pairs distances of the small graph
    for level in (0, 1, 2, 3, 9):
        B = synth.frontiers(A, 8, level, 7)
        assert B.nrows == A.nrows and B.ncols == 8
        for s in range(8):
            members = sorted(v for v in range(A.nrows) if s in B.col[B.rp[v]:B.rp[v + 1]])
            # the column is the level set of one source, and the 8 sources are distinct
            matches = [c for c in range(A.nrows) if sorted(np.nonzero(dist[c] == level)[0].tolist()) == members]
            assert matches, (level, s)
        # rows sorted, values in [-1, 1)
        for v in range(B.nrows):
            c = B.col[B.rp[v]:B.rp[v + 1]]
            assert np.all(np.diff(c) > 0)
        assert np.all((B.val >= -1) & (B.val < 1))


def test_frontier_sources_distinct_and_seeded():
    A = synth.rmat(8, 8, 0.57, 0.19, 0.19, 2)
    B0 = synth.frontiers(A, 32, 0, 11)
    assert B0.nnz == 32                                   # level 0: each source itself
    rows = np.repeat(np.arange(A.nrows), np.diff(B0.rp))
    assert len(set(rows.tolist())) == 32                  # distinct sources
    B1 = synth.frontiers(A, 32, 2, 11)
    B2 = synth.frontiers(A, 32, 2, 11)
    assert np.array_equal(B1.col, B2.col) and np.array_equal(B1.val, B2.val)
