"""Host logic of bench.py: the BFS byte model it applies to the oracle's
replay of a direction schedule."""
import numpy as np

import bench
import graphgen as gg
import oracle
from tests import helpers as H


def test_all_top_down_bytes_equal_the_reached_set_formula():
    # every reached vertex is a frontier once and every out-edge of it is
    # examined once: 4 E + 8 R + 12 (R - 1)
    host = gg.rmat(10, 16, seed=3)
    for root in (0, 5, 700):
        level, _, nlev = oracle.bfs(host.off, host.idx, root)
        dirs = np.zeros(nlev, dtype=np.int8)
        fr, ex, di = oracle.bfs_replay(host.off, host.idx, root, dirs)
        reached = level >= 0
        E = int(np.diff(host.off)[reached].sum())
        R = int(reached.sum())
        assert bench.bfs_replay_bytes(host.n, fr, ex, di, dirs) == 4 * E + 8 * R + 12 * (R - 1)


def test_bottom_up_bytes_of_a_star_from_its_centre():
    # step 0: the nine leaves each scan their one in-edge and find the centre;
    # step 1: nothing is left unvisited, only the three bitmaps are read
    host = H.star(10)
    dirs = np.array([1, 1], dtype=np.int8)
    fr, ex, di = oracle.bfs_replay(host.off, host.idx, 0, dirs)
    assert list(ex) == [9, 0] and list(di) == [9, 0]
    assert bench.bfs_replay_bytes(10, fr, ex, di, dirs) == (4 * 9 + 8 * 9 + 8 * 9 + 3 * 2) + 3 * 2
