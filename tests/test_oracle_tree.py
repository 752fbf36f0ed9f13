"""Pins of the oracle's cluster tree (oracle/tree.py) against Sec. 2.1 / Fig. 1."""
import numpy as np
import pytest

from oracle.tree import bisection_tree, tree_from_arrays


def test_fig1_numbering_and_intervals():
    # Fig. 1: a three-level tree, root [1,n], children 1,2 and grandchildren
    # 3,4,5,6 with the quarter intervals; children of i are 2i+1, 2i+2.
    n = 400
    t = bisection_tree(n, n // 4)
    assert t.n_nodes == 7
    for i in range(3):
        assert t.left[i] == 2 * i + 1 and t.right[i] == 2 * i + 2
    q = n // 4
    assert [(t.lo[i], t.hi[i]) for i in (3, 4, 5, 6)] == [(0, q), (q, 2 * q), (2 * q, 3 * q), (3 * q, n)]
    assert (t.lo[2], t.hi[2]) == (n // 2, n)
    assert t.height[0] == 2 and all(t.height[i] == 0 for i in (3, 4, 5, 6))


@pytest.mark.parametrize("n,leaf", [(1, 4), (5, 5), (6, 5), (129, 64), (1000, 64), (1023, 7), (65536, 256)])
def test_partition_invariants(n, leaf):
    t = bisection_tree(n, leaf)
    assert (t.lo[0], t.hi[0]) == (0, n)
    covered = np.zeros(n, dtype=int)
    for v in range(t.n_nodes):
        if t.is_leaf(v):
            assert 1 <= t.size(v) <= leaf
            covered[t.lo[v]:t.hi[v]] += 1
            assert t.height[v] == 0
        else:
            a, b = t.left[v], t.right[v]
            assert t.size(v) > leaf
            assert t.lo[a] == t.lo[v] and t.hi[a] == t.lo[b] and t.hi[b] == t.hi[v]
            assert t.size(a) == t.size(v) // 2
            assert t.height[v] == 1 + max(t.height[a], t.height[b])
            assert t.parent[a] == v and t.parent[b] == v
            assert a > v and b > v
    assert np.all(covered == 1)


def test_complete_tree_sizes():
    t = bisection_tree(65536, 256)
    assert len(t.leaves()) == 256 and t.n_nodes == 511 and t.height[0] == 8
    t = bisection_tree(16384, 128)
    assert len(t.leaves()) == 128 and t.height[0] == 7
    t = bisection_tree(1024, 64)
    assert len(t.leaves()) == 16 and t.n_nodes == 31 and t.height[0] == 4


def test_uneven_depths():
    # 129 = 64 + 65: the left child is a leaf, the right one splits again
    t = bisection_tree(129, 64)
    assert t.is_leaf(1) and not t.is_leaf(2) and t.height[0] == 2 and t.height[1] == 0


def test_user_tree_roundtrip_and_validation():
    t = bisection_tree(300, 40)
    u = tree_from_arrays(t.lo, t.hi, t.left, t.right)
    assert u.height == t.height and u.parent == t.parent
    bad_hi = list(t.hi)
    bad_hi[1] -= 1
    with pytest.raises(ValueError):
        tree_from_arrays(t.lo, bad_hi, t.left, t.right)
