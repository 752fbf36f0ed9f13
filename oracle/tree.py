"""Binary cluster tree on the index set [0, n) (Sec. 2.1, Fig. 1).

Every node tau owns an interval I_tau = [lo, hi); the root owns [0, n); the
children of a node split its interval into two disjoint, adjacent halves.
Reading taken where the paper is silent on the split rule: an interval of
m > leaf_size indices is split into its first floor(m/2) and last ceil(m/2)
indices; intervals of at most leaf_size indices are leaves.

Nodes are numbered breadth-first from the root (0); for a complete tree this
is the paper's numbering (children of i are 2i+1 and 2i+2).  The height of
a leaf is 0 and that of an inner node is one more than the larger height of
its children; the level-synchronous schedule processes nodes by height,
which keeps children before parents also in uneven trees (Sec. 4.2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class ClusterTree:
    lo: list = field(default_factory=list)
    hi: list = field(default_factory=list)
    left: list = field(default_factory=list)
    right: list = field(default_factory=list)
    parent: list = field(default_factory=list)
    height: list = field(default_factory=list)

    @property
    def n_nodes(self) -> int:
        return len(self.lo)

    def is_leaf(self, t: int) -> bool:
        return self.left[t] < 0

    def size(self, t: int) -> int:
        return self.hi[t] - self.lo[t]

    def nodes_at_height(self, h: int) -> list:
        return [t for t in range(self.n_nodes) if self.height[t] == h]

    def leaves(self) -> list:
        return [t for t in range(self.n_nodes) if self.is_leaf(t)]


def bisection_tree(n: int, leaf_size: int) -> ClusterTree:
    if n < 1 or leaf_size < 1:
        raise ValueError("n and leaf_size must be positive")
    t = ClusterTree()
    t.lo.append(0)
    t.hi.append(n)
    t.left.append(-1)
    t.right.append(-1)
    t.parent.append(-1)
    head = 0
    while head < len(t.lo):  # breadth-first
        lo, hi = t.lo[head], t.hi[head]
        m = hi - lo
        if m > leaf_size:
            mid = lo + m // 2
            for a, b in ((lo, mid), (mid, hi)):
                t.lo.append(a)
                t.hi.append(b)
                t.left.append(-1)
                t.right.append(-1)
                t.parent.append(head)
            t.left[head] = len(t.lo) - 2
            t.right[head] = len(t.lo) - 1
        head += 1
    t.height = [0] * len(t.lo)
    for v in range(len(t.lo) - 1, -1, -1):  # children have larger numbers
        if t.left[v] >= 0:
            t.height[v] = 1 + max(t.height[t.left[v]], t.height[t.right[v]])
    return t


def tree_from_arrays(lo, hi, left, right) -> ClusterTree:
    """Tree given by the caller (root 0, -1 = no child); validated."""
    t = ClusterTree(list(map(int, lo)), list(map(int, hi)), list(map(int, left)),
                    list(map(int, right)))
    nn = t.n_nodes
    t.parent = [-1] * nn
    for v in range(nn):
        if (t.left[v] < 0) != (t.right[v] < 0):
            raise ValueError("a node has exactly one child")
        if t.left[v] >= 0:
            a, b = t.left[v], t.right[v]
            if t.lo[a] != t.lo[v] or t.hi[a] != t.lo[b] or t.hi[b] != t.hi[v]:
                raise ValueError("children do not split the parent interval")
            t.parent[a] = v
            t.parent[b] = v
    order = np.argsort(-np.arange(nn))
    t.height = [0] * nn
    changed = True
    while changed:  # small trees only; fixed point of the height recursion
        changed = False
        for v in order:
            if t.left[v] >= 0:
                h = 1 + max(t.height[t.left[v]], t.height[t.right[v]])
                if h != t.height[v]:
                    t.height[v] = h
                    changed = True
    return t
