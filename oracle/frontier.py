"""Persistent active sets across Picard iterations (FP64 oracle).

TEST INFRASTRUCTURE ONLY: the tests and the smoke check use this module; the
product path never imports it.

Follows Section 5.3 (Algorithm 6, the multiscale Picard scheme with its
widening and narrowing of active sets, and the implementation note on the
memory set U) in the pairwise reading that the descent uses (Algorithm 5 read
pairwise): the active set of a candidate particle pair is a set of triangle
pairs, kept between calls.  Written as an explicit tree of triangle pairs so
that nothing here depends on how the GPU path lays its state out:

- the active set starts as all pairs of root triangles (Algorithm 6, first
  statement);
- one step evaluates every active pair with the exact comparison-based
  distance (Section 3): a pair whose distance exceeds eps_a + eps_b is "no
  contact"; a pair of fine triangles within it is a contact; a pair with a
  surrogate within it is replaced by the pairs of its children, one level
  only (widening; only the non-fine side unfolds);
- a pair whose child pairs are all active and all "no contact" in this step
  gets them replaced by itself (narrowing, the clean-up of Algorithm 6),
  unless the memory set vetoes it.  The memory set of a candidate particle
  pair holds every pair whose child pairs were once removed this way; it
  only grows, so once removed pairs have come back they are never removed
  again.

``Frontier.leaves()`` lists the active pairs in depth-first order (children
in (child of a) x (child of b) row-major order, root pairs likewise), with a
flag word: bit 0 = this pair is in the memory set, bit d >= 1 = this pair's
ancestor at depth d - 1 is in the memory set (so the child pairs of that
ancestor may not be narrowed).
"""
from __future__ import annotations

import numpy as np

from . import OracleTree, tri_tri_batch

PRUNE, KEEP, UNFOLD = 0, 1, 2


class _Node:
    __slots__ = ("a", "b", "depth", "kids")

    def __init__(self, a: int, b: int, depth: int):
        self.a, self.b, self.depth = a, b, depth
        self.kids = None        # child pairs while unfolded


class Frontier:
    """Active sets of all candidate particle pairs of one tree topology."""

    def __init__(self, t: OracleTree, pairs=None):
        P = np.asarray(t.pairs if pairs is None else pairs).reshape(-1, 2)
        self.child_begin = t.child_begin
        self.child_count = t.child_count
        self.tops = []
        self.memory = set()     # pairs (a, b) whose child pairs were removed once
        for pi, pj in P:
            top = _Node(-1, -1, -1)
            ri = range(int(t.root_begin[pi]), int(t.root_begin[pi] + t.root_count[pi]))
            rj = range(int(t.root_begin[pj]), int(t.root_begin[pj] + t.root_count[pj]))
            top.kids = [_Node(a, b, 0) for a in ri for b in rj]
            self.tops.append(top)

    # ------------------------------------------------------------ traversal
    def _walk(self):
        """(leaf, flags, parent) in depth-first order."""
        out = []

        def visit(node, parent, flags):
            mem = (node.a, node.b) in self.memory
            if node.kids is None:
                out.append((node, flags | int(mem), parent))
                return
            # the child pairs of `node` sit at depth node.depth + 1
            f = flags | ((1 << (node.depth + 1)) if mem else 0)
            for c in node.kids:
                visit(c, node, f)

        for top in self.tops:
            for c in top.kids:
                visit(c, None, 0)
        return out

    def leaves(self) -> np.ndarray:
        """(n, 4) int64 rows [a, b, flags, depth] in depth-first order."""
        w = self._walk()
        return np.array([[n.a, n.b, f, n.depth] for n, f, _ in w], np.int64).reshape(-1, 4)

    def _children(self, t: int):
        c = int(self.child_count[t])
        return [t] if c == 0 else list(range(int(self.child_begin[t]), int(self.child_begin[t]) + c))

    # ------------------------------------------------------------ one step
    def step(self, t: OracleTree) -> dict:
        """Evaluate every active pair at the positions of ``t`` (same topology),
        then narrow and widen.  Returns this step's contacts and counts."""
        w = self._walk()
        n = len(w)
        a = np.array([x[0].a for x in w], np.int64)
        b = np.array([x[0].b for x in w], np.int64)
        if n:
            X = t.verts[t.tris[a]]
            Y = t.verts[t.tris[b]]
            r = tri_tri_batch(np.stack([X, Y], axis=1))
            d = r["d"]
        else:
            d = np.zeros(0)
        delta = t.eps[a] + t.eps[b]
        fine = (t.child_count[a] == 0) & (t.child_count[b] == 0)
        out = np.where(d > delta, PRUNE, np.where(fine, KEEP, UNFOLD))
        margin = float(np.min(np.abs(d - delta) / np.maximum(delta, 1e-300))) if n else np.inf
        keep = out == KEEP
        res = {"a": a[keep], "b": b[keep], "d": d[keep], "outcome": out, "leaves_in": n,
               "margin": margin}

        # narrowing: groups of child pairs all active and all "no contact"
        by_parent = {}
        for k, (node, _, parent) in enumerate(w):
            if parent is not None:
                by_parent.setdefault(id(parent), (parent, []))[1].append(k)
        collapsed = 0
        for parent, ks in by_parent.values():
            if len(ks) != len(parent.kids) or (parent.a, parent.b) in self.memory:
                continue
            if all(out[k] == PRUNE for k in ks):
                parent.kids = None
                self.memory.add((parent.a, parent.b))
                collapsed += 1

        # widening: one level below every pair a surrogate of which is in range
        unfolded = 0
        for k, (node, _, _) in enumerate(w):
            if out[k] == UNFOLD:
                node.kids = [_Node(x, y, node.depth + 1) for x in self._children(node.a)
                             for y in self._children(node.b)]
                unfolded += 1
        res["unfolded"] = unfolded
        res["collapsed"] = collapsed
        return res

    def run_until_fixed(self, t: OracleTree, max_steps: int = 64) -> list:
        """Steps at fixed positions until a step neither widens nor narrows."""
        hist = []
        for _ in range(max_steps):
            r = self.step(t)
            hist.append(r)
            if r["unfolded"] == 0 and r["collapsed"] == 0:
                return hist
        raise RuntimeError("active sets kept changing")
