"""Textbook pointer octree and recursive Barnes-Hut walk, in pure Python.

An independent check of the oracle's Morton-key tree: cubes are split by
comparing coordinates with cube midpoints (no keys, no sorting), following
the recursive subdivision of the paper's introduction and Fig. 2.  It uses
the same readings of the paper as the oracle (root cube anchored at the
minimum corner with a power-of-two side; depth limit 21; single-child cubes
removed; side-length opening test against the centre of mass) but none of
its code.  Meant for small N only.
"""
from __future__ import annotations

import math

MAX_LEVEL = 21


class Node:
    __slots__ = ("level", "cell", "ids", "children", "M", "com", "pre")

    def __init__(self, level, cell, ids):
        self.level = level
        self.cell = cell          # integer cube coordinates at this level
        self.ids = ids            # particle indices (original numbering)
        self.children = []
        self.M = 0.0
        self.com = (0.0, 0.0, 0.0)
        self.pre = -1


def root_cube(pos):
    lo = [min(p[d] for p in pos) for d in range(3)]
    hi = [max(p[d] for p in pos) for d in range(3)]
    ext = max(hi[d] - lo[d] for d in range(3))
    if ext == 0.0:
        return lo, 1.0
    _, e = math.frexp(ext)
    return lo, math.ldexp(1.0, e)


def build(pos, mass, leaf_cap=1):
    """Returns (root, nodes_in_preorder, lo, L)."""
    pos = [tuple(float(v) for v in p) for p in pos]
    lo, L = root_cube(pos)
    off = [tuple(p[d] - lo[d] for d in range(3)) for p in pos]

    def split(level, cell, ids):
        # keep subdividing while the cube is crowded and not at the depth limit;
        # a cube whose particles all go to one sub-cube is replaced by that sub-cube
        while True:
            if len(ids) <= leaf_cap or level == MAX_LEVEL:
                return Node(level, cell, ids)
            half = L / 2 ** (level + 1)
            groups = {}
            for i in ids:
                bits = []
                for d in range(3):
                    mid = (2 * cell[d] + 1) * half      # exact: power-of-two multiples
                    bits.append(1 if off[i][d] >= mid else 0)
                octant = 4 * bits[0] + 2 * bits[1] + bits[2]
                groups.setdefault(octant, []).append(i)
            kids = []
            for octant in sorted(groups):
                b = ((octant >> 2) & 1, (octant >> 1) & 1, octant & 1)
                kids.append((tuple(2 * cell[d] + b[d] for d in range(3)), groups[octant]))
            if len(kids) == 1:
                level, cell, ids = level + 1, kids[0][0], kids[0][1]
                continue
            node = Node(level, cell, ids)
            node.children = [split(level + 1, c, g) for c, g in kids]
            return node

    root = split(0, (0, 0, 0), list(range(len(pos))))
    nodes = []

    def number(nd):
        nd.pre = len(nodes)
        nodes.append(nd)
        for c in nd.children:
            number(c)

    number(root)
    for nd in nodes:
        m = math.fsum(mass[i] for i in nd.ids)
        nd.M = m
        nd.com = tuple(math.fsum(mass[i] * pos[i][d] for i in nd.ids) / m for d in range(3))
    return root, nodes, lo, L


def walk(root, nodes, pos, mass, L, i, theta, eps, G=1.0, radius2=None):
    """Recursive BH force on body i.  Returns (acc, accepted node ids, pair partner ids).
    radius2(node, side) gives r^2 of the test r^2 < theta^2 D^2 (default: side^2)."""
    x = [float(v) for v in pos[i]]
    acc = [0.0, 0.0, 0.0]
    mono, pairs = [], []

    def add(y, m):
        d = [y[c] - x[c] for c in range(3)]
        r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps * eps
        if r2 == 0.0:
            return
        w = G * m / (r2 * math.sqrt(r2))
        for c in range(3):
            acc[c] += w * d[c]

    def visit(nd):
        D2 = sum((nd.com[c] - x[c]) ** 2 for c in range(3))
        s = L / 2 ** nd.level
        r2 = s * s if radius2 is None else radius2(nd, s)
        if r2 < theta * theta * D2:
            add(nd.com, nd.M)
            mono.append(nd.pre)
        elif not nd.children:
            for j in sorted(nd.ids):
                if j != i:
                    add(pos[j], mass[j])
                    pairs.append(j)
        else:
            for c in nd.children:
                visit(c)

    visit(root)
    return acc, mono, pairs
