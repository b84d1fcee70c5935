"""Cluster tree and block cluster tree of the H-matrix (Sec. III-A, eq. 21).

Test infrastructure: a plain, slow reference for the host tree builder,
written from the method's description, not from the library.

The paper fixes the admissibility condition (eq. 21: the smaller of the two
cluster diameters at most eta times their distance) and leaves the rest
open.  The reading taken here:
  * clusters are sets of whole patches of one object; a cluster with at
    most `leaf` unknowns (unknowns per node x its nodes), or with a single
    patch, is a leaf;
  * otherwise its patches are ordered by centroid coordinate along the
    longest axis of the cluster's node bounding box (the lowest axis index
    on equal extents; equal coordinates ordered by patch index) and cut in
    the middle, the first half (floor of half the count) going left;
  * diameter = diagonal of the bounding box, distance = gap between the two
    boxes (zero when they touch or overlap);
  * a block (t, s) is low-rank when the gap is positive, eq. 21 holds and no
    node of t has a patch of s in its near set (so near pairs are always
    integrated by the singular quadrature, inside dense blocks); it is dense
    when t or s is a leaf; otherwise it splits into the four child pairs;
  * objects of a batch are independent: one tree and one diagonal block
    tree per object.
The patch order of the tree is the order of the leaves, left to right.
"""
from __future__ import annotations

import math

import numpy as np


class Cluster:
    def __init__(self, patches, lo, hi):
        self.patches = patches        # original patch indices, tree order
        self.lo, self.hi = lo, hi     # node bounding box
        self.kids = ()

    @property
    def is_leaf(self):
        return not self.kids


def _box(patches, pbox):
    lo = tuple(min(pbox[p][d] for p in patches) for d in range(3))
    hi = tuple(max(pbox[p][3 + d] for p in patches) for d in range(3))
    return lo, hi


def build_cluster(patches, centroid, pbox, patch_nodes, upn, leaf):
    """Recursive bisection of a list of patches (see the module notes)."""
    lo, hi = _box(patches, pbox)
    unknowns = upn * sum(patch_nodes[p] for p in patches)
    if unknowns <= leaf or len(patches) == 1:
        return Cluster(list(patches), lo, hi)
    ext = [hi[d] - lo[d] for d in range(3)]
    ax = ext.index(max(ext))
    order = sorted(patches, key=lambda p: (centroid[p][ax], p))
    half = len(order) // 2
    left = build_cluster(order[:half], centroid, pbox, patch_nodes, upn, leaf)
    right = build_cluster(order[half:], centroid, pbox, patch_nodes, upn, leaf)
    c = Cluster(left.patches + right.patches, lo, hi)
    c.kids = (left, right)
    return c


def diameter(c):
    dx, dy, dz = (c.hi[d] - c.lo[d] for d in range(3))
    return math.sqrt(dx * dx + dy * dy + dz * dz)


def distance(a, b):
    g = [max(0.0, a.lo[d] - b.hi[d], b.lo[d] - a.hi[d]) for d in range(3)]
    return math.sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2])


def block_leaves(t, s, eta, near):
    """Leaf blocks of the block tree under (t, s), depth first with the
    children in the order (t1, s1), (t1, s2), (t2, s1), (t2, s2): a list of
    (kind, t, s) with kind "lr" or "dense".  `near` is the set of (target
    patch, source patch) pairs of near interactions."""
    d = distance(t, s)
    touching = any((a, b) in near for a in t.patches for b in s.patches)
    if d > 0.0 and min(diameter(t), diameter(s)) <= eta * d and not touching:
        return [("lr", t, s)]
    if t.is_leaf or s.is_leaf:
        return [("dense", t, s)]
    out = []
    for a in t.kids:
        for b in s.kids:
            out += block_leaves(a, b, eta, near)
    return out


def build(patch_obj, centroid, pbox, patch_nodes, near, upn, leaf, eta):
    """Trees of every object: (patch order, leaf blocks), the blocks as
    (kind, t_first, t_end, s_first, s_end) in tree positions, objects in
    order."""
    n_obj = max(patch_obj) + 1
    order, blocks = [], []
    for o in range(n_obj):
        mine = [p for p in range(len(patch_obj)) if patch_obj[p] == o]
        root = build_cluster(mine, centroid, pbox, patch_nodes, upn, leaf)
        base = len(order)
        order += root.patches
        pos = {p: base + i for i, p in enumerate(root.patches)}
        for kind, t, s in block_leaves(root, root, eta, near):
            blocks.append((kind, pos[t.patches[0]], pos[t.patches[-1]] + 1, pos[s.patches[0]], pos[s.patches[-1]] + 1))
    return order, blocks


def patch_inputs(nodes_per_object, near_per_object):
    """Per-patch inputs of the builder from the node sets of the objects:
    object index, centroid (mean of the nodes), node bounding box, node
    count, and the (target patch, source patch) near pairs, with patches
    numbered across objects in order."""
    patch_obj, centroid, pbox, patch_nodes, near = [], [], [], [], set()
    base = 0
    for o, (nd, pairs) in enumerate(zip(nodes_per_object, near_per_object)):
        q2 = nd.q * nd.q
        r = np.asarray(nd.r).reshape(nd.n_patches, q2, 3)
        for p in range(nd.n_patches):
            patch_obj.append(o)
            centroid.append(tuple(float(x) for x in r[p].mean(axis=0)))
            pbox.append(tuple(float(x) for x in np.concatenate([r[p].min(axis=0), r[p].max(axis=0)])))
            patch_nodes.append(q2)
        for (t, p, _u, _v, _self) in pairs:
            near.add((base + t // q2, base + p))
        base += nd.n_patches
    return patch_obj, centroid, pbox, patch_nodes, near
