"""Host logic of the H-matrix structure (Sec. III-A, eq. 21): the library's
tree builder, compiled here from its source with the host compiler behind a
flat-array shim, against the oracle's tree, exactly (patch order and every
leaf block); and the oracle's tree against what the method fixes whatever
the bisection rule: the leaf blocks tile each object's matrix once, every
low-rank block satisfies eq. 21 on boxes recomputed from the raw nodes and
holds no near pair, every dense block has a leaf cluster on one side."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

from oracle import geometry as G, mfie, tree as OT
from synth import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2408_17116_amd", "csrc")
SHIM = os.path.join(ROOT, "tests", "host", "tree_shim.cpp")

CASES = {
    "sphere_s3q4_leaf64": ([W.tiny_sphere(s=3, q=4, k0=3.0)], 2, 64, 1.0),
    "ellipsoid_s4q3_leaf40": ([W.ObjectSpec(axes=(2.0, 1.0, 0.5), center=(0.0, 0.0, 0.0), s=4, q=3, k0=2.0)],
                              2, 40, 1.0),
    "ellipsoid_batch3_leaf256": (W.ellipsoid_batch(3, seed=2), 2, 256, 1.0),
    "sphere_4_unknowns_per_node": ([W.tiny_sphere(s=3, q=4, k0=3.0)], 4, 128, 1.0),
    "sphere_eta_half": ([W.tiny_sphere(s=4, q=3, k0=3.0)], 2, 36, 0.5),
    # eta = 2 admits boxes closer than a patch diameter: the near-pair
    # exclusion decides blocks that eq. 21 alone would make low-rank
    "ellipsoid_eta_two": ([W.ObjectSpec(axes=(2.0, 1.0, 0.5), center=(0.0, 0.0, 0.0), s=4, q=3, k0=2.0)],
                          2, 18, 2.0),
}


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("tree") / "libtreeshim.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, SHIM,
                    os.path.join(CSRC, "tree.cpp"), "-o", out], check=True)
    lib = C.CDLL(out)
    ip, dp = C.POINTER(C.c_int), C.POINTER(C.c_double)
    lib.tree_leaves.argtypes = [C.c_int, C.c_int, C.c_int, ip, ip, dp, dp, ip, ip, C.c_int, C.c_double, ip, ip,
                                C.c_int]
    lib.tree_leaves.restype = C.c_int
    lib.component_leaves.argtypes = lib.tree_leaves.argtypes[:-3] + [ip, C.c_int]
    lib.component_leaves.restype = C.c_int
    return lib


_cache = {}


def _case(name):
    if name not in _cache:
        specs, upn, leaf, eta = CASES[name]
        nds = [G.build_nodes(s) for s in specs]
        pairs = [mfie.near_pairs(nd) for nd in nds]
        _cache[name] = (nds, OT.patch_inputs(nds, pairs), upn, leaf, eta)
    return _cache[name]


def _library_tree(lib, inp, upn, leaf, eta):
    patch_obj, centroid, pbox, patch_nodes, near = inp
    P = len(patch_obj)
    lists = [sorted(b for (a, b) in near if a == p) for p in range(P)]
    ptr = np.zeros(P + 1, np.int32)
    ptr[1:] = np.cumsum([len(v) for v in lists])
    idx = np.array([b for v in lists for b in v], np.int32)
    a = lambda x, t: np.ascontiguousarray(x, dtype=t)
    po, cn, pb, pn = a(patch_obj, np.int32), a(centroid, np.float64), a(pbox, np.float64), a(patch_nodes, np.int32)
    order = np.zeros(P, np.int32)
    cap = 4 * P * P
    blocks = np.zeros(5 * cap, np.int32)
    ip = lambda x: x.ctypes.data_as(C.POINTER(C.c_int))
    dp = lambda x: x.ctypes.data_as(C.POINTER(C.c_double))
    n = lib.tree_leaves(P, max(patch_obj) + 1, upn, ip(po), ip(pn), dp(cn), dp(pb), ip(ptr), ip(idx), leaf, eta,
                        ip(order), ip(blocks), cap)
    assert n > 0
    kinds = {1: "lr", 0: "dense"}
    return list(order), [(kinds[b[0]], *map(int, b[1:])) for b in blocks[:5 * n].reshape(n, 5)]


@pytest.mark.parametrize("name", list(CASES))
def test_library_tree_equals_oracle_tree(shim, name):
    _nds, inp, upn, leaf, eta = _case(name)
    order_o, blocks_o = OT.build(inp[0], inp[1], inp[2], inp[3], inp[4], upn, leaf, eta)
    order_l, blocks_l = _library_tree(shim, inp, upn, leaf, eta)
    n_lr = sum(b[0] == "lr" for b in blocks_o)
    print(f"{name}: {len(order_o)} patches, {len(blocks_o)} leaf blocks ({n_lr} low-rank)")
    assert order_l == order_o
    assert blocks_l == blocks_o


@pytest.mark.parametrize("name", list(CASES))
def test_oracle_tree_tiles_the_matrix_with_admissible_low_rank_blocks(name):
    nds, inp, upn, leaf, eta = _case(name)
    patch_obj, _centroid, _pbox, patch_nodes, near = inp
    order, blocks = OT.build(patch_obj, inp[1], inp[2], patch_nodes, near, upn, leaf, eta)
    P = len(order)
    assert sorted(order) == list(range(P))
    # raw node coordinates per original patch, across objects
    pts = []
    for nd in nds:
        q2 = nd.q * nd.q
        pts += [np.asarray(nd.r)[p * q2:(p + 1) * q2] for p in range(nd.n_patches)]
    cover = np.zeros((P, P), np.int32)
    n_lr = 0
    for kind, t0, t1, s0, s1 in blocks:
        tp, sp = order[t0:t1], order[s0:s1]
        assert len({patch_obj[p] for p in tp + sp}) == 1          # within one object
        cover[t0:t1, s0:s1] += 1
        if kind == "lr":
            n_lr += 1
            bt, bs = np.concatenate([pts[p] for p in tp]), np.concatenate([pts[p] for p in sp])
            lo_t, hi_t, lo_s, hi_s = bt.min(0), bt.max(0), bs.min(0), bs.max(0)
            gap = np.maximum(0.0, np.maximum(lo_t - hi_s, lo_s - hi_t))
            dist = np.linalg.norm(gap)
            assert dist > 0.0
            assert min(np.linalg.norm(hi_t - lo_t), np.linalg.norm(hi_s - lo_s)) <= eta * dist * (1 + 1e-12)
            assert not any((a, b) in near for a in tp for b in sp)
        else:
            small = lambda ps: len(ps) == 1 or upn * sum(patch_nodes[p] for p in ps) <= leaf
            assert small(tp) or small(sp)
    same_obj = np.equal.outer([patch_obj[p] for p in order], [patch_obj[p] for p in order])
    assert (cover[same_obj] == 1).all() and (cover[~same_obj] == 0).all()
    assert n_lr > 0


@pytest.mark.parametrize("name", ["sphere_s3q4_leaf64", "sphere_4_unknowns_per_node", "ellipsoid_batch3_leaf256"])
def test_component_wise_structure_tiles_the_permuted_matrix(shim, name):
    """The component-wise ordering (Sec. III-A, eqs. 22-23): every leaf of
    the node tree gives one leaf per pair of components, holding exactly the
    rows of its row component and the columns of its column component in the
    component-by-component order, so the leaves tile each object's permuted
    matrix once; the pivots are the leaves of one component against itself
    on the node tree's diagonal leaves."""
    _nds, inp, upn, leaf, eta = _case(name)
    patch_obj, centroid, pbox, patch_nodes, near = inp
    order, blocks = _library_tree(shim, inp, upn, leaf, eta)
    P = len(patch_obj)
    lists = [sorted(b for (a, b) in near if a == p) for p in range(P)]
    ptr = np.zeros(P + 1, np.int32)
    ptr[1:] = np.cumsum([len(v) for v in lists])
    idx = np.array([b for v in lists for b in v], np.int32)
    a_ = lambda x, t: np.ascontiguousarray(x, dtype=t)
    po, cn, pb, pn = a_(patch_obj, np.int32), a_(centroid, np.float64), a_(pbox, np.float64), a_(patch_nodes, np.int32)
    cap = upn * upn * len(blocks) + 1
    out = np.zeros(13 * cap, np.int32)
    ip = lambda x: x.ctypes.data_as(C.POINTER(C.c_int))
    dp = lambda x: x.ctypes.data_as(C.POINTER(C.c_double))
    n = shim.component_leaves(P, max(patch_obj) + 1, upn, ip(po), ip(pn), dp(cn), dp(pb), ip(ptr), ip(idx), leaf, eta,
                              ip(out), cap)
    assert n == upn * upn * len(blocks)
    L = out[:13 * n].reshape(n, 13)
    # tree-order node ranges of the objects
    node0 = np.concatenate([[0], np.cumsum([patch_nodes[p] for p in order])])
    objs = sorted(set(patch_obj))
    orng = {}
    for pos, p in enumerate(order):
        o = patch_obj[p]
        lo, hi = orng.get(o, (node0[pos], node0[pos + 1]))
        orng[o] = (min(lo, node0[pos]), max(hi, node0[pos + 1]))
    N = upn * node0[-1]
    cover = np.zeros((N, N), np.int8)
    n_diag = 0
    for (kind, r0, m, c0, nc, skind, tn0, tn, sn0, sn, a, b, diag) in L:
        assert kind == skind
        o = next(o for o in objs if orng[o][0] <= tn0 < orng[o][1])
        on0, on1 = orng[o]
        assert on0 <= sn0 and sn0 + sn <= on1                    # within one object
        base, no = upn * on0, on1 - on0
        assert (r0, m) == (base + a * no + tn0 - on0, tn)
        assert (c0, nc) == (base + b * no + sn0 - on0, sn)
        assert diag == (a == b and tn0 == sn0 and tn == sn)
        n_diag += int(diag)
        cover[r0:r0 + m, c0:c0 + nc] += 1
    for o in objs:
        lo, hi = upn * orng[o][0], upn * orng[o][1]
        assert (cover[lo:hi, lo:hi] == 1).all()
    assert cover.sum() == sum((upn * (orng[o][1] - orng[o][0])) ** 2 for o in objs)
    n_node_diag = sum(1 for (k, t0, t1, s0, s1) in blocks if k == "dense" and (t0, t1) == (s0, s1))
    assert n_diag == upn * n_node_diag
