"""The octree neighbour links the library builds (host code, no GPU), leaf by
leaf and face by face against a search of the tree from its root: the leaf
across a face at the leaf's level or coarser, or the refined node there.  A
wrong link sends a crossing into the wrong cell, so every entry is checked."""
import numpy as np
import pytest

from paper_1409_4480_amd import colt, inputs

EDGE, SEARCH, LEAF = 0xFFFFFFFF, 0xFFFFFFFE, 0x80000000


def tree_geometry(child):
    """Depth and lowest corner (in finest-cell units) of every node."""
    nn = len(child)
    depth = np.full(nn, -1)
    depth[0] = 0
    order = [0]
    for i in order:
        if child[i] >= 0:
            for o in range(8):
                depth[child[i] + o] = depth[i] + 1
                order.append(child[i] + o)
    dmax = int(depth.max())
    lo = np.zeros((nn, 3), np.int64)
    for i in order:
        if child[i] >= 0:
            half = 1 << (dmax - depth[i] - 1)
            for o in range(8):
                lo[child[i] + o] = lo[i] + half * np.array([o & 1, (o >> 1) & 1, (o >> 2) & 1])
    return depth, lo, dmax


def descend(child, lo, dmax, q, max_depth):
    """The node holding finest cell q, no deeper than max_depth."""
    node, lvl = 0, 0
    while child[node] >= 0 and lvl < max_depth:
        half = 1 << (dmax - lvl - 1)
        octant = sum(1 << d for d in range(3) if q[d] - lo[node][d] >= half)
        node = child[node] + octant
        lvl += 1
    return node, lvl


@pytest.mark.parametrize("case", ["nfw", "galaxy_like", "uniform"])
def test_links_match_a_search_of_the_tree(case):
    if case == "nfw":
        child = inputs.nfw_octree(base_level=3, max_extra=3, leaves_target=(4000, 9000),
                                  turb_n=16, n_photons=1)["grid"]["child"]
    elif case == "galaxy_like":
        child, _, _, _ = inputs.build_octree(
            np.array([-1.0, -1.0, -1.0]), 2.0, 2, 4,
            lambda c, w, l: (np.abs(np.linalg.norm(c, axis=1) - 0.5) < w) | (c[:, 2] > 0.7))
    else:
        child, _, _, _ = inputs.build_octree(np.array([0.0, 0.0, 0.0]), 1.0, 3, 0,
                                             lambda c, w, l: np.zeros(len(c), bool))
    child = np.asarray(child, np.int64)
    links = colt.octree_links(child)
    depth, lo, dmax = tree_geometry(child)
    leaves = np.flatnonzero(child < 0)
    assert links.shape == (len(leaves), 6)
    leaf_index = {int(n): j for j, n in enumerate(leaves)}
    extent = 1 << dmax
    kinds = {"edge": 0, "leaf": 0, "node": 0}
    for j, node in enumerate(leaves):
        dl = int(depth[node])
        size = 1 << (dmax - dl)
        for face in range(6):
            a = face >> 1
            q = lo[node].copy()
            q[a] = q[a] + size if face & 1 else q[a] - 1
            e = int(links[j, face])
            if q[a] < 0 or q[a] >= extent:
                assert e == EDGE, (j, face)
                kinds["edge"] += 1
                continue
            assert e != EDGE and e != SEARCH, (j, face)
            across, lvl = descend(child, lo, dmax, q, dl)
            if e & LEAF:
                assert child[across] < 0 and leaf_index[int(across)] == e & 0x7FFFFFF
                assert (e >> 27) & 15 == dl - lvl
                kinds["leaf"] += 1
            else:
                assert child[across] >= 0 and across == e and lvl == dl
                kinds["node"] += 1
    assert kinds["edge"] > 0 and kinds["leaf"] > 0
    if case != "uniform":
        assert kinds["node"] > 0       # refined neighbours occur and are descended


def test_links_reject_a_malformed_tree():
    bad = np.array([1, -1, -1, -1, -1, -1, -1, -1, 5], np.int32)   # node 8 reached twice
    with pytest.raises(RuntimeError):
        colt.octree_links(bad)
