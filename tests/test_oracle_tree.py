"""Pins of the oracle's octree and interaction lists against what the
treecode section requires of them: for every target leaf the accepted boxes
and the direct leaves partition the sources exactly once, every accepted
box satisfies the paper's per-target acceptance criterion for every target
of the leaf, leaves respect the size limit, and boxes are octree cells.
CPU only."""

import numpy as np
import pytest

from oracle import tree
from synth import workload


def _mesh(name):
    w = workload(name)
    v = w["verts"][w["tris"]]
    cen = v.mean(axis=1)
    bary = np.array([[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])
    nodes = np.einsum("qk,jkd->jqd", bary, v)
    return cen, nodes


@pytest.fixture(scope="module")
def sphere():
    return _mesh("sphere_5120")


@pytest.mark.parametrize("leaf,theta", [(64, 0.5), (300, 0.5), (40, 0.8)])
def test_lists_partition_sources_and_meet_mac(sphere, leaf, theta):
    cen, nodes = sphere
    N = len(cen)
    boxes = tree.build(cen, nodes, leaf)
    L = tree.lists(boxes, theta)
    n_m2p = 0
    for t, (m2p, p2p) in L.items():
        T = boxes[t]
        cover = np.zeros(N, dtype=int)
        for b in m2p + p2p:
            cover[boxes[b]["panels"]] += 1
        assert (cover == 1).all()
        for b in p2p:
            assert not boxes[b]["children"]
        x = cen[T["panels"]]
        for b in m2p:
            B = boxes[b]
            dist = np.linalg.norm(x - B["centre"], axis=1)
            assert (B["R"] < theta * dist).all()
        n_m2p += len(m2p)
    assert n_m2p > 0


def test_boxes_are_octree_cells(sphere):
    cen, nodes = sphere
    q = tree.quantise(cen)
    boxes = tree.build(cen, nodes, 64)
    for b in boxes:
        P = b["panels"]
        if b["children"]:
            assert len(P) > 64
            kids = sorted(j for c in b["children"] for j in boxes[c]["panels"])
            assert kids == sorted(P)
        else:
            assert len(P) <= 64
        # one cell: every panel shares the grid prefix of its level
        s = tree.LEVELS - b["level"]
        pref = q[P] >> s
        assert (pref == pref[0]).all()
        # radii bound every node / centroid
        nd = nodes[P].reshape(-1, 3)
        assert np.linalg.norm(nd - b["centre"], axis=1).max() <= b["R"] * (1 + 1e-15)
        assert np.linalg.norm(cen[P] - b["centre"], axis=1).max() <= b["RT"] * (1 + 1e-15)


def test_theta_zero_is_all_direct(sphere):
    cen, nodes = sphere
    boxes = tree.build(cen, nodes, 64)
    for m2p, p2p in tree.lists(boxes, 1e-9).values():
        assert m2p == []
        assert sum(len(boxes[b]["panels"]) for b in p2p) == len(cen)
