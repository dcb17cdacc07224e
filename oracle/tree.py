"""Octree and interaction lists of the treecode (section "The treecode
algorithm"), written plainly for checking the library's tree.  Test
infrastructure only.

Readings (shared with the library, stated once here):
  * panels are binned by their centroids on a 2^21 grid over the bounding
    cube (per-axis minimum, largest extent); a cell is split into its eight
    octants while it holds more than `leaf` panels (the leaf size counts
    panels, so a panel's far nodes stay together);
  * a box's expansion centre is the midpoint of the bounding box of its
    panels' far nodes, R_B the largest node distance from it; R_T the
    largest centroid distance of a target leaf from its own centre;
  * lists are built per target leaf T by descending from the root: a box B
    is accepted (M2P) when |c_B - c_T| - R_T > 0 and R_B < theta (|c_B - c_T|
    - R_T); a leaf that fails goes to the P2P list; other boxes are opened.
    Acceptance implies the paper's per-target criterion R_B / |x - c_B| <
    theta for every target x of T.

Boxes are returned as sets of user panel indices so that a comparison does
not depend on how either side numbers them.
"""

import numpy as np

LEVELS = 21


def quantise(cen):
    """Integer grid coordinates [N, 3] of the centroids."""
    lo = cen.min(axis=0)
    ext = max(float((cen.max(axis=0) - lo).max()), 1e-12)
    u = (cen - lo) / ext
    return np.minimum(2 ** LEVELS - 1, np.maximum(0, np.floor(u * 2 ** LEVELS))).astype(np.int64)


def octant(qj, level):
    """Child octant of grid point qj at depth `level` (1-based)."""
    s = LEVELS - level
    return ((qj[0] >> s) & 1) << 2 | ((qj[1] >> s) & 1) << 1 | ((qj[2] >> s) & 1)


def build(cen, nodes, leaf):
    """Octree over panels.  cen [N,3] centroids, nodes [N, nf, 3] far nodes.
    Returns a list of boxes, each a dict with panels (sorted user indices),
    children (box indices), level, centre, R (node radius), RT (centroid
    radius)."""
    q = quantise(cen)
    boxes = []

    def make(panels, level):
        b = len(boxes)
        boxes.append({"panels": panels, "children": [], "level": level})
        if len(panels) > leaf and level < LEVELS:
            groups = {}
            for j in panels:
                groups.setdefault(octant(q[j], level + 1), []).append(j)
            kids = []
            for o in sorted(groups):
                kids.append(make(groups[o], level + 1))
            boxes[b]["children"] = kids
        return b

    make(list(range(len(cen))), 0)
    for b in boxes:
        nd = nodes[b["panels"]].reshape(-1, 3)
        c = 0.5 * (nd.min(axis=0) + nd.max(axis=0))
        b["centre"] = c
        b["R"] = float(np.sqrt(((nd - c) ** 2).sum(axis=1).max()))
        b["RT"] = float(np.sqrt(((cen[b["panels"]] - c) ** 2).sum(axis=1).max()))
    return boxes


def lists(boxes, theta):
    """Per target leaf (box index): (M2P box indices, P2P leaf indices)."""
    out = {}
    for t, T in enumerate(boxes):
        if T["children"]:
            continue
        m2p, p2p = [], []
        stack = [0]
        while stack:
            b = stack.pop()
            B = boxes[b]
            sep = float(np.linalg.norm(B["centre"] - T["centre"])) - T["RT"]
            if sep > 0.0 and B["R"] < theta * sep:
                m2p.append(b)
            elif not B["children"]:
                p2p.append(b)
            else:
                stack.extend(reversed(B["children"]))
        out[t] = (m2p, p2p)
    return out
