"""Treecode operator product (section "The treecode algorithm"), written
plainly from the oracle's own pieces.  Test infrastructure only.

For every target leaf T of the octree (``oracle.tree``) and every target
collocation point x in it, each of the four far-field sums
    S_VL = sum_g sV_g G_L(x, y_g),      S_KL = sum_g sK_g n_g . grad_y G_L(x, y_g)
    S_VY = sum_g sV_g G_Y(x, y_g),      S_KY = sum_g sK_g n_g . grad_y G_Y(x, y_g)
(far-rule nodes y_g of panel j, sV_g = w_g A_j dphi_j, sK_g = w_g A_j phi_j,
G = 1/(4 pi r) and exp(-kappa r)/(4 pi r)) is split by T's lists:
  * boxes B accepted by the MAC: the Taylor series of G in the source point
    about B's centre c_B, G(x, c_B + h) = sum_k a_k(x - c_B) h^k, gives
        sum_{g in B} sV_g G(x, y_g) ~ sum_{|k| <= P} a_k m_k(B),
        m_k(B) = sum_{g in B} sV_g h_g^k,
        sum_{g in B} sK_g n_g . grad_y G(x, y_g) ~ sum_{|k| <= PK} a_k mK_k(B),
        mK_k(B) = sum_{g in B} sK_g sum_a k_a n_a h_g^(k - e_a)
    with a_k from the power series of ``oracle.taylor`` (not from the
    recurrences the paper cites);
  * leaves in the direct list: the far rule, pair by pair.
The product then adds the near-field corrections (singular and
near-singular pairs: the method's entry minus the far-rule entry), which
``bie.Mesh.near_correction_sums`` evaluates pair by pair, and combines the
sums as in eq. integral_eq.

PK is the order of the double-layer expansion.  The double-layer moment of
degree |k| holds h^(|k|-1), so PK = P would truncate the double layer one
degree below the single layer.  The reading taken (the paper names one
expansion order for both kernels): PK = P + 1, both layers carried to
degree P in the source displacement h.  ``double_layer_order`` selects
another PK (used to measure what the extra degree buys).
"""

import numpy as np

from . import bie, geometry, quadrature, taylor, tree

FOUR_PI = 4.0 * np.pi


def far_nodes(mesh, far=3):
    """Far-rule nodes [N, nq, 3] and weights [nq] of every panel."""
    bary, w = quadrature.far_rule(far)
    return geometry.quad_points(mesh.geo, bary), np.asarray(w)


def _direct_far(xt, ys, nys, sv, sk, kappa):
    """Far-rule sums [nt, 4] of targets xt [nt,3] over nodes ys [ns,3]
    with node normals nys, strengths sv, sk."""
    R = xt[:, None, :] - ys[None, :, :]
    r = np.sqrt(np.einsum("tsd,tsd->ts", R, R))
    nR = np.einsum("tsd,sd->ts", R, nys)
    e = np.exp(-kappa * r)
    out = np.empty((len(xt), 4))
    out[:, 0] = (sv[None, :] / (FOUR_PI * r)).sum(1)
    out[:, 1] = (sk[None, :] * nR / (FOUR_PI * r ** 3)).sum(1)
    out[:, 2] = (sv[None, :] * e / (FOUR_PI * r)).sum(1)
    out[:, 3] = (sk[None, :] * nR * (1.0 + kappa * r) * e / (FOUR_PI * r ** 3)).sum(1)
    return out


class Treecode:
    """Octree, lists and far-rule data of one mesh for the oracle product."""

    def __init__(self, mesh, theta, P, leaf, far=3, double_layer_order=None):
        self.mesh, self.theta, self.P, self.leaf = mesh, float(theta), int(P), int(leaf)
        self.PK = self.P + 1 if double_layer_order is None else int(double_layer_order)
        self.nodes, self.w = far_nodes(mesh, far)
        self.boxes = tree.build(mesh.cen, self.nodes, leaf)
        self.lists = tree.lists(self.boxes, theta)

    def far_sums(self, phi, dphi, rows=None):
        """Treecode far-field sums (no near-field corrections): [N, 4], or
        [len(rows), 4] for the target panels ``rows`` only."""
        m = self.mesh
        N, nq = m.N, len(self.w)
        kappa = m.kappa
        wa = self.w[None, :] * m.area[:, None]                  # [N, nq]
        sv = (wa * np.asarray(dphi)[:, None]).reshape(-1)
        sk = (wa * np.asarray(phi)[:, None]).reshape(-1)
        ys = self.nodes.reshape(-1, 3)
        nys = np.repeat(m.nrm, nq, axis=0)
        Pm = max(self.P, self.PK)
        ks = taylor.multi_indices(Pm)
        nV = len(taylor.multi_indices(self.P))
        nK = len(taylor.multi_indices(self.PK))
        moments = {}

        def box_moments(b):
            if b not in moments:
                B = self.boxes[b]
                g = (np.asarray(B["panels"])[:, None] * nq + np.arange(nq)[None, :]).reshape(-1)
                mv, mk = taylor.moments(ys[g], nys[g], sv[g], sk[g], B["centre"], Pm)
                moments[b] = (mv[:nV], mk[:nK])
            return moments[b]

        out = np.zeros((N, 4))
        keep = np.ones(N, bool) if rows is None else np.isin(np.arange(N), rows)
        pairs_t, pairs_b = [], []
        for t, (m2p, p2p) in self.lists.items():
            T = np.asarray(self.boxes[t]["panels"])
            T = T[keep[T]]
            if len(T) == 0:
                continue
            if p2p:
                src = np.concatenate([np.asarray(self.boxes[b]["panels"]) for b in p2p])
                g = (src[:, None] * nq + np.arange(nq)[None, :]).reshape(-1)
                out[T] += _direct_far(m.cen[T], ys[g], nys[g], sv[g], sk[g], kappa)
            for b in m2p:
                pairs_t.append(T)
                pairs_b.append(np.full(len(T), b))
        if pairs_t:
            ti = np.concatenate(pairs_t)
            bi = np.concatenate(pairs_b)
            centres = np.array([self.boxes[b]["centre"] for b in range(len(self.boxes))])
            chunk = 20000
            for s in range(0, len(ti), chunk):
                tt, bb = ti[s:s + chunk], bi[s:s + chunk]
                D = m.cen[tt] - centres[bb]
                aL = taylor.laplace_coefficients_batch(D, Pm)
                aY = taylor.yukawa_coefficients_batch(D, Pm, kappa) if kappa > 0 else aL
                mv = np.stack([box_moments(b)[0] for b in bb], axis=1)   # [nV, n]
                mk = np.stack([box_moments(b)[1] for b in bb], axis=1)   # [nK, n]
                contrib = np.stack([(aL[:nV] * mv).sum(0), (aL[:nK] * mk).sum(0),
                                    (aY[:nV] * mv).sum(0), (aY[:nK] * mk).sum(0)],
                                   axis=1) / FOUR_PI
                np.add.at(out, tt, contrib)
        return out if rows is None else out[np.asarray(rows)]

    def operator_sums(self, phi, dphi, rows=None):
        """Treecode sums including the near-field corrections ([N, 4], or
        [len(rows), 4] for the target panels ``rows``)."""
        far = self.far_sums(phi, dphi, rows)
        if rows is None:
            return far + self.mesh.near_correction_sums(phi, dphi)
        near = np.concatenate([self.mesh.near_correction_sums(phi, dphi, rows=(int(i), int(i) + 1))
                               for i in rows])
        return far + near

    def matvec(self, x, eps_in, eps_out, rows=None):
        """y = A x with the treecode operator; with ``rows``, the entries
        [y1[rows], y2[rows]] only."""
        N = self.mesh.N
        s = self.operator_sums(x[:N], x[N:], rows)
        phi = x[:N] if rows is None else x[:N][np.asarray(rows)]
        return bie.system_apply(s, phi, eps_in, eps_out)


def matvec(mesh, x, eps_in, eps_out, theta, P, leaf, double_layer_order=None):
    return Treecode(mesh, theta, P, leaf, double_layer_order=double_layer_order).matvec(
        x, eps_in, eps_out)
