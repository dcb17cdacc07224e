// Integrals over one flat panel, templated on the scalar type so that the
// adjoint can differentiate them (dual numbers) with respect to the panel
// vertices and the target point.  Integral-equation normalisation
// (G = 1/(4 pi r)).
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "dual.hpp"

namespace pbmp {

constexpr double kPanelInv4Pi = 0.07957747154594767;

// V_L and V_Y of a flat panel seen from a point c lying inside it.  The
// panel is split at c into three sub-triangles; for edge (a, b) at distance h
// from c, with s the signed coordinate along the edge from the foot of the
// perpendicular, the radial integral is done in closed form:
//   int 1/(4 pi r) dA         = 1/(4 pi) h [asinh(s_b/h) - asinh(s_a/h)],
//   int e^{-k r}/(4 pi r) dA  = 1/(4 pi) int (1 - e^{-k rho})/k dtheta,
// rho = h / cos(theta) the distance to the edge.  The Yukawa remainder
// (1 - e^{-k rho})/k - rho is integrated over u = asinh(s/h) (rho = h cosh u,
// dtheta = du / cosh u) with Gauss-Legendre nodes along the edge.
template <class S>
__device__ inline void singular_panel_t(const S v[3][3], const S c[3], double kappa,
                                        const RuleArgs &ru, S &VL, S &VY) {
  S lap(0.0), rem(0.0);
  for (int e = 0; e < 3; ++e) {
    const S *a = v[e];
    const S *b = v[e == 2 ? 0 : e + 1];
    const S ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const S len = sqrt(ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2]);
    const S t[3] = {ab[0] / len, ab[1] / len, ab[2] / len};
    const S ca[3] = {a[0] - c[0], a[1] - c[1], a[2] - c[2]};
    const S sa = ca[0] * t[0] + ca[1] * t[1] + ca[2] * t[2];
    const S sb = sa + len;
    // h = |ca x t|
    const S x0 = ca[1] * t[2] - ca[2] * t[1];
    const S x1 = ca[2] * t[0] - ca[0] * t[2];
    const S x2 = ca[0] * t[1] - ca[1] * t[0];
    const S h = sqrt(x0 * x0 + x1 * x1 + x2 * x2);
    const S ua = asinh(sa / h), ub = asinh(sb / h);
    lap = lap + h * (ub - ua);
    if (kappa > 0.0) {
      const S half = 0.5 * (ub - ua), mid = 0.5 * (ub + ua);
      S acc(0.0);
      for (int g = 0; g < ru.ngl; ++g) {
        const S u = mid + half * ru.glx[g];
        const S ch = cosh(u);
        const S rho = h * ch;
        acc = acc + ru.glw[g] * ((-1.0 / kappa) * expm1(-kappa * rho) - rho) / ch;
      }
      rem = rem + half * acc;
    }
  }
  VL = lap * kPanelInv4Pi;
  VY = (lap + rem) * kPanelInv4Pi;
}

// (V_L, K_L, V_Y, K_Y) of panel v (normal n, area A) at point x with the
// nq-node rule (b, w).
template <class S>
__device__ inline void panel_rule_t(const S v[3][3], const S n[3], const S &A,
                                    const S x[3], int nq, const double (*b)[3],
                                    const double *w, double kappa, S out[4]) {
  S vl(0.0), kl(0.0), vy(0.0), ky(0.0);
  for (int q = 0; q < nq; ++q) {
    S R[3];
    for (int d = 0; d < 3; ++d)
      R[d] = x[d] - (b[q][0] * v[0][d] + b[q][1] * v[1][d] + b[q][2] * v[2][d]);
    const S r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    const S r = sqrt(r2);
    const S inv = 1.0 / r;
    const S inv3 = inv / r2;
    const S nR = n[0] * R[0] + n[1] * R[1] + n[2] * R[2];
    const S ek = exp(-kappa * r);
    const S wA = w[q] * A;
    vl = vl + wA * inv;
    kl = kl + wA * nR * inv3;
    vy = vy + wA * ek * inv;
    ky = ky + wA * nR * (1.0 + kappa * r) * ek * inv3;
  }
  out[0] = vl * kPanelInv4Pi;
  out[1] = kl * kPanelInv4Pi;
  out[2] = vy * kPanelInv4Pi;
  out[3] = ky * kPanelInv4Pi;
}

// centroid, unit normal and area of a panel from its vertices
template <class S>
__device__ inline void panel_frame_t(const S v[3][3], S c[3], S n[3], S &A) {
  const S e1[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
  const S e2[3] = {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
  const S cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                   e1[0] * e2[1] - e1[1] * e2[0]};
  const S nn = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
  for (int d = 0; d < 3; ++d) {
    c[d] = (v[0][d] + v[1][d] + v[2][d]) / 3.0;
    n[d] = cr[d] / nn;
  }
  A = 0.5 * nn;
}

}  // namespace pbmp
