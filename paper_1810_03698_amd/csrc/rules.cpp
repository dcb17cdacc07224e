// Quadrature rules of the boundary-element discretisation (section "The
// boundary element method"): a low-order far-field rule (1 or 3 nodes), a
// 19-node near-singular rule, and Gauss-Legendre nodes for the edge
// integrals of the singular panel.  The paper prints none of the nodes; the
// 19-node rule is read as the fully symmetric degree-9 rule with orbits
// 1 + 4 x (a,a,1-2a) + 1 x (a,b,1-a-b), whose 12 parameters are fixed here
// by Gauss-Newton on the moment equations of all monomials of degree <= 9.
#include <cmath>
#include <cstring>
#include <utility>

#include "common.hpp"

namespace pbmp {

TriRule far_rule(int k) {
  TriRule r;
  if (k == 1) {
    r.n = 1;
    r.b[0][0] = r.b[0][1] = r.b[0][2] = 1.0 / 3.0;
    r.w[0] = 1.0;
  } else if (k == 3) {
    r.n = 3;
    for (int i = 0; i < 3; ++i) {
      for (int j = 0; j < 3; ++j) r.b[i][j] = (i == j) ? 2.0 / 3.0 : 1.0 / 6.0;
      r.w[i] = 1.0 / 3.0;
    }
  } else {
    throw Error(PBMP_EARG, "gauss_far must be 1 or 3");
  }
  return r;
}

namespace {

// The moment system is ill-conditioned (smallest singular value ~1e-6), so
// a solution whose residual is at double rounding can still be ~1e-11 away
// from the rule.  Gauss-Newton therefore runs in binary128 arithmetic, and
// every barycentric coordinate is rounded to double only at the end.
using Q = __float128;

Q qabs(Q x) { return x < 0 ? -x : x; }

// (1/area) * integral of x^i y^j over the triangle (0,0),(1,0),(0,1)
//   = 2 i! j! / (i + j + 2)!
Q moment(int i, int j) {
  Q num = 2, den = 1;
  for (int k = 2; k <= i; ++k) num *= k;
  for (int k = 2; k <= j; ++k) num *= k;
  for (int k = 2; k <= i + j + 2; ++k) den *= k;
  return num / den;
}

struct Node {
  Q x, y, w;
  Q dx[12], dy[12], dw[12];  // derivatives w.r.t. the 12 parameters
};

// Expand parameters t = [w0, (a_k, w_k) k=0..3, a, b, w] into 19 nodes.
void expand(const Q *t, Node *nd) {
  for (int p = 0; p < 19; ++p) {
    nd[p].x = nd[p].y = nd[p].w = 0;
    for (int k = 0; k < 12; ++k) nd[p].dx[k] = nd[p].dy[k] = nd[p].dw[k] = 0;
  }
  int p = 0;
  nd[p].x = nd[p].y = Q(1) / 3;
  nd[p].w = t[0];
  nd[p].dw[0] = 1;
  ++p;
  for (int k = 0; k < 4; ++k) {
    const int ia = 1 + 2 * k, iw = 2 + 2 * k;
    const Q a = t[ia], w = t[iw];
    // barycentric (l1,l2,l3); (x,y) = (l2,l3)
    const Q bx[3] = {a, 1 - 2 * a, a};
    const Q by[3] = {1 - 2 * a, a, a};
    const int dbx[3] = {1, -2, 1};
    const int dby[3] = {-2, 1, 1};
    for (int q = 0; q < 3; ++q, ++p) {
      nd[p].x = bx[q];
      nd[p].y = by[q];
      nd[p].w = w;
      nd[p].dx[ia] = dbx[q];
      nd[p].dy[ia] = dby[q];
      nd[p].dw[iw] = 1;
    }
  }
  const Q a = t[9], b = t[10], w = t[11], c = 1 - a - b;
  // the six permutations of (a, b, c) as (l1, l2, l3)
  const Q L[6][3] = {{a, b, c}, {a, c, b}, {b, a, c},
                     {b, c, a}, {c, a, b}, {c, b, a}};
  // d(l)/da and d(l)/db for each slot
  const int DA[6][3] = {{1, 0, -1}, {1, -1, 0}, {0, 1, -1},
                        {0, -1, 1}, {-1, 1, 0}, {-1, 0, 1}};
  const int DB[6][3] = {{0, 1, -1}, {0, -1, 1}, {1, 0, -1},
                        {1, -1, 0}, {-1, 0, 1}, {-1, 1, 0}};
  for (int q = 0; q < 6; ++q, ++p) {
    nd[p].x = L[q][1];
    nd[p].y = L[q][2];
    nd[p].w = w;
    nd[p].dx[9] = DA[q][1];
    nd[p].dy[9] = DA[q][2];
    nd[p].dx[10] = DB[q][1];
    nd[p].dy[10] = DB[q][2];
    nd[p].dw[11] = 1;
  }
}

Q ipow(Q x, int k) {
  Q r = 1;
  for (int i = 0; i < k; ++i) r *= x;
  return r;
}

// Solve the n x n system A z = rhs by Gaussian elimination with pivoting.
void solve_dense(int n, Q *A, Q *rhs) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (qabs(A[r * n + c]) > qabs(A[piv * n + c])) piv = r;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(rhs[c], rhs[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      Q f = A[r * n + c] / A[c * n + c];
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      rhs[r] -= f * rhs[c];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    Q s = rhs[c];
    for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * rhs[k];
    rhs[c] = s / A[c * n + c];
  }
}

}  // namespace

TriRule near_rule19() {
  // rough starting point; Gauss-Newton converges to the unique nearby
  // solution with positive weights and interior nodes
  const double t0[12] = {0.1, 0.49, 0.03, 0.44, 0.08, 0.19, 0.08, 0.045, 0.025,
                         0.037, 0.22, 0.043};
  Q t[12];
  for (int k = 0; k < 12; ++k) t[k] = t0[k];
  const int deg = 9;
  Node nd[19];
  Q maxres = 1;
  for (int it = 0; it < 100; ++it) {
    expand(t, nd);
    Q JtJ[144], Jtr[12];
    for (int k = 0; k < 144; ++k) JtJ[k] = 0;
    for (int k = 0; k < 12; ++k) Jtr[k] = 0;
    maxres = 0;
    for (int i = 0; i <= deg; ++i)
      for (int j = 0; i + j <= deg; ++j) {
        Q r = -moment(i, j);
        Q J[12];
        for (int k = 0; k < 12; ++k) J[k] = 0;
        for (int p = 0; p < 19; ++p) {
          const Q xi = ipow(nd[p].x, i), yj = ipow(nd[p].y, j);
          r += nd[p].w * xi * yj;
          const Q dxi = i ? i * ipow(nd[p].x, i - 1) : Q(0);
          const Q dyj = j ? j * ipow(nd[p].y, j - 1) : Q(0);
          for (int k = 0; k < 12; ++k)
            J[k] += nd[p].dw[k] * xi * yj +
                    nd[p].w * (dxi * nd[p].dx[k] * yj + xi * dyj * nd[p].dy[k]);
        }
        if (qabs(r) > maxres) maxres = qabs(r);
        for (int a = 0; a < 12; ++a) {
          Jtr[a] -= J[a] * r;
          for (int b = 0; b < 12; ++b) JtJ[a * 12 + b] += J[a] * J[b];
        }
      }
    if (maxres < Q(1e-30)) break;
    solve_dense(12, JtJ, Jtr);
    for (int k = 0; k < 12; ++k) t[k] += Jtr[k];
  }
  expand(t, nd);
  TriRule r;
  r.n = 19;
  for (int p = 0; p < 19; ++p) {
    r.b[p][0] = (double)(1 - nd[p].x - nd[p].y);
    r.b[p][1] = (double)nd[p].x;
    r.b[p][2] = (double)nd[p].y;
    r.w[p] = (double)nd[p].w;
    if (!(r.w[p] > 0.0 && r.b[p][0] > 0.0 && r.b[p][1] > 0.0 && r.b[p][2] > 0.0))
      throw Error(PBMP_EARG, "near-singular rule: Gauss-Newton left the admissible set");
  }
  if (!(maxres < Q(1e-28))) throw Error(PBMP_EARG, "near-singular rule did not converge");
  return r;
}

void gauss_legendre(int n, double *x, double *w) {
  // Newton on P_n from the Tricomi-type initial guess
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        // one more evaluation at the converged node for the weight
        p0 = 1.0;
        p1 = z;
        for (int k = 2; k <= n; ++k) {
          double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        break;
      }
    }
    x[i] = -z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

}  // namespace pbmp
