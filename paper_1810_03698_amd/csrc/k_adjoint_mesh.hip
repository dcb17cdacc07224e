// Adjoint with respect to the surface vertices.  The energy depends on the
// mesh through the operator entries (collocation points c_i, far nodes y_jq,
// normals n_j, areas A_j, near-singular and singular integrals), the
// right-hand side at the collocation points, and the readout at the sites.
// Pair sums are accumulated into per-panel gradients with respect to
// (c, y_q, n, A) -- the far-rule operator pairs directly here, or with the
// treecode's lists and expansions (k_tree.hip) when the product uses them;
// near/self corrections are differentiated directly in the vertices with
// dual numbers; a last kernel chains everything to the vertices.  All FP64.
#include <cmath>

#include "dual.hpp"
#include "kernels.hpp"
#include "tree.hpp"
#include "pair.hpp"
#include "panel.hpp"

namespace pbmp {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;
constexpr int kB = 256;
constexpr int kT = 64;

// per target panel i: d/dc_i of sum_j lambda_x . A x (far rule everywhere)
__global__ __launch_bounds__(kB) void k_op_grad_target(int N, int nf,
                                                       const double *__restrict__ src64,
                                                       const double *__restrict__ geo,
                                                       const double *__restrict__ x,
                                                       const double *__restrict__ lam,
                                                       double kappa, double eps_ratio,
                                                       RuleArgs ru, double *__restrict__ gc) {
  __shared__ double sh[kT * 15];
  const int i = blockIdx.x * kB + threadIdx.x;
  const int il = min(i, N - 1);
  const double c[3] = {geo[il], geo[N + il], geo[2 * N + il]};
  const double l1 = lam[il], l2 = lam[N + il];
  double g[3] = {0.0, 0.0, 0.0};
  for (int j0 = 0; j0 < N; j0 += kT) {
    const int nj = min(kT, N - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < nj * 15; e += kB) {
      const int j = j0 + e / 15, k = e % 15;
      const double *rec = src64 + 16 * (size_t)j;
      sh[e] = k < 12 ? rec[k] : (k == 12 ? geo[6 * N + j] : (k == 13 ? x[j] : x[N + j]));
    }
    __syncthreads();
    for (int e = 0; e < nj; ++e) {
      const double *s = sh + 15 * e;
      const double alpha = s[12] * kInv4Pi;
      const double a1 = l1 * s[13], a2 = l1 * s[14], a3 = l2 * s[13], a4 = eps_ratio * l2 * s[14];
      for (int q = 0; q < nf; ++q) {
        const double R[3] = {c[0] - s[3 * q], c[1] - s[3 * q + 1], c[2] - s[3 * q + 2]};
        double gR[3], gn[3];
        op_pair(R, s + 9, kappa, a1, a2, a3, a4, gR, gn);
        for (int d = 0; d < 3; ++d) g[d] += alpha * ru.fw[q] * gR[d];
      }
    }
  }
  if (i < N)
    for (int d = 0; d < 3; ++d) gc[3 * i + d] = g[d];
}

// per source panel j: d/dy_jq, d/dn_j, d/dA_j of sum_i lambda_x . A x
__global__ __launch_bounds__(kB) void k_op_grad_source(int N, int nf,
                                                       const double *__restrict__ src64,
                                                       const double *__restrict__ geo,
                                                       const double *__restrict__ x,
                                                       const double *__restrict__ lam,
                                                       double kappa, double eps_ratio,
                                                       RuleArgs ru, double *__restrict__ gy,
                                                       double *__restrict__ gn,
                                                       double *__restrict__ gA) {
  __shared__ double sh[kT * 5];
  const int j = blockIdx.x * kB + threadIdx.x;
  const int jl = min(j, N - 1);
  const double *rec = src64 + 16 * (size_t)jl;
  const double n[3] = {rec[9], rec[10], rec[11]};
  const double A = geo[6 * N + jl];
  const double ph = x[jl], dp = x[N + jl];
  double ay[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, an[3] = {0, 0, 0}, aA = 0.0;
  for (int i0 = 0; i0 < N; i0 += kT) {
    const int ni = min(kT, N - i0);
    __syncthreads();
    for (int e = threadIdx.x; e < ni * 5; e += kB) {
      const int i = i0 + e / 5, k = e % 5;
      sh[e] = k < 3 ? geo[k * N + i] : lam[(k - 3) * N + i];
    }
    __syncthreads();
    for (int e = 0; e < ni; ++e) {
      const double *s = sh + 5 * e;
      const double a1 = s[3] * ph, a2 = s[3] * dp, a3 = s[4] * ph, a4 = eps_ratio * s[4] * dp;
      for (int q = 0; q < nf; ++q) {
        const double R[3] = {s[0] - rec[3 * q], s[1] - rec[3 * q + 1], s[2] - rec[3 * q + 2]};
        double gR[3], gnn[3];
        const double f = op_pair(R, n, kappa, a1, a2, a3, a4, gR, gnn);
        const double w = ru.fw[q] * kInv4Pi;
        for (int d = 0; d < 3; ++d) {
          ay[3 * q + d] -= w * A * gR[d];
          an[d] += w * A * gnn[d];
        }
        aA += w * f;
      }
    }
  }
  if (j < N) {
    for (int k = 0; k < 9; ++k) gy[9 * j + k] = ay[k];
    for (int d = 0; d < 3; ++d) gn[3 * j + d] = an[d];
    gA[j] = aA;
  }
}

// Near/self correction entries (fine - far rule) differentiated in the
// target point and the source panel's vertices: ge[e][0..2] = d/dc_i,
// ge[e][3..11] = d/dv_j (for the self entry, c_i is the panel's own centroid
// and everything is carried by the vertices).
__global__ void k_near_grad(int N, const int *__restrict__ rowptr, const int *__restrict__ col,
                            const double *__restrict__ verts, const int *__restrict__ tri,
                            const double *__restrict__ geo, const double *__restrict__ x,
                            const double *__restrict__ lam, double kappa, double eps_ratio,
                            RuleArgs ru, double *__restrict__ ge) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double l1 = lam[i], l2 = lam[N + i];
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const int j = col[e];
    const double a1 = l1 * x[j], a2 = l1 * x[N + j], a3 = l2 * x[j], a4 = eps_ratio * l2 * x[N + j];
    using D = Dual<12>;
    D v[3][3], c[3], n[3], A, cj[3];
    for (int a = 0; a < 3; ++a)
      for (int d = 0; d < 3; ++d) v[a][d] = D::var(verts[3 * tri[3 * j + a] + d], 3 + 3 * a + d);
    panel_frame_t<D>(v, cj, n, A);
    if (j == i) {
      for (int d = 0; d < 3; ++d) c[d] = cj[d];
    } else {
      for (int d = 0; d < 3; ++d) c[d] = D::var(geo[d * N + i], d);
    }
    D fine[4], coarse[4];
    if (j == i) {
      singular_panel_t<D>(v, c, kappa, ru, fine[0], fine[2]);
      fine[1] = D(0.0);
      fine[3] = D(0.0);
    } else {
      panel_rule_t<D>(v, n, A, c, ru.nn, ru.nb, ru.nw, kappa, fine);
    }
    panel_rule_t<D>(v, n, A, c, ru.nf, ru.fb, ru.fw, kappa, coarse);
    const D E = a1 * (fine[1] - coarse[1]) - a2 * (fine[0] - coarse[0]) -
                a3 * (fine[3] - coarse[3]) + a4 * (fine[2] - coarse[2]);
    for (int k = 0; k < 12; ++k) ge[12 * (size_t)e + k] = E.d[k];
  }
}

// gc[i] += sum of the row's target parts; gv[j] += sum of the column's
// vertex parts (transposed lists), in a fixed order.
__global__ void k_near_grad_reduce(int N, const int *__restrict__ rowptr,
                                   const int *__restrict__ trow, const int *__restrict__ tent,
                                   const double *__restrict__ ge, double *__restrict__ gc,
                                   double *__restrict__ gv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double c[3] = {0, 0, 0};
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e)
    for (int d = 0; d < 3; ++d) c[d] += ge[12 * (size_t)e + d];
  for (int d = 0; d < 3; ++d) gc[3 * i + d] += c[d];
  double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int t = trow[i]; t < trow[i + 1]; ++t)
    for (int k = 0; k < 9; ++k) v[k] += ge[12 * (size_t)tent[t] + 3 + k];
  for (int k = 0; k < 9; ++k) gv[9 * i + k] += v[k];
}

// d/dc_i of -lambda_1 . f: -sigma_i sum_m grad phi_m(c_i)
__global__ void k_rhs_centroid_grad(int N, int M, const double *__restrict__ geo,
                                    const double *__restrict__ sigma,
                                    const double *__restrict__ xyz, const double *__restrict__ q,
                                    const double *__restrict__ p, const double *__restrict__ Q,
                                    double *__restrict__ gc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double g[3] = {0, 0, 0};
  for (int m = 0; m < M; ++m) {
    const double R[3] = {geo[i] - xyz[3 * m], geo[N + i] - xyz[3 * m + 1],
                         geo[2 * N + i] - xyz[3 * m + 2]};
    const double rr = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    const double ri = 1.0 / sqrt(rr);
    const double ri2 = ri * ri, ri3 = ri * ri2, ri5 = ri3 * ri2, ri7 = ri5 * ri2;
    const double *pm = p + 3 * m, *Qm = Q + 9 * m;
    double QR[3];
    for (int a = 0; a < 3; ++a)
      QR[a] = 0.5 * ((Qm[3 * a] + Qm[a]) * R[0] + (Qm[3 * a + 1] + Qm[3 + a]) * R[1] +
                     (Qm[3 * a + 2] + Qm[6 + a]) * R[2]);
    const double S = QR[0] * R[0] + QR[1] * R[1] + QR[2] * R[2];
    const double pR = pm[0] * R[0] + pm[1] * R[1] + pm[2] * R[2];
    for (int a = 0; a < 3; ++a)
      g[a] += -q[m] * R[a] * ri3 + pm[a] * ri3 - 3.0 * pR * R[a] * ri5 + QR[a] * ri5 -
              2.5 * S * R[a] * ri7;
  }
  for (int a = 0; a < 3; ++a) gc[3 * i + a] -= sigma[i] * g[a];
}

// Readout geometry: panel j's share sum_l W'_l . reac_l, far rule with the
// node data differentiated in (R, n); near sites with the 19-node rule
// differentiated in the vertices.
template <class S>
__device__ inline void node_data_t(const S R[3], const S n[3], S g[10], S h[10]) {
  const S rr = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
  const S i1 = 1.0 / sqrt(rr);
  const S i2 = i1 * i1, i3 = i1 * i2, i5 = i3 * i2, i7 = i5 * i2;
  const S nR = n[0] * R[0] + n[1] * R[1] + n[2] * R[2];
  g[0] = i1;
  h[0] = nR * i3;
  for (int a = 0; a < 3; ++a) {
    g[1 + a] = -R[a] * i3;
    h[1 + a] = n[a] * i3 - 3.0 * nR * R[a] * i5;
  }
  int o = 4;
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b) {
      S gg = 3.0 * R[a] * R[b] * i5;
      S hh = -3.0 * (n[a] * R[b] + n[b] * R[a]) * i5 + 15.0 * nR * R[a] * R[b] * i7;
      if (a == b) {
        gg = gg - i3;
        hh = hh - 3.0 * nR * i5;
      }
      g[o] = gg;
      h[o] = hh;
      ++o;
    }
}

template <class S>
__device__ inline S wdot(const double *W, const S v[10]) {
  S s = W[0] * v[0];
  for (int k = 1; k < 10; ++k) s = s + W[k] * v[k];
  return s;
}

__global__ __launch_bounds__(kB) void k_readout_geom_grad(
    int N, int M, int nf, const double *__restrict__ src64, const double *__restrict__ geo,
    const double *__restrict__ verts, const int *__restrict__ tri, RuleArgs ru,
    const double *__restrict__ x, const double *__restrict__ xyz, const double *__restrict__ W,
    const int *__restrict__ tsrow, const int *__restrict__ tscol, double *__restrict__ gy,
    double *__restrict__ gn, double *__restrict__ gA, double *__restrict__ gv) {
  __shared__ double sh[kT * 13];
  using D6 = Dual<6>;
  const int j = blockIdx.x * kB + threadIdx.x;
  const int jl = min(j, N - 1);
  const double *rec = src64 + 16 * (size_t)jl;
  const double A = geo[6 * N + jl];
  const double ph = x[jl], dp = x[N + jl];
  double ay[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, an[3] = {0, 0, 0}, aA = 0.0;
  for (int l0 = 0; l0 < M; l0 += kT) {
    const int nl = min(kT, M - l0);
    __syncthreads();
    for (int e = threadIdx.x; e < nl * 13; e += kB) {
      const int l = l0 + e / 13, k = e % 13;
      sh[e] = k < 3 ? xyz[3 * l + k] : W[10 * l + k - 3];
    }
    __syncthreads();
    for (int e = 0; e < nl; ++e) {
      const double *s = sh + 13 * e;
      for (int q = 0; q < nf; ++q) {
        D6 R[3], n[3];
        for (int d = 0; d < 3; ++d) {
          R[d] = D6::var(s[d] - rec[3 * q + d], d);
          n[d] = D6::var(rec[9 + d], 3 + d);
        }
        D6 g[10], h[10];
        node_data_t<D6>(R, n, g, h);
        const D6 val = dp * wdot<D6>(s + 3, g) - ph * wdot<D6>(s + 3, h);
        const double w = ru.fw[q];
        for (int d = 0; d < 3; ++d) {
          ay[3 * q + d] -= w * A * val.d[d];  // R = r_l - y
          an[d] += w * A * val.d[3 + d];
        }
        aA += w * val.v;
      }
    }
  }
  if (j >= N) return;
  for (int k = 0; k < 9; ++k) gy[9 * j + k] += ay[k];
  for (int d = 0; d < 3; ++d) gn[3 * j + d] += an[d];
  gA[j] += aA;
  // near sites: (19-node - far) rule, in the vertices
  using D9 = Dual<9>;
  D9 v[3][3], c[3], n[3], Ad;
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) v[a][d] = D9::var(verts[3 * tri[3 * j + a] + d], 3 * a + d);
  panel_frame_t<D9>(v, c, n, Ad);
  double gacc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int t = tsrow[j]; t < tsrow[j + 1]; ++t) {
    const int l = tscol[t];
    const double *Wl = W + 10 * l;
    D9 tot(0.0);
    for (int pass = 0; pass < 2; ++pass) {
      const int nq = pass ? nf : ru.nn;
      for (int q = 0; q < nq; ++q) {
        const double *b = pass ? ru.fb[q] : ru.nb[q];
        const double wq = pass ? -ru.fw[q] : ru.nw[q];
        D9 R[3];
        for (int d = 0; d < 3; ++d)
          R[d] = xyz[3 * l + d] - (b[0] * v[0][d] + b[1] * v[1][d] + b[2] * v[2][d]);
        D9 g[10], h[10];
        node_data_t<D9>(R, n, g, h);
        tot = tot + (wq * Ad) * (dp * wdot<D9>(Wl, g) - ph * wdot<D9>(Wl, h));
      }
    }
    for (int k = 0; k < 9; ++k) gacc[k] += tot.d[k];
  }
  for (int k = 0; k < 9; ++k) gv[9 * j + k] += gacc[k];
}

// chain (c, y_q, n, A) gradients of panel j to its three vertices, plus the
// direct vertex parts: out[9j..9j+8]
__global__ void k_chain_vertices(int N, int nf, const double *__restrict__ verts,
                                 const int *__restrict__ tri, RuleArgs ru,
                                 const double *__restrict__ gc, const double *__restrict__ gy,
                                 const double *__restrict__ gn, const double *__restrict__ gA,
                                 const double *__restrict__ gv, double *__restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  using D9 = Dual<9>;
  D9 v[3][3], c[3], n[3], A;
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) v[a][d] = D9::var(verts[3 * tri[3 * j + a] + d], 3 * a + d);
  panel_frame_t<D9>(v, c, n, A);
  D9 T = gA[j] * A;
  for (int d = 0; d < 3; ++d) T = T + gc[3 * j + d] * c[d] + gn[3 * j + d] * n[d];
  for (int q = 0; q < nf; ++q)
    for (int d = 0; d < 3; ++d) {
      const D9 y = ru.fb[q][0] * v[0][d] + ru.fb[q][1] * v[1][d] + ru.fb[q][2] * v[2][d];
      T = T + gy[9 * j + 3 * q + d] * y;
    }
  for (int k = 0; k < 9; ++k) out[9 * j + k] = T.d[k] + gv[9 * j + k];
}

}  // namespace

void launch_mesh_adjoint(hipStream_t s, int N, int M, int nf, const double *src64,
                         const double *geo, const double *verts, const int *tri,
                         const RuleArgs &ru, const int *rowptr, const int *col,
                         const int *trow, const int *tent, const int *tsrow,
                         const int *tscol, const double *x, const double *lam,
                         const double *sigma, const double *xyz, const double *q,
                         const double *p, const double *Q, const double *Wp, double kappa,
                         double eps_ratio, double *work, double *ge, double *out, Tree *tree,
                         double *part, double *partT) {
  // work: gc[3N] gy[9N] gn[3N] gA[N] gv[9N]
  double *gc = work, *gy = gc + 3 * (size_t)N, *gn = gy + 9 * (size_t)N,
         *gA = gn + 3 * (size_t)N, *gv = gA + N;
  PBMP_HIP(hipMemsetAsync(work, 0, sizeof(double) * 25 * (size_t)N, s));
  const dim3 g1((N + kB - 1) / kB);
  // far-rule operator entries: with the treecode's lists and expansions
  // (the derivative of the treecode operator), else every pair directly
  if (tree) {
    tree_mesh_adjoint_far(*tree, s, nf, N, geo, src64, lam, kappa, eps_ratio, part, partT, gc,
                          gy, gn, gA);
  } else {
    hipLaunchKernelGGL(k_op_grad_target, g1, dim3(kB), 0, s, N, nf, src64, geo, x, lam, kappa,
                       eps_ratio, ru, gc);
    hipLaunchKernelGGL(k_op_grad_source, g1, dim3(kB), 0, s, N, nf, src64, geo, x, lam, kappa,
                       eps_ratio, ru, gy, gn, gA);
  }
  hipLaunchKernelGGL(k_near_grad, dim3((N + 63) / 64), dim3(64), 0, s, N, rowptr, col, verts,
                     tri, geo, x, lam, kappa, eps_ratio, ru, ge);
  hipLaunchKernelGGL(k_near_grad_reduce, g1, dim3(kB), 0, s, N, rowptr, trow, tent, ge, gc,
                     gv);
  hipLaunchKernelGGL(k_rhs_centroid_grad, g1, dim3(kB), 0, s, N, M, geo, sigma, xyz, q, p, Q,
                     gc);
  hipLaunchKernelGGL(k_readout_geom_grad, g1, dim3(kB), 0, s, N, M, nf, src64, geo, verts, tri,
                     ru, x, xyz, Wp, tsrow, tscol, gy, gn, gA, gv);
  hipLaunchKernelGGL(k_chain_vertices, g1, dim3(kB), 0, s, N, nf, verts, tri, ru, gc, gy, gn,
                     gA, gv, out);
  PBMP_HIP(hipGetLastError());
}

}  // namespace pbmp
