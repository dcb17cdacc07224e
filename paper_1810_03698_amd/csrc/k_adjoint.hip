// Adjoint (backward) kernels of the solvation energy.  The converged forward
// state satisfies
//   vacuum:    mu_v = alpha (E_perm + T mu_v)
//   dissolved: A x = [f(d + mu_d); 0],  mu_d = alpha (E_perm + T mu_d + E_s(x))
// and dG = C/2 sum_l D_l [reac_l(x) + ind_l(mu_d - mu_v)].  The gradient
// is assembled from a Lagrangian with multipliers lambda_v, lambda_x,
// lambda_d; the kernels below evaluate its pieces.  All FP64.  Derivatives
// of pair terms with respect to positions use forward-mode duals on the
// pair vector, so the damped-tensor hierarchy (Thole factors included) is
// differentiated exactly.
#include <cmath>

#include "dual.hpp"
#include "kernels.hpp"

namespace pbmp {

namespace {

using D3 = Dual<3>;

// ---- pair functions, templated on the scalar type -----------------------

// gradient (in the evaluation point) of the literal multipole potential
// q/R + p.R/R^3 + (1/2) Q_ab R_a R_b / R^5, R = evaluation point - source
template <class S>
__device__ inline void perm_grad(const S R[3], double q, const double *p,
                                 const double *Q, S g[3]) {
  const S rr = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
  const S ri = 1.0 / sqrt(rr);
  const S ri2 = ri * ri, ri3 = ri * ri2, ri5 = ri3 * ri2, ri7 = ri5 * ri2;
  S QR[3];
  for (int a = 0; a < 3; ++a)
    QR[a] = 0.5 * ((Q[3 * a] + Q[a]) * R[0] + (Q[3 * a + 1] + Q[3 + a]) * R[1] +
                   (Q[3 * a + 2] + Q[6 + a]) * R[2]);
  const S Sq = QR[0] * R[0] + QR[1] * R[1] + QR[2] * R[2];
  const S pR = p[0] * R[0] + p[1] * R[1] + p[2] * R[2];
  for (int a = 0; a < 3; ++a)
    g[a] = -q * R[a] * ri3 + p[a] * ri3 - 3.0 * pR * R[a] * ri5 + QR[a] * ri5 -
           2.5 * Sq * R[a] * ri7;
}

// Thole-damped potential data of dipole mu at R: (phi, grad, hessian upper)
template <class S>
__device__ inline void damped_data(const S R[3], const double *mu, double aprod,
                                   double ta, S out[10]) {
  const S rr = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
  const S rad = sqrt(rr);
  const S ri = 1.0 / rad;
  const S ri3 = ri / rr, ri5 = ri3 / rr, ri7 = ri5 / rr;
  S l3(1.0), l5(1.0), l7(1.0);
  if (aprod > 0.0) {
    const S sd = (ta / ::sqrt(aprod)) * (rr * rad);
    const S es = exp(-sd);
    l3 = 1.0 - es;
    l5 = 1.0 - (1.0 + sd) * es;
    l7 = 1.0 - (1.0 + sd + 0.6 * sd * sd) * es;
  }
  const S uR = mu[0] * R[0] + mu[1] * R[1] + mu[2] * R[2];
  out[0] = l3 * uR * ri3;
  for (int a = 0; a < 3; ++a) out[1 + a] = l3 * mu[a] * ri3 - 3.0 * l5 * uR * R[a] * ri5;
  int o = 4;
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b) {
      S t = -3.0 * l5 * (mu[a] * R[b] + mu[b] * R[a]) * ri5 + 15.0 * l7 * uR * R[a] * R[b] * ri7;
      if (a == b) t = t - 3.0 * l5 * uR * ri5;
      out[o++] = t;
    }
}

// Single- and double-layer kernel data of one node at R = target - node
// (value, grad, hessian upper), G = 1/r and H = n.R/r^3.
template <class S>
__device__ inline void node_data(const S R[3], const double *n, S g[10], S h[10]) {
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
__device__ inline S dot10(const double *W, const S v[10]) {
  S s = W[0] * v[0];
  for (int k = 1; k < 10; ++k) s = s + W[k] * v[k];
  return s;
}

__device__ inline void load_panel(const double *verts, const int *tri, int j, double v[3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) v[a][d] = verts[3 * tri[3 * j + a] + d];
}

// ---- kernels -------------------------------------------------------------

// W'_l = c (q, d, Q/6 packed on the hessian upper triangle) + (0, wd, 0)
__global__ void k_make_weights(int M, double c, const double *__restrict__ q,
                               const double *__restrict__ d, const double *__restrict__ Q,
                               const double *__restrict__ wd, double *__restrict__ W) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= M) return;
  const double *Ql = Q + 9 * l;
  double *w = W + 10 * l;
  w[0] = c * q[l];
  for (int a = 0; a < 3; ++a) w[1 + a] = c * d[3 * l + a] + (wd ? wd[3 * l + a] : 0.0);
  w[4] = c * Ql[0] / 6.0;
  w[5] = c * (Ql[1] + Ql[3]) / 6.0;
  w[6] = c * (Ql[2] + Ql[6]) / 6.0;
  w[7] = c * Ql[4] / 6.0;
  w[8] = c * (Ql[5] + Ql[7]) / 6.0;
  w[9] = c * Ql[8] / 6.0;
}

// out[j] = -d/dphi_j, out[N+j] = -d/ddphi_j of sum_l W_l . reac_l(x), i.e.
// minus the transposed readout (far rule everywhere, near rule on the
// panel's near sites via the transposed site list).
__global__ __launch_bounds__(256) void k_readout_T(
    int N, int M, int nf, const double *__restrict__ src64, const double *__restrict__ geo,
    const double *__restrict__ verts, const int *__restrict__ tri, RuleArgs ru,
    const double *__restrict__ xyz, const double *__restrict__ W,
    const int *__restrict__ tsrow, const int *__restrict__ tscol, double *__restrict__ out) {
  constexpr int kT = 64;
  __shared__ double sh[kT * 13];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int jl = min(j, N - 1);
  const double *rec = src64 + 16 * (size_t)jl;
  const double n[3] = {rec[9], rec[10], rec[11]};
  const double A = geo[6 * N + jl];
  double sg = 0.0, sh_ = 0.0;
  for (int l0 = 0; l0 < M; l0 += kT) {
    const int nl = min(kT, M - l0);
    __syncthreads();
    for (int e = threadIdx.x; e < nl * 13; e += blockDim.x) {
      const int l = l0 + e / 13, k = e % 13;
      sh[e] = k < 3 ? xyz[3 * l + k] : W[10 * l + k - 3];
    }
    __syncthreads();
    for (int e = 0; e < nl; ++e) {
      const double *s = sh + 13 * e;
      for (int q = 0; q < nf; ++q) {
        const double R[3] = {s[0] - rec[3 * q], s[1] - rec[3 * q + 1], s[2] - rec[3 * q + 2]};
        double g[10], h[10];
        node_data<double>(R, n, g, h);
        sg += ru.fw[q] * dot10<double>(s + 3, g);
        sh_ += ru.fw[q] * dot10<double>(s + 3, h);
      }
    }
  }
  if (j >= N) return;
  // near sites: far rule -> 19-node rule
  double v[3][3];
  load_panel(verts, tri, j, v);
  for (int t = tsrow[j]; t < tsrow[j + 1]; ++t) {
    const int l = tscol[t];
    const double P[3] = {xyz[3 * l], xyz[3 * l + 1], xyz[3 * l + 2]};
    for (int q = 0; q < nf; ++q) {
      const double R[3] = {P[0] - rec[3 * q], P[1] - rec[3 * q + 1], P[2] - rec[3 * q + 2]};
      double g[10], h[10];
      node_data<double>(R, n, g, h);
      sg -= ru.fw[q] * dot10<double>(W + 10 * l, g);
      sh_ -= ru.fw[q] * dot10<double>(W + 10 * l, h);
    }
    for (int q = 0; q < ru.nn; ++q) {
      double R[3];
      for (int d = 0; d < 3; ++d)
        R[d] = P[d] - (ru.nb[q][0] * v[0][d] + ru.nb[q][1] * v[1][d] + ru.nb[q][2] * v[2][d]);
      double g[10], h[10];
      node_data<double>(R, n, g, h);
      sg += ru.nw[q] * dot10<double>(W + 10 * l, g);
      sh_ += ru.nw[q] * dot10<double>(W + 10 * l, h);
    }
  }
  out[j] = A * sh_;       // -(-A sum h)
  out[N + j] = -A * sg;   // -(A sum g)
}

// grad at the sites of the potential of point charges sigma_i at the
// centroids: out[3m] = sum_i sigma_i (c_i - r_m)/|c_i - r_m|^3
__global__ __launch_bounds__(256) void k_charge_field(int N, const double *__restrict__ geo,
                                                     const double *__restrict__ sigma,
                                                     const double *__restrict__ xyz,
                                                     double *__restrict__ out) {
  __shared__ double red[3][256];
  const int m = blockIdx.x;
  const double P[3] = {xyz[3 * m], xyz[3 * m + 1], xyz[3 * m + 2]};
  double a[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < N; i += 256) {
    const double R[3] = {geo[i] - P[0], geo[N + i] - P[1], geo[2 * N + i] - P[2]};
    const double rr = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    const double ri = 1.0 / sqrt(rr);
    const double w = sigma[i] * ri * ri * ri;
    for (int d = 0; d < 3; ++d) a[d] += w * R[d];
  }
  for (int d = 0; d < 3; ++d) red[d][threadIdx.x] = a[d];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int d = 0; d < 3; ++d) red[d][threadIdx.x] += red[d][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 3) out[3 * m + threadIdx.x] = red[threadIdx.x][0];
}

// J_mu[m] = sum_{l != m} W_l . d ind_l / d mu_m  (damped, / eps_in)
__global__ void k_jmu(int M, const double *__restrict__ W, const double *__restrict__ xyz,
                      const double *__restrict__ alpha, double ta, double inv_eps,
                      double *__restrict__ out) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int l = 0; l < M; ++l) {
    if (l == m) continue;
    const double R[3] = {xyz[3 * l] - xyz[3 * m], xyz[3 * l + 1] - xyz[3 * m + 1],
                         xyz[3 * l + 2] - xyz[3 * m + 2]};
    for (int a = 0; a < 3; ++a) {
      double e[3] = {0.0, 0.0, 0.0};
      e[a] = 1.0;
      double dd[10];
      damped_data<double>(R, e, alpha[l] * alpha[m], ta, dd);
      acc[a] += dot10<double>(W + 10 * l, dd);
    }
  }
  for (int a = 0; a < 3; ++a) out[3 * m + a] = acc[a] * inv_eps;
}

// Ordered site pair (a target, b source), R = r_a - r_b:
//   F_ab(R) = [masked] wsum_a . grad phi_perm,b(R)
//           + wv_a . grad phi_d(R; mu_v,b) + wd_a . grad phi_d(R; mu_d,b)
//           + W_a . data_d(R; dmu_b)                          (all / eps_in)
// with W_a = c (q, d, Q/6) weights.  Gradient w.r.t. site positions:
// r_a += dF_ab/dR, r_b -= dF_ab/dR.  Parameter gradient of b as the
// permanent source: d/d(q_b, d_b, Q_b) of the first term.
__global__ void k_site_pairs(int M, const double *__restrict__ xyz,
                             const double *__restrict__ q, const double *__restrict__ d,
                             const double *__restrict__ Q, const int *__restrict__ group,
                             const double *__restrict__ alpha, double ta, double inv_eps,
                             const double *__restrict__ Wc, const double *__restrict__ wv,
                             const double *__restrict__ wd, const double *__restrict__ mu_v,
                             const double *__restrict__ mu_d, double *__restrict__ g_r,
                             double *__restrict__ g_q, double *__restrict__ g_d,
                             double *__restrict__ g_Q) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= M) return;
  double gr[3] = {0.0, 0.0, 0.0}, gq = 0.0, gd[3] = {0.0, 0.0, 0.0}, gQ[9];
  for (int k = 0; k < 9; ++k) gQ[k] = 0.0;
  for (int m = 0; m < M; ++m) {
    if (m == l) continue;
    for (int role = 0; role < 2; ++role) {
      // role 0: l target, m source; role 1: m target, l source
      const int a = role ? m : l, b = role ? l : m;
      D3 R[3];
      for (int k = 0; k < 3; ++k) R[k] = D3::var(xyz[3 * a + k] - xyz[3 * b + k], k);
      D3 F(0.0);
      const double wsum[3] = {wv[3 * a] + wd[3 * a], wv[3 * a + 1] + wd[3 * a + 1],
                              wv[3 * a + 2] + wd[3 * a + 2]};
      if (group[a] != group[b]) {
        D3 gp[3];
        perm_grad<D3>(R, q[b], d + 3 * b, Q + 9 * b, gp);
        for (int k = 0; k < 3; ++k) F = F + wsum[k] * gp[k];
      }
      const double ap = alpha[a] * alpha[b];
      D3 dd[10];
      damped_data<D3>(R, mu_v + 3 * b, ap, ta, dd);
      for (int k = 0; k < 3; ++k) F = F + wv[3 * a + k] * dd[1 + k];
      damped_data<D3>(R, mu_d + 3 * b, ap, ta, dd);
      for (int k = 0; k < 3; ++k) F = F + wd[3 * a + k] * dd[1 + k];
      const double dmu[3] = {mu_d[3 * b] - mu_v[3 * b], mu_d[3 * b + 1] - mu_v[3 * b + 1],
                             mu_d[3 * b + 2] - mu_v[3 * b + 2]};
      damped_data<D3>(R, dmu, ap, ta, dd);
      F = F + dot10<D3>(Wc + 10 * a, dd);
      const double sgn = role ? -1.0 : 1.0;
      for (int k = 0; k < 3; ++k) gr[k] += sgn * inv_eps * F.d[k];
      if (role == 1 && group[a] != group[b]) {
        // l is the permanent source b: d/dq, d/dd, d/dQ of wsum . grad phi
        double Rv[3] = {R[0].v, R[1].v, R[2].v};
        const double rr = Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2];
        const double ri = 1.0 / ::sqrt(rr);
        const double ri3 = ri * ri * ri, ri5 = ri3 * ri * ri, ri7 = ri5 * ri * ri;
        const double wR = wsum[0] * Rv[0] + wsum[1] * Rv[1] + wsum[2] * Rv[2];
        gq += inv_eps * (-wR * ri3);
        for (int k = 0; k < 3; ++k) gd[k] += inv_eps * (wsum[k] * ri3 - 3.0 * wR * Rv[k] * ri5);
        for (int x = 0; x < 3; ++x)
          for (int y = 0; y < 3; ++y)
            gQ[3 * x + y] += inv_eps * (0.5 * (wsum[x] * Rv[y] + Rv[x] * wsum[y]) * ri5 -
                                        2.5 * wR * Rv[x] * Rv[y] * ri7);
      }
    }
  }
  for (int k = 0; k < 3; ++k) g_r[3 * l + k] = gr[k];
  g_q[l] = gq;
  for (int k = 0; k < 3; ++k) g_d[3 * l + k] = gd[k];
  for (int k = 0; k < 9; ++k) g_Q[9 * l + k] = gQ[k];
}

// d/dr_l of W'_l . reac_l(x): the readout at the site differentiated in its
// position (far rule over all panels, near rule on the site's near panels).
__global__ __launch_bounds__(256) void k_readout_grad(
    int N, int M, int nf, const double *__restrict__ src64, const double *__restrict__ verts,
    const int *__restrict__ tri, RuleArgs ru, const double *__restrict__ geo,
    const double *__restrict__ x, const double *__restrict__ xyz,
    const double *__restrict__ W, const int *__restrict__ srow, const int *__restrict__ scol,
    double *__restrict__ g_r) {
  __shared__ double red[3][256];
  const int l = blockIdx.x;
  D3 P[3];
  for (int k = 0; k < 3; ++k) P[k] = D3::var(xyz[3 * l + k], k);
  const double *w = W + 10 * l;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int j = threadIdx.x; j < N; j += 256) {
    const double *rec = src64 + 16 * (size_t)j;
    const double n[3] = {rec[9], rec[10], rec[11]};
    const double A = geo[6 * N + j];
    const double ph = x[j], dp = x[N + j];
    for (int q = 0; q < nf; ++q) {
      D3 R[3];
      for (int k = 0; k < 3; ++k) R[k] = P[k] - rec[3 * q + k];
      D3 g[10], h[10];
      node_data<D3>(R, n, g, h);
      const D3 t = (ru.fw[q] * A) * (dp * dot10<D3>(w, g) - ph * dot10<D3>(w, h));
      for (int k = 0; k < 3; ++k) acc[k] += t.d[k];
    }
  }
  for (int e = srow[l] + threadIdx.x; e < srow[l + 1]; e += 256) {
    const int j = scol[e];
    double v[3][3];
    load_panel(verts, tri, j, v);
    const double *rec = src64 + 16 * (size_t)j;
    const double n[3] = {rec[9], rec[10], rec[11]};
    const double A = geo[6 * N + j];
    const double ph = x[j], dp = x[N + j];
    for (int pass = 0; pass < 2; ++pass) {
      const int nq = pass ? nf : ru.nn;
      for (int q = 0; q < nq; ++q) {
        const double *b = pass ? ru.fb[q] : ru.nb[q];
        const double wq = pass ? -ru.fw[q] : ru.nw[q];
        D3 R[3];
        for (int k = 0; k < 3; ++k)
          R[k] = P[k] - (b[0] * v[0][k] + b[1] * v[1][k] + b[2] * v[2][k]);
        D3 g[10], h[10];
        node_data<D3>(R, n, g, h);
        const D3 t = (wq * A) * (dp * dot10<D3>(w, g) - ph * dot10<D3>(w, h));
        for (int k = 0; k < 3; ++k) acc[k] += t.d[k];
      }
    }
  }
  for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 3) g_r[3 * l + threadIdx.x] = red[threadIdx.x][0];
}

// Right-hand-side term -lambda_1 . f: per source site m, with
// sigma_i = lambda_1,i / (4 pi eps_in) and R = c_i - r_m:
//   g_q -= sum sigma/R, g_p -= sum sigma R/R^3, g_Q -= sum sigma R R/(2 R^5),
//   g_r += sum sigma grad phi_m(R)   (phi_m with p = d + mu_d)
__global__ __launch_bounds__(256) void k_rhs_grad(int N, const double *__restrict__ geo,
                                                 const double *__restrict__ sigma,
                                                 const double *__restrict__ xyz,
                                                 const double *__restrict__ q,
                                                 const double *__restrict__ p,
                                                 const double *__restrict__ Q,
                                                 double *__restrict__ g_r,
                                                 double *__restrict__ g_q,
                                                 double *__restrict__ g_d,
                                                 double *__restrict__ g_Q) {
  constexpr int NA = 16;
  __shared__ double red[NA][256];
  const int m = blockIdx.x;
  double acc[NA];
  for (int k = 0; k < NA; ++k) acc[k] = 0.0;
  for (int i = threadIdx.x; i < N; i += 256) {
    const double R[3] = {geo[i] - xyz[3 * m], geo[N + i] - xyz[3 * m + 1],
                         geo[2 * N + i] - xyz[3 * m + 2]};
    const double s = sigma[i];
    const double rr = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    const double ri = 1.0 / sqrt(rr);
    const double ri3 = ri * ri * ri, ri5 = ri3 * ri * ri;
    acc[0] -= s * ri;
    for (int a = 0; a < 3; ++a) acc[1 + a] -= s * R[a] * ri3;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) acc[4 + 3 * a + b] -= s * 0.5 * R[a] * R[b] * ri5;
    double g[3];
    perm_grad<double>(R, q[m], p + 3 * m, Q + 9 * m, g);
    for (int a = 0; a < 3; ++a) acc[13 + a] += s * g[a];
  }
  for (int k = 0; k < NA; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int k = 0; k < NA; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    g_q[m] = red[0][0];
    for (int a = 0; a < 3; ++a) g_d[3 * m + a] = red[1 + a][0];
    for (int k = 0; k < 9; ++k) g_Q[9 * m + k] = red[4 + k][0];
    for (int a = 0; a < 3; ++a) g_r[3 * m + a] = red[13 + a][0];
  }
}

// z = M^{-T} u for the transposed 2x2 panel blocks [[1/2, 1/2],[-a, e b]]
__global__ void k_precond_T(int N, const double *__restrict__ diag, double e,
                            const double *__restrict__ u, double *__restrict__ z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double a = diag[i], b = diag[N + i];
  const double det = 0.5 * (e * b + a);
  z[i] = (e * b * u[i] - 0.5 * u[N + i]) / det;
  z[N + i] = (a * u[i] + 0.5 * u[N + i]) / det;
}

__global__ void k_scale_sites(int M, const double *__restrict__ alpha,
                              const double *__restrict__ lam, double *__restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 3 * M) w[i] = alpha[i / 3] * lam[i];
}

// lam <- (1-w) lam + w (E + F - J); sums |dlam|^2 and |lam|^2
__global__ void k_adj_update(int M, double omega, const double *__restrict__ E,
                             const double *__restrict__ F, const double *__restrict__ J,
                             double Jsign, double *__restrict__ lam, double *__restrict__ out2) {
  __shared__ double r1[256], r2[256];
  double a1 = 0.0, a2 = 0.0;
  for (int i = threadIdx.x; i < 3 * M; i += 256) {
    const double tgt = E[i] + (F ? F[i] : 0.0) + Jsign * J[i];
    const double nw = (1.0 - omega) * lam[i] + omega * tgt;
    a1 += (nw - lam[i]) * (nw - lam[i]);
    a2 += nw * nw;
    lam[i] = nw;
  }
  r1[threadIdx.x] = a1;
  r2[threadIdx.x] = a2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      r1[threadIdx.x] += r1[threadIdx.x + s];
      r2[threadIdx.x] += r2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out2[0] = r1[0];
    out2[1] = r2[0];
  }
}


// Potential data (phi, grad, hessian upper) at every site of the other
// sites' permanent multipoles, unmasked and undamped (the vacuum Coulomb
// energy uses them; eq. energy_multipole_polarizable): the hessian is the
// dual-number derivative of the gradient.
__global__ void k_perm_potential(int M, const double *__restrict__ xyz,
                                 const double *__restrict__ q, const double *__restrict__ d,
                                 const double *__restrict__ Q, double inv_eps,
                                 double *__restrict__ out) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= M) return;
  double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int m = 0; m < M; ++m) {
    if (m == l) continue;
    D3 R[3];
    for (int a = 0; a < 3; ++a) R[a] = D3::var(xyz[3 * l + a] - xyz[3 * m + a], a);
    D3 g[3];
    perm_grad<D3>(R, q[m], d + 3 * m, Q + 9 * m, g);
    const double r[3] = {R[0].v, R[1].v, R[2].v};
    const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double ri = 1.0 / sqrt(rr), ri3 = ri / rr, ri5 = ri3 / rr;
    const double *pm = d + 3 * m, *Qm = Q + 9 * m;
    double S = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) S += 0.5 * (Qm[3 * a + b] + Qm[3 * b + a]) * r[a] * r[b];
    acc[0] += q[m] * ri + (pm[0] * r[0] + pm[1] * r[1] + pm[2] * r[2]) * ri3 + 0.5 * S * ri5;
    for (int a = 0; a < 3; ++a) acc[1 + a] += g[a].v;
    int o = 4;
    for (int a = 0; a < 3; ++a)
      for (int b = a; b < 3; ++b) acc[o++] += g[a].d[b];
  }
  for (int k = 0; k < 10; ++k) out[10 * (size_t)l + k] = acc[k] * inv_eps;
}

}  // namespace

void launch_make_weights(hipStream_t s, int M, double c, const double *q, const double *d,
                         const double *Q, const double *wd, double *W) {
  hipLaunchKernelGGL(k_make_weights, dim3((M + 127) / 128), dim3(128), 0, s, M, c, q, d, Q,
                     wd, W);
  PBMP_HIP(hipGetLastError());
}

void launch_readout_T(hipStream_t s, int N, int M, const double *src64, const double *geo,
                      const double *verts, const int *tri, const RuleArgs &ru,
                      const double *xyz, const double *W, const int *tsrow, const int *tscol,
                      double *out) {
  hipLaunchKernelGGL(k_readout_T, dim3((N + 255) / 256), dim3(256), 0, s, N, M, ru.nf, src64,
                     geo, verts, tri, ru, xyz, W, tsrow, tscol, out);
  PBMP_HIP(hipGetLastError());
}

void launch_charge_field(hipStream_t s, int N, int M, const double *geo, const double *sigma,
                         const double *xyz, double *out) {
  hipLaunchKernelGGL(k_charge_field, dim3(M), dim3(256), 0, s, N, geo, sigma, xyz, out);
  PBMP_HIP(hipGetLastError());
}

void launch_jmu(hipStream_t s, int M, const double *W, const double *xyz, const double *alpha,
                double ta, double eps_in, double *out) {
  hipLaunchKernelGGL(k_jmu, dim3((M + 63) / 64), dim3(64), 0, s, M, W, xyz, alpha, ta,
                     1.0 / eps_in, out);
  PBMP_HIP(hipGetLastError());
}

void launch_site_pairs(hipStream_t s, int M, const double *xyz, const double *q,
                       const double *d, const double *Q, const int *group,
                       const double *alpha, double ta, double eps_in, const double *Wc,
                       const double *wv, const double *wd, const double *mu_v,
                       const double *mu_d, double *g_r, double *g_q, double *g_d,
                       double *g_Q) {
  hipLaunchKernelGGL(k_site_pairs, dim3((M + 63) / 64), dim3(64), 0, s, M, xyz, q, d, Q, group,
                     alpha, ta, 1.0 / eps_in, Wc, wv, wd, mu_v, mu_d, g_r, g_q, g_d, g_Q);
  PBMP_HIP(hipGetLastError());
}

void launch_readout_grad(hipStream_t s, int N, int M, const double *src64, const double *verts,
                         const int *tri, const RuleArgs &ru, const double *geo,
                         const double *x, const double *xyz, const double *W,
                         const int *srow, const int *scol, double *g_r) {
  hipLaunchKernelGGL(k_readout_grad, dim3(M), dim3(256), 0, s, N, M, ru.nf, src64, verts, tri,
                     ru, geo, x, xyz, W, srow, scol, g_r);
  PBMP_HIP(hipGetLastError());
}

void launch_rhs_grad(hipStream_t s, int N, int M, const double *geo, const double *sigma,
                     const double *xyz, const double *q, const double *p, const double *Q,
                     double *g_r, double *g_q, double *g_d, double *g_Q) {
  hipLaunchKernelGGL(k_rhs_grad, dim3(M), dim3(256), 0, s, N, geo, sigma, xyz, q, p, Q, g_r,
                     g_q, g_d, g_Q);
  PBMP_HIP(hipGetLastError());
}

void launch_precond_T(hipStream_t s, int N, const double *diag, double eps_ratio,
                      const double *u, double *z) {
  hipLaunchKernelGGL(k_precond_T, dim3((N + 255) / 256), dim3(256), 0, s, N, diag, eps_ratio, u,
                     z);
  PBMP_HIP(hipGetLastError());
}

void launch_scale_sites(hipStream_t s, int M, const double *alpha, const double *lam,
                        double *w) {
  hipLaunchKernelGGL(k_scale_sites, dim3((3 * M + 255) / 256), dim3(256), 0, s, M, alpha, lam,
                     w);
  PBMP_HIP(hipGetLastError());
}

void launch_adj_update(hipStream_t s, int M, double omega, const double *E, const double *F,
                       const double *J, double Jsign, double *lam, double *out2) {
  hipLaunchKernelGGL(k_adj_update, dim3(1), dim3(256), 0, s, M, omega, E, F, J, Jsign, lam,
                     out2);
  PBMP_HIP(hipGetLastError());
}

void launch_perm_potential(hipStream_t s, int M, const double *xyz, const double *q,
                           const double *d, const double *Q, double eps_in, double *out) {
  if (M <= 0) return;
  hipLaunchKernelGGL(k_perm_potential, dim3((M + 127) / 128), dim3(128), 0, s, M, xyz, q, d, Q,
                     1.0 / eps_in, out);
  PBMP_HIP(hipGetLastError());
}

}  // namespace pbmp
