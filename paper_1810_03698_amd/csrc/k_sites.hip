// Kernels at the point-multipole sites: right-hand side (eq. rhs_multipole),
// reaction-potential readout (eq. pot_solvent, Efield_solv, ddphi),
// multipole Coulomb fields (eq. Efield_mult, appendix derivatives) with the
// group masking and Thole damping of the section "Calculation of the
// electric field", the relaxed induced-dipole update and the energy sum of
// eq. energy_multipole_polarizable.
#include <cmath>

#include "kernels.hpp"

namespace pbmp {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;
constexpr double kFourPi = 12.566370614359172;

// ------------------------------------------------------------------ RHS
// Site record in LDS: x y z q px py pz Qxx Qxy Qxz Qyy Qyz Qzz
constexpr int kSiteRec = 13;
constexpr int kSiteTile = 128;

template <bool FP64>
__global__ __launch_bounds__(256) void k_rhs(int N, int M,
                                             const double *__restrict__ geo,
                                             const double *__restrict__ xyz,
                                             const double *__restrict__ q,
                                             const double *__restrict__ p,
                                             const double *__restrict__ Q9,
                                             double scale,
                                             double *__restrict__ f) {
  __shared__ double sh[kSiteTile * kSiteRec];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int il = min(i, N - 1);
  const double cx = geo[il], cy = geo[N + il], cz = geo[2 * N + il];
  double acc = 0.0;
  for (int k0 = 0; k0 < M; k0 += kSiteTile) {
    const int nk = min(kSiteTile, M - k0);
    __syncthreads();
    for (int e = threadIdx.x; e < nk; e += blockDim.x) {
      const int k = k0 + e;
      double *r = sh + kSiteRec * e;
      r[0] = xyz[3 * k];
      r[1] = xyz[3 * k + 1];
      r[2] = xyz[3 * k + 2];
      r[3] = q[k];
      r[4] = p[3 * k];
      r[5] = p[3 * k + 1];
      r[6] = p[3 * k + 2];
      r[7] = Q9[9 * k];
      r[8] = Q9[9 * k + 1];
      r[9] = Q9[9 * k + 2];
      r[10] = Q9[9 * k + 4];
      r[11] = Q9[9 * k + 5];
      r[12] = Q9[9 * k + 8];
    }
    __syncthreads();
    for (int e = 0; e < nk; ++e) {
      const double *r = sh + kSiteRec * e;
      if (FP64) {
        const double X = cx - r[0], Y = cy - r[1], Z = cz - r[2];
        const double rr = X * X + Y * Y + Z * Z;
        const double ri = 1.0 / sqrt(rr);
        const double ri2 = ri * ri;
        const double pR = r[4] * X + r[5] * Y + r[6] * Z;
        const double QRR = r[7] * X * X + r[10] * Y * Y + r[12] * Z * Z +
                           2.0 * (r[8] * X * Y + r[9] * X * Z + r[11] * Y * Z);
        acc += ri * (r[3] + ri2 * (pR + 0.5 * QRR * ri2));
      } else {
        const float X = (float)(cx - r[0]), Y = (float)(cy - r[1]),
                    Z = (float)(cz - r[2]);
        const float rr = fmaf(X, X, fmaf(Y, Y, Z * Z));
        const float ri = __builtin_amdgcn_rsqf(rr);
        const float ri2 = ri * ri;
        const float pR = (float)r[4] * X + (float)r[5] * Y + (float)r[6] * Z;
        const float QRR = (float)r[7] * X * X + (float)r[10] * Y * Y +
                          (float)r[12] * Z * Z +
                          2.0f * ((float)r[8] * X * Y + (float)r[9] * X * Z +
                                  (float)r[11] * Y * Z);
        acc += (double)(ri * ((float)r[3] + ri2 * (pR + 0.5f * QRR * ri2)));
      }
    }
  }
  if (i < N) f[i] = acc * scale;
}

// ------------------------------------------------------------- readout
// Kernel values of one source node at a target, for the single layer
// (G = 1/r) and double layer (H = n.R/r^3) with their first and second
// derivatives in the target point: out[0..9] = G data, out[10..19] = H data
// (order: value, d/dx, d/dy, d/dz, xx, xy, xz, yy, yz, zz).
template <class T, bool FULL>
__device__ inline void node_kernels(T X, T Y, T Z, T nx, T ny, T nz, T nR,
                                    T *g, T *h) {
  const T rr = X * X + Y * Y + Z * Z;
  T i1;
  if constexpr (sizeof(T) == 4)
    i1 = __builtin_amdgcn_rsqf(rr);
  else
    i1 = T(1) / sqrt(rr);
  const T i2 = i1 * i1;
  const T i3 = i1 * i2;
  const T i5 = i3 * i2;
  const T R[3] = {X, Y, Z};
  const T n[3] = {nx, ny, nz};
  g[0] += i1;
  h[0] += nR * i3;
  for (int a = 0; a < 3; ++a) {
    g[1 + a] -= R[a] * i3;
    h[1 + a] += n[a] * i3 - T(3) * nR * R[a] * i5;
  }
  if constexpr (FULL) {
    const T i7 = i5 * i2;
    int o = 4;
    for (int a = 0; a < 3; ++a)
      for (int b = a; b < 3; ++b) {
        const T del = (a == b) ? T(1) : T(0);
        g[o] += T(3) * R[a] * R[b] * i5 - del * i3;
        h[o] += T(-3) * (n[a] * R[b] + n[b] * R[a] + nR * del) * i5 +
                T(15) * nR * R[a] * R[b] * i7;
        ++o;
      }
  }
}

// Far-field readout: one site per lane (64 sites per block), the panels of
// one source chunk staged through LDS in tiles of kRoTile records (coalesced
// 16-byte loads of the contiguous records, all issued before the first
// store), per-chunk partial sums part[chunk][site][k].  Per panel the sums
// are formed as in the operator: node differences from FP64 positions, the
// kernels in T, the panel's strengths applied before the FP64 accumulation.
constexpr int kRoTile = 64;

template <bool FP64, bool FULL>
__global__ __launch_bounds__(64) void k_readout_far(
    int N, int M, int nf, const double *__restrict__ src64,
    const float *__restrict__ src32, const double *__restrict__ xyz, int chunk,
    double *__restrict__ part) {
  constexpr int NO = FULL ? 10 : 4;
  typedef double d2 __attribute__((ext_vector_type(2)));
  typedef float f4 __attribute__((ext_vector_type(4)));
  __shared__ __align__(16) double s64[kRoTile * 16];
  __shared__ __align__(16) float s32[FP64 ? 4 : kRoTile * 16];
  const int lane = (int)threadIdx.x;
  const int l = blockIdx.x * 64 + lane;
  const int lc = min(l, M - 1);
  const int j0 = blockIdx.y * chunk, j1 = min(N, j0 + chunk);
  const double P[3] = {xyz[3 * lc], xyz[3 * lc + 1], xyz[3 * lc + 2]};
  double acc[NO];
  for (int k = 0; k < NO; ++k) acc[k] = 0.0;
  for (int jt = j0; jt < j1; jt += kRoTile) {
    const int nj = min(kRoTile, j1 - jt);
    __syncthreads();
    {
      const d2 *g = reinterpret_cast<const d2 *>(src64 + 16 * (size_t)jt);
      d2 *d = reinterpret_cast<d2 *>(s64);
      const int n = nj * 8;
      d2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = lane + 64 * u;
        if (e < n) v[u] = g[e];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = lane + 64 * u;
        if (e < n) d[e] = v[u];
      }
      if constexpr (!FP64) {
        const f4 *g32 = reinterpret_cast<const f4 *>(src32 + 16 * (size_t)jt);
        f4 *d32 = reinterpret_cast<f4 *>(s32);
        const int n32 = nj * 4;
        f4 w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = lane + 64 * u;
          if (e < n32) w[u] = g32[e];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = lane + 64 * u;
          if (e < n32) d32[e] = w[u];
        }
      }
    }
    __syncthreads();
    for (int jj = 0; jj < nj; ++jj) {
      const double *r64 = s64 + 16 * jj;
      if constexpr (FP64) {
        double g[NO], h[NO];
        for (int k = 0; k < NO; ++k) g[k] = h[k] = 0.0;
        const double nR = r64[9] * P[0] + r64[10] * P[1] + r64[11] * P[2] - r64[12];
        for (int qn = 0; qn < nf; ++qn)
          node_kernels<double, FULL>(P[0] - r64[3 * qn], P[1] - r64[3 * qn + 1],
                                     P[2] - r64[3 * qn + 2], r64[9], r64[10], r64[11],
                                     nR, g, h);
        for (int k = 0; k < NO; ++k) acc[k] += r64[13] * g[k] - r64[14] * h[k];
      } else {
        const float *r = s32 + 16 * jj;
        float g[NO], h[NO];
        for (int k = 0; k < NO; ++k) g[k] = h[k] = 0.0f;
        const float nR = (float)(r64[9] * P[0] + r64[10] * P[1] + r64[11] * P[2] - r64[12]);
        for (int qn = 0; qn < nf; ++qn)
          node_kernels<float, FULL>((float)(P[0] - r64[3 * qn]),
                                    (float)(P[1] - r64[3 * qn + 1]),
                                    (float)(P[2] - r64[3 * qn + 2]), r[9], r[10],
                                    r[11], nR, g, h);
        for (int k = 0; k < NO; ++k)
          acc[k] += (double)(r[13] * g[k] - r[14] * h[k]);
      }
    }
  }
  if (l < M)
    for (int k = 0; k < NO; ++k) part[((size_t)blockIdx.y * M + l) * NO + k] = acc[k];
}

// Near-singular correction at the sites (19-node rule instead of the far
// rule for panels with |r_l - c_j| < eta sqrt(A_j)), chunk sum, and the
// 4 pi factor to physical units.  One 64-lane block per site.
template <bool FULL>
__global__ __launch_bounds__(64) void k_readout_near(
    int N, int M, int nchunk, const double *__restrict__ part,
    const double *__restrict__ verts, const int *__restrict__ tri,
    const double *__restrict__ geo, RuleArgs ru, const double *__restrict__ x,
    const double *__restrict__ xyz, const int *__restrict__ srow,
    const int *__restrict__ scol, double *__restrict__ out) {
  constexpr int NO = FULL ? 10 : 4;
  __shared__ double red[64];
  const int l = blockIdx.x;
  const double P[3] = {xyz[3 * l], xyz[3 * l + 1], xyz[3 * l + 2]};
  double acc[NO];
  for (int k = 0; k < NO; ++k) acc[k] = 0.0;
  for (int e = srow[l] + threadIdx.x; e < srow[l + 1]; e += blockDim.x) {
    const int j = scol[e];
    double v[3][3];
    for (int a = 0; a < 3; ++a)
      for (int d = 0; d < 3; ++d) v[a][d] = verts[3 * tri[3 * j + a] + d];
    const double n[3] = {geo[3 * N + j], geo[4 * N + j], geo[5 * N + j]};
    const double A = geo[6 * N + j];
    const double ph = x[j], dp = x[N + j];
    for (int pass = 0; pass < 2; ++pass) {
      const int nq = pass ? ru.nf : ru.nn;
      const double sign = pass ? -1.0 : 1.0;
      for (int qn = 0; qn < nq; ++qn) {
        const double *b = pass ? ru.fb[qn] : ru.nb[qn];
        const double w = pass ? ru.fw[qn] : ru.nw[qn];
        double y[3];
        for (int d = 0; d < 3; ++d) y[d] = b[0] * v[0][d] + b[1] * v[1][d] + b[2] * v[2][d];
        const double X = P[0] - y[0], Y = P[1] - y[1], Z = P[2] - y[2];
        const double nR = n[0] * X + n[1] * Y + n[2] * Z;
        double g[NO], h[NO];
        for (int k = 0; k < NO; ++k) g[k] = h[k] = 0.0;
        node_kernels<double, FULL>(X, Y, Z, n[0], n[1], n[2], nR, g, h);
        const double sa = sign * w * A * dp * kInv4Pi;
        const double sb = sign * w * A * ph * kInv4Pi;
        for (int k = 0; k < NO; ++k) acc[k] += sa * g[k] - sb * h[k];
      }
    }
  }
  // the far chunks' partial sums join the lanes' near sums (chunk c on lane
  // c mod 64), then a fixed-order tree over the lanes
  for (int k = 0; k < NO; ++k) {
    double v = acc[k];
    for (int c = threadIdx.x; c < nchunk; c += blockDim.x) v += part[((size_t)c * M + l) * NO + k];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[(size_t)l * NO + k] = kFourPi * red[0];
    __syncthreads();
  }
}

// ------------------------------------------------------------- Coulomb
// Sum over the 64 lanes of a wave (every lane receives the total).
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// The site-pair kernels below take one wave per site l, lanes over the
// sources m (strided), and reduce over the wave at the end.
__global__ __launch_bounds__(64) void k_perm_field(int M, const double *__restrict__ xyz,
                                                   const double *__restrict__ q,
                                                   const double *__restrict__ d,
                                                   const double *__restrict__ Q9,
                                                   const int *__restrict__ group,
                                                   double inv_eps, double *__restrict__ E) {
  const int l = blockIdx.x;
  const int lane = (int)threadIdx.x;
  const double P[3] = {xyz[3 * l], xyz[3 * l + 1], xyz[3 * l + 2]};
  const int gl = group[l];
  double g[3] = {0.0, 0.0, 0.0};
  for (int m = lane; m < M; m += 64) {
    if (group[m] == gl) continue;  // includes m == l
    const double R[3] = {P[0] - xyz[3 * m], P[1] - xyz[3 * m + 1],
                         P[2] - xyz[3 * m + 2]};
    const double rr = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    const double ri = 1.0 / sqrt(rr);
    const double ri2 = ri * ri, ri3 = ri * ri2, ri5 = ri3 * ri2, ri7 = ri5 * ri2;
    const double *pm = d + 3 * m;
    const double *Qm = Q9 + 9 * m;
    double QR[3];
    for (int a = 0; a < 3; ++a)
      QR[a] = Qm[3 * a] * R[0] + Qm[3 * a + 1] * R[1] + Qm[3 * a + 2] * R[2];
    const double S = QR[0] * R[0] + QR[1] * R[1] + QR[2] * R[2];
    const double pR = pm[0] * R[0] + pm[1] * R[1] + pm[2] * R[2];
    for (int a = 0; a < 3; ++a)
      g[a] += -q[m] * R[a] * ri3 + pm[a] * ri3 - 3.0 * pR * R[a] * ri5 +
              QR[a] * ri5 - 2.5 * S * R[a] * ri7;
  }
  for (int a = 0; a < 3; ++a) g[a] = wave_sum(g[a]);
  if (lane == 0)
    for (int a = 0; a < 3; ++a) E[3 * l + a] = -g[a] * inv_eps;
}

template <bool FULL>
__global__ __launch_bounds__(64) void k_induced(int M, const double *__restrict__ xyz,
                                                const double *__restrict__ mu,
                                                const double *__restrict__ alpha, double ta,
                                                double inv_eps, double *__restrict__ out) {
  const int l = blockIdx.x;
  const int lane = (int)threadIdx.x;
  const double P[3] = {xyz[3 * l], xyz[3 * l + 1], xyz[3 * l + 2]};
  const double al = alpha[l];
  double acc[10];
  for (int k = 0; k < 10; ++k) acc[k] = 0.0;
  for (int m = lane; m < M; m += 64) {
    if (m == l) continue;
    const double R[3] = {P[0] - xyz[3 * m], P[1] - xyz[3 * m + 1],
                         P[2] - xyz[3 * m + 2]};
    const double rr = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    const double rad = sqrt(rr);
    const double ri = 1.0 / rad;
    const double ri2 = ri * ri, ri3 = ri * ri2, ri5 = ri3 * ri2, ri7 = ri5 * ri2;
    double l3 = 1.0, l5 = 1.0, l7 = 1.0;
    const double ap = al * alpha[m];
    if (ap > 0.0) {
      const double sd = ta * rr * rad / sqrt(ap);
      const double es = exp(-sd);
      l3 = 1.0 - es;
      l5 = 1.0 - (1.0 + sd) * es;
      l7 = 1.0 - (1.0 + sd + 0.6 * sd * sd) * es;
    }
    const double *u = mu + 3 * m;
    const double uR = u[0] * R[0] + u[1] * R[1] + u[2] * R[2];
    acc[0] += l3 * uR * ri3;
    for (int a = 0; a < 3; ++a) acc[1 + a] += l3 * u[a] * ri3 - 3.0 * l5 * uR * R[a] * ri5;
    if (FULL) {
      int o = 4;
      for (int a = 0; a < 3; ++a)
        for (int b = a; b < 3; ++b) {
          const double del = (a == b) ? 1.0 : 0.0;
          acc[o++] += -3.0 * l5 * (u[a] * R[b] + u[b] * R[a] + uR * del) * ri5 +
                      15.0 * l7 * uR * R[a] * R[b] * ri7;
        }
    }
  }
  if (FULL) {
    for (int k = 0; k < 10; ++k) acc[k] = wave_sum(acc[k]);
    if (lane == 0)
      for (int k = 0; k < 10; ++k) out[10 * l + k] = acc[k] * inv_eps;
  } else {
    for (int a = 0; a < 3; ++a) acc[1 + a] = wave_sum(acc[1 + a]);
    if (lane == 0)
      for (int a = 0; a < 3; ++a) out[3 * l + a] = -acc[1 + a] * inv_eps;
  }
}

__global__ void k_scf_update(int M, const double *__restrict__ alpha,
                             const double *__restrict__ Eperm,
                             const double *__restrict__ Eind,
                             const double *__restrict__ solv, int stride,
                             double omega, double *__restrict__ mu,
                             double *__restrict__ dmu2) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int l = threadIdx.x; l < M; l += blockDim.x) {
    for (int a = 0; a < 3; ++a) {
      double E = Eperm[3 * l + a] + Eind[3 * l + a];
      if (solv) E -= solv[(size_t)stride * l + 1 + a];
      const double old = mu[3 * l + a];
      const double nw = (1.0 - omega) * old + omega * alpha[l] * E;
      mu[3 * l + a] = nw;
      acc += (nw - old) * (nw - old);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *dmu2 = red[0];
}

__device__ inline double apply_D(const double *q, const double *d,
                                 const double *Q, int l, const double *v) {
  // q phi + d.grad phi + (1/6) sum_ab Q_ab H_ab, H from its upper triangle
  const double H[3][3] = {{v[4], v[5], v[6]}, {v[5], v[7], v[8]}, {v[6], v[8], v[9]}};
  double qh = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) qh += Q[9 * l + 3 * a + b] * H[a][b];
  return q[l] * v[0] + d[3 * l] * v[1] + d[3 * l + 1] * v[2] + d[3 * l + 2] * v[3] +
         qh / 6.0;
}

__global__ void k_energy(int M, const double *__restrict__ q,
                         const double *__restrict__ d,
                         const double *__restrict__ Q9,
                         const double *__restrict__ reac,
                         const double *__restrict__ ind, double *__restrict__ e) {
  __shared__ double r1[256], r2[256];
  double a1 = 0.0, a2 = 0.0;
  for (int l = threadIdx.x; l < M; l += blockDim.x) {
    a1 += apply_D(q, d, Q9, l, reac + 10 * (size_t)l);
    a2 += apply_D(q, d, Q9, l, ind + 10 * (size_t)l);
  }
  r1[threadIdx.x] = a1;
  r2[threadIdx.x] = a2;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      r1[threadIdx.x] += r1[threadIdx.x + w];
      r2[threadIdx.x] += r2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    e[0] = 0.5 * r1[0];
    e[1] = 0.5 * r2[0];
  }
}

// Total dipole of the molecule for the vacuum and dissolved dipoles:
// sum_l q_l (r_l - o) + d_l + mu_l with o the mean site position, e*A.
__global__ void k_total_dipole(int M, const double *__restrict__ xyz,
                               const double *__restrict__ q,
                               const double *__restrict__ d,
                               const double *__restrict__ mu_v,
                               const double *__restrict__ mu_d,
                               double *__restrict__ out) {
  constexpr int K = 13;  // sum q, sum q r, sum r, sum (d + mu_v), sum mu_d - mu_v
  __shared__ double red[K][256];
  double a[K];
  for (int k = 0; k < K; ++k) a[k] = 0.0;
  for (int l = threadIdx.x; l < M; l += blockDim.x) {
    const double ql = q[l];
    a[0] += ql;
    for (int c = 0; c < 3; ++c) {
      const double r = xyz[3 * l + c];
      a[1 + c] += ql * r;
      a[4 + c] += r;
      a[7 + c] += d[3 * l + c] + mu_v[3 * l + c];
      a[10 + c] += mu_d[3 * l + c] - mu_v[3 * l + c];
    }
  }
  for (int k = 0; k < K; ++k) red[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < K; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) {
    const int c = threadIdx.x;
    const double pv = red[1 + c][0] - red[0][0] * red[4 + c][0] / M + red[7 + c][0];
    out[c] = pv;
    out[3 + c] = pv + red[10 + c][0];
  }
}

}  // namespace

void launch_total_dipole(hipStream_t s, int M, const double *xyz, const double *q,
                         const double *d, const double *mu_v, const double *mu_d,
                         double *out) {
  hipLaunchKernelGGL(k_total_dipole, dim3(1), dim3(256), 0, s, M, xyz, q, d, mu_v,
                     mu_d, out);
  PBMP_HIP(hipGetLastError());
}

void launch_rhs(hipStream_t s, bool fp64, int N, int M, const double *geo,
                const double *xyz, const double *q, const double *p,
                const double *Q9, double eps_in, double *f) {
  const double scale = kInv4Pi / eps_in;
  if (fp64)
    hipLaunchKernelGGL(k_rhs<true>, dim3((N + 255) / 256), dim3(256), 0, s, N,
                       M, geo, xyz, q, p, Q9, scale, f);
  else
    hipLaunchKernelGGL(k_rhs<false>, dim3((N + 255) / 256), dim3(256), 0, s, N,
                       M, geo, xyz, q, p, Q9, scale, f);
  PBMP_HIP(hipGetLastError());
}

int readout_chunks(int N, int M) {
  // about 4096 blocks, each chunk at least one tile of panels
  const int tiles = (std::max(M, 1) + 63) / 64;
  const int c = (4096 + tiles - 1) / tiles;
  return std::max(1, std::min(c, N / kRoTile));
}

void launch_readout(hipStream_t s, bool fp64, bool full, int N, int M,
                    const double *src64, const float *src32, const double *geo,
                    const double *verts, const int *tri, const RuleArgs &ru,
                    const double *x, const double *xyz, const int *srow,
                    const int *scol, int nchunk, double *part, double *out) {
  if (M <= 0) return;
  const int chunk = (N + nchunk - 1) / nchunk;
  dim3 grid((M + 63) / 64, nchunk);
#define PBMP_RO(F64, FULL)                                                   \
  hipLaunchKernelGGL((k_readout_far<F64, FULL>), grid, dim3(64), 0, s, N, M, \
                     ru.nf, src64, src32, xyz, chunk, part)
  if (fp64 && full) PBMP_RO(true, true);
  else if (fp64) PBMP_RO(true, false);
  else if (full) PBMP_RO(false, true);
  else PBMP_RO(false, false);
#undef PBMP_RO
  PBMP_HIP(hipGetLastError());
  if (full)
    hipLaunchKernelGGL(k_readout_near<true>, dim3(M), dim3(64), 0, s, N, M,
                       nchunk, part, verts, tri, geo, ru, x, xyz, srow, scol, out);
  else
    hipLaunchKernelGGL(k_readout_near<false>, dim3(M), dim3(64), 0, s, N, M,
                       nchunk, part, verts, tri, geo, ru, x, xyz, srow, scol, out);
  PBMP_HIP(hipGetLastError());
}

void launch_perm_field(hipStream_t s, int M, const double *xyz,
                       const double *q, const double *d, const double *Q9,
                       const int *group, double eps_in, double *E) {
  if (M <= 0) return;
  hipLaunchKernelGGL(k_perm_field, dim3(M), dim3(64), 0, s, M,
                     xyz, q, d, Q9, group, 1.0 / eps_in, E);
  PBMP_HIP(hipGetLastError());
}

void launch_induced(hipStream_t s, bool full, int M, const double *xyz,
                    const double *mu, const double *alpha, double thole_a,
                    double eps_in, double *out) {
  if (M <= 0) return;
  if (full)
    hipLaunchKernelGGL(k_induced<true>, dim3(M), dim3(64), 0, s,
                       M, xyz, mu, alpha, thole_a, 1.0 / eps_in, out);
  else
    hipLaunchKernelGGL(k_induced<false>, dim3(M), dim3(64), 0, s,
                       M, xyz, mu, alpha, thole_a, 1.0 / eps_in, out);
  PBMP_HIP(hipGetLastError());
}

void launch_scf_update(hipStream_t s, int M, const double *alpha,
                       const double *Eperm, const double *Eind,
                       const double *solv10, int solv_stride, double omega,
                       double *mu, double *dmu2) {
  hipLaunchKernelGGL(k_scf_update, dim3(1), dim3(256), 0, s, M, alpha, Eperm,
                     Eind, solv10, solv_stride, omega, mu, dmu2);
  PBMP_HIP(hipGetLastError());
}

void launch_energy(hipStream_t s, int M, const double *q, const double *d,
                   const double *Q9, const double *reac10, const double *ind10,
                   double *e) {
  hipLaunchKernelGGL(k_energy, dim3(1), dim3(256), 0, s, M, q, d, Q9, reac10,
                     ind10, e);
  PBMP_HIP(hipGetLastError());
}

}  // namespace pbmp
