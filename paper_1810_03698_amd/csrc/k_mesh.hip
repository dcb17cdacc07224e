// Per-mesh kernels: panel geometry, singular and near-singular corrections,
// winding numbers.  All FP64 (section "The boundary element method":
// singular, near-singular and far integration regions).
#include <cmath>

#include "kernels.hpp"
#include "pair.hpp"
#include "panel.hpp"

namespace pbmp {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;  // 1 / (4 pi)

__device__ inline void load_tri(const double *verts, const int *tri, int j,
                                double v[3][3]) {
  for (int k = 0; k < 3; ++k) {
    const int iv = tri[3 * j + k];
    v[k][0] = verts[3 * iv];
    v[k][1] = verts[3 * iv + 1];
    v[k][2] = verts[3 * iv + 2];
  }
}

__global__ void k_panel_geometry(int N, const double *__restrict__ verts,
                                 const int *__restrict__ tri, RuleArgs ru,
                                 double *__restrict__ geo,
                                 double *__restrict__ src64,
                                 float *__restrict__ src32,
                                 float *__restrict__ tgt32) {
  // Same IEEE operation order as a plain sequential evaluation (no
  // contraction), so that near/far decisions are reproducible.
#pragma clang fp contract(off)
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double v[3][3];
  load_tri(verts, tri, j, v);
  double e1[3], e2[3];
  for (int d = 0; d < 3; ++d) {
    e1[d] = v[1][d] - v[0][d];
    e2[d] = v[2][d] - v[0][d];
  }
  const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1],
                        e1[2] * e2[0] - e1[0] * e2[2],
                        e1[0] * e2[1] - e1[1] * e2[0]};
  const double nn = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
  double c[3], n[3];
  for (int d = 0; d < 3; ++d) {
    c[d] = (v[0][d] + v[1][d] + v[2][d]) / 3.0;
    n[d] = cr[d] / nn;
  }
  for (int d = 0; d < 3; ++d) {
    geo[d * N + j] = c[d];
    geo[(3 + d) * N + j] = n[d];
    tgt32[d * N + j] = (float)c[d];
  }
  geo[6 * N + j] = 0.5 * nn;
  double rec[16];
  for (int k = 0; k < 16; ++k) rec[k] = 0.0;
  for (int q = 0; q < ru.nf; ++q)
    for (int d = 0; d < 3; ++d)
      rec[3 * q + d] = ru.fb[q][0] * v[0][d] + ru.fb[q][1] * v[1][d] + ru.fb[q][2] * v[2][d];
  for (int d = 0; d < 3; ++d) rec[9 + d] = n[d];
  rec[12] = n[0] * rec[0] + n[1] * rec[1] + n[2] * rec[2];
  for (int k = 0; k < 13; ++k) {
    src64[16 * (size_t)j + k] = rec[k];
    src32[16 * (size_t)j + k] = (float)rec[k];
  }
}

__global__ void k_near_values(int fp64, int N, const int *__restrict__ rowptr,
                              const int *__restrict__ col,
                              const double *__restrict__ verts,
                              const int *__restrict__ tri,
                              const double *__restrict__ geo,
                              const double *__restrict__ src64,
                              const float *__restrict__ src32,
                              const float *__restrict__ tgt32, RuleArgs ru,
                              double kappa, double *__restrict__ val,
                              double *__restrict__ diag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double x[3] = {geo[i], geo[N + i], geo[2 * N + i]};
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const int j = col[e];
    double v[3][3];
    load_tri(verts, tri, j, v);
    const double n[3] = {geo[3 * N + j], geo[4 * N + j], geo[5 * N + j]};
    const double A = geo[6 * N + j];
    double fine[4], coarse[4];
    if (j == i) {
      singular_panel_t<double>(v, x, kappa, ru, fine[0], fine[2]);
      fine[1] = 0.0;
      fine[3] = 0.0;
      diag[i] = fine[0];
      diag[N + i] = fine[2];
    } else {
      panel_rule_t<double>(v, n, A, x, ru.nn, ru.nb, ru.nw, kappa, fine);
    }
    // the far-rule value exactly as the far-field product evaluates it
    const double wA = A * kInv4Pi / ru.nf;
    if (fp64) {
      double t[4];
      panel_terms<double>(src64 + 16 * (size_t)j, ru.nf, x[0], x[1], x[2], kappa,
                          0.0, t);
      for (int k = 0; k < 4; ++k) coarse[k] = wA * t[k];
    } else {
      float t[4];
      panel_terms<float>(src32 + 16 * (size_t)j, ru.nf, tgt32[i], tgt32[N + i],
                         tgt32[2 * N + i], (float)kappa,
                         (float)(-kappa * 1.4426950408889634), t);
      for (int k = 0; k < 4; ++k) coarse[k] = wA * (double)t[k];
    }
    for (int k = 0; k < 4; ++k) val[4 * (size_t)e + k] = fine[k] - coarse[k];
  }
}

// Winding number of point p: sum of signed solid angles / (4 pi), with the
// triangle solid angle of Van Oosterom and Strackee.
__global__ void k_winding(int N, const double *__restrict__ verts,
                          const int *__restrict__ tri,
                          const double *__restrict__ pts,
                          double *__restrict__ wind) {
  __shared__ double red[256];
  const int l = blockIdx.x;
  const double p[3] = {pts[3 * l], pts[3 * l + 1], pts[3 * l + 2]};
  double acc = 0.0;
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    double v[3][3];
    load_tri(verts, tri, j, v);
    double a[3], b[3], c[3];
    for (int d = 0; d < 3; ++d) {
      a[d] = v[0][d] - p[d];
      b[d] = v[1][d] - p[d];
      c[d] = v[2][d] - p[d];
    }
    const double la = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    const double lb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    const double lc = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    const double trip = a[0] * (b[1] * c[2] - b[2] * c[1]) +
                        a[1] * (b[2] * c[0] - b[0] * c[2]) +
                        a[2] * (b[0] * c[1] - b[1] * c[0]);
    const double ab = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    const double ac = a[0] * c[0] + a[1] * c[1] + a[2] * c[2];
    const double bc = b[0] * c[0] + b[1] * c[1] + b[2] * c[2];
    acc += 2.0 * atan2(trip, la * lb * lc + ab * lc + ac * lb + bc * la);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) wind[l] = red[0] * kInv4Pi;
}

}  // namespace

void launch_panel_geometry(hipStream_t s, int N, const double *verts,
                           const int *tri, const RuleArgs &ru, double *geo,
                           double *src64, float *src32, float *tgt32) {
  if (N <= 0) return;
  PBMP_HIP(hipMemsetAsync(src64, 0, sizeof(double) * 16 * (size_t)N, s));
  PBMP_HIP(hipMemsetAsync(src32, 0, sizeof(float) * 16 * (size_t)N, s));
  hipLaunchKernelGGL(k_panel_geometry, dim3((N + 255) / 256), dim3(256), 0, s,
                     N, verts, tri, ru, geo, src64, src32, tgt32);
  PBMP_HIP(hipGetLastError());
}

void launch_near_values(hipStream_t s, bool fp64, int N, const int *rowptr,
                        const int *col, const double *verts, const int *tri,
                        const double *geo, const double *src64,
                        const float *src32, const float *tgt32,
                        const RuleArgs &ru, double kappa, double *val,
                        double *diag) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_near_values, dim3((N + 127) / 128), dim3(128), 0, s,
                     fp64 ? 1 : 0, N, rowptr, col, verts, tri, geo, src64, src32,
                     tgt32, ru, kappa, val, diag);
  PBMP_HIP(hipGetLastError());
}

void launch_winding(hipStream_t s, int N, int M, const double *verts,
                    const int *tri, const double *pts, double *wind) {
  if (M <= 0) return;
  hipLaunchKernelGGL(k_winding, dim3(M), dim3(256), 0, s, N, verts, tri, pts,
                     wind);
  PBMP_HIP(hipGetLastError());
}

}  // namespace pbmp
