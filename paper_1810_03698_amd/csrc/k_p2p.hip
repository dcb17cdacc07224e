// Far-field source-target (P2P) sums of the boundary-integral operator
// (section "The treecode algorithm": the product is an N-body problem with
// the Gauss nodes as sources and the collocation points as targets), and the
// step that turns the four operator sums into y = A x (eq. integral_eq).
//
// Layout: one target per lane (TPT targets per thread), source panels staged
// through LDS in tiles; every lane reads the same panel record (LDS
// broadcast).  A panel record is 16 words: three far-field nodes, the unit
// normal, the plane offset n.y and the two strengths s_V, s_K.  Because the
// nodes of a flat panel share its plane, n.(x - y_q) = n.x - n.y0 for all q.
//
// Per (target, node) pair the four kernels need one reciprocal square root
// and one exponential:  V_L += 1/r, V_Y += e^{-kr}/r, K_L += 1/r^3,
// K_Y += (1 + kr) e^{-kr}/r^3; the panel's sums are then weighted by s_V and
// s_K n.R.  FP32 variant: per-tile FP32 sums folded into FP64 accumulators.
#include <cmath>

#include "kernels.hpp"
#include "pair.hpp"

namespace pbmp {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;
constexpr int kBlock = 256;
constexpr int kTile = 128;  // panels per LDS tile

__global__ void k_pack_strengths(int N, int nf, const double *__restrict__ geo,
                                 const double *__restrict__ x,
                                 double *__restrict__ src64,
                                 float *__restrict__ src32) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const double wA = geo[6 * N + j] * kInv4Pi / nf;  // equal-weight rules
  const double sv = wA * x[N + j];
  const double sk = wA * x[j];
  src64[16 * (size_t)j + 13] = sv;
  src64[16 * (size_t)j + 14] = sk;
  src32[16 * (size_t)j + 13] = (float)sv;
  src32[16 * (size_t)j + 14] = (float)sk;
}

template <int NF, int TPT, bool FLOOR>
__global__ __launch_bounds__(kBlock) void k_p2p_f32(
    const float4 *__restrict__ src, int N, const float *__restrict__ tgt,
    int Nt, int chunk, float kappa, float nk_log2e, double *__restrict__ part) {
  __shared__ float4 sh[kTile * 4];
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(N, j0 + chunk);
  float px[TPT], py[TPT], pz[TPT];
  int ti[TPT];
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    ti[k] = blockIdx.x * (kBlock * TPT) + k * kBlock + threadIdx.x;
    const int tl = min(ti[k], Nt - 1);
    px[k] = tgt[tl];
    py[k] = tgt[Nt + tl];
    pz[k] = tgt[2 * Nt + tl];
  }
  double S[TPT][4];
#pragma unroll
  for (int k = 0; k < TPT; ++k)
    for (int c = 0; c < 4; ++c) S[k][c] = 0.0;

  for (int jt = j0; jt < j1; jt += kTile) {
    const int nj = min(kTile, j1 - jt);
    __syncthreads();
    for (int e = threadIdx.x; e < nj * 4; e += kBlock) sh[e] = src[(size_t)jt * 4 + e];
    __syncthreads();
    float a[TPT][4];
#pragma unroll
    for (int k = 0; k < TPT; ++k)
      for (int c = 0; c < 4; ++c) a[k][c] = 0.0f;
    for (int jj = 0; jj < nj; ++jj) {
      const float4 r0 = sh[4 * jj], r1 = sh[4 * jj + 1], r2 = sh[4 * jj + 2],
                   r3 = sh[4 * jj + 3];
      // r0 = y0x y0y y0z y1x | r1 = y1y y1z y2x y2y | r2 = y2z nx ny nz
      // r3 = n.y0, s_V, s_K, 0
      const float yx[3] = {r0.x, r0.w, r1.z};
      const float yy[3] = {r0.y, r1.x, r1.w};
      const float yz[3] = {r0.z, r1.y, r2.x};
#pragma unroll
      for (int k = 0; k < TPT; ++k) {
        // single layer accumulated per node with the strength; double layer
        // per panel (shared n.R): kl = sum 1/r^3, A = sum e/r^3, B = sum e/r^2
        float kl = 0.f, A = 0.f, B = 0.f;
        float d0x = 0.f, d0y = 0.f, d0z = 0.f;
#pragma unroll
        for (int q = 0; q < NF; ++q) {
          const float dx = px[k] - yx[q], dy = py[k] - yy[q], dz = pz[k] - yz[q];
          if (q == 0) {
            d0x = dx;
            d0y = dy;
            d0z = dz;
          }
          float ri, er;
          node_core<FLOOR>(dx, dy, dz, nk_log2e, ri, er);
          const float ri2 = ri * ri;
          a[k][0] = fmaf(r3.y, ri, a[k][0]);
          a[k][2] = fmaf(r3.y, er, a[k][2]);
          kl = fmaf(ri2, ri, kl);
          A = fmaf(er, ri2, A);
          B = fmaf(er, ri, B);
        }
        const float nR = normal_dist(r2.y, r2.z, r2.w, d0x, d0y, d0z);
        const float skn = r3.z * nR;
        a[k][1] = fmaf(skn, kl, a[k][1]);
        a[k][3] = fmaf(skn, fmaf(kappa, B, A), a[k][3]);
      }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k)
      for (int c = 0; c < 4; ++c) S[k][c] += (double)a[k][c];
  }
#pragma unroll
  for (int k = 0; k < TPT; ++k)
    if (ti[k] < Nt)
      for (int c = 0; c < 4; ++c)
        part[((size_t)blockIdx.y * 4 + c) * Nt + ti[k]] = S[k][c];
}

template <int NF>
__global__ __launch_bounds__(kBlock) void k_p2p_f64(
    const double *__restrict__ src, int N, const double *__restrict__ geo,
    int Nt, int chunk, double kappa, double *__restrict__ part) {
  constexpr int kTile64 = 64;
  __shared__ double sh[kTile64 * 16];
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(N, j0 + chunk);
  const int ti = blockIdx.x * kBlock + threadIdx.x;
  const int tl = min(ti, Nt - 1);
  const double px = geo[tl], py = geo[Nt + tl], pz = geo[2 * Nt + tl];
  double S[4] = {0.0, 0.0, 0.0, 0.0};
  for (int jt = j0; jt < j1; jt += kTile64) {
    const int nj = min(kTile64, j1 - jt);
    __syncthreads();
    for (int e = threadIdx.x; e < nj * 16; e += kBlock) sh[e] = src[(size_t)jt * 16 + e];
    __syncthreads();
    for (int jj = 0; jj < nj; ++jj) {
      const double *r = sh + 16 * jj;
      double t[4];
      panel_terms<double>(r, NF, px, py, pz, kappa, 0.0, t);
      S[0] += r[13] * t[0];
      S[1] += r[14] * t[1];
      S[2] += r[13] * t[2];
      S[3] += r[14] * t[3];
    }
  }
  if (ti < Nt)
    for (int c = 0; c < 4; ++c) part[((size_t)blockIdx.y * 4 + c) * Nt + ti] = S[c];
}

__global__ void k_finish(int N, int nchunk, const double *__restrict__ part,
                         const int *__restrict__ rowptr,
                         const int *__restrict__ col,
                         const double *__restrict__ val,
                         const double *__restrict__ x, double eps_ratio,
                         double *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double S[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c = 0; c < nchunk; ++c)
    for (int k = 0; k < 4; ++k) S[k] += part[((size_t)c * 4 + k) * N + i];
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const int j = col[e];
    const double ph = x[j], dp = x[N + j];
    S[0] += val[4 * (size_t)e] * dp;
    S[1] += val[4 * (size_t)e + 1] * ph;
    S[2] += val[4 * (size_t)e + 2] * dp;
    S[3] += val[4 * (size_t)e + 3] * ph;
  }
  const double ph = x[i];
  y[i] = 0.5 * ph + S[1] - S[0];
  y[N + i] = 0.5 * ph - S[3] + eps_ratio * S[2];
}

// Transposed far-field sums: targets are the far-field nodes of panel j
// (normal n_j), sources the collocation points c_i with weights z1_i, z2_i:
//   T_VL_j = sum_q w A_j/(4 pi) sum_i z1_i / r,   T_KL_j = ... z1_i n_j.(c_i - y)/r^3
//   T_VY_j = ... z2_i e^{-kr}/r,                   T_KY_j = ... z2_i n_j.(c_i-y)(1+kr)e^{-kr}/r^3
template <class T>
__global__ __launch_bounds__(kBlock) void k_p2p_transpose(
    int N, int nf, const T *__restrict__ src, const T *__restrict__ tgt,
    const double *__restrict__ geo, const double *__restrict__ z, int chunk,
    T kappa, T nk, double *__restrict__ part) {
  __shared__ T sh[kTile * 5];
  const int j = blockIdx.x * kBlock + threadIdx.x;
  const int jl = min(j, N - 1);
  T rec[16];
  for (int k = 0; k < 16; ++k) rec[k] = src[16 * (size_t)jl + k];
  const int i0 = blockIdx.y * chunk, i1 = min(N, i0 + chunk);
  double S[4] = {0.0, 0.0, 0.0, 0.0};
  for (int it = i0; it < i1; it += kTile) {
    const int ni = min(kTile, i1 - it);
    __syncthreads();
    for (int e = threadIdx.x; e < ni; e += kBlock) {
      const int i = it + e;
      sh[5 * e] = tgt[i];
      sh[5 * e + 1] = tgt[N + i];
      sh[5 * e + 2] = tgt[2 * N + i];
      sh[5 * e + 3] = (T)z[i];
      sh[5 * e + 4] = (T)z[N + i];
    }
    __syncthreads();
    T a[4] = {T(0), T(0), T(0), T(0)};
    for (int e = 0; e < ni; ++e) {
      T t[4];
      panel_terms<T>(rec, nf, sh[5 * e], sh[5 * e + 1], sh[5 * e + 2], kappa, nk, t);
      const T z1 = sh[5 * e + 3], z2 = sh[5 * e + 4];
      a[0] += z1 * t[0];
      a[1] += z1 * t[1];
      a[2] += z2 * t[2];
      a[3] += z2 * t[3];
    }
    for (int c = 0; c < 4; ++c) S[c] += (double)a[c];
  }
  if (j < N) {
    const double wA = geo[6 * N + j] * kInv4Pi / nf;
    for (int c = 0; c < 4; ++c) part[((size_t)blockIdx.y * 4 + c) * N + j] = wA * S[c];
  }
}

// (A^T z) from the transposed far partials, the transposed near/self
// correction (entries of column j) and the identity terms.
__global__ void k_finish_transpose(int N, int nchunk, const double *__restrict__ part,
                                   const int *__restrict__ trow,
                                   const int *__restrict__ tcol,
                                   const int *__restrict__ tent,
                                   const double *__restrict__ val,
                                   const double *__restrict__ z, double eps_ratio,
                                   double *__restrict__ y) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double S[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c = 0; c < nchunk; ++c)
    for (int k = 0; k < 4; ++k) S[k] += part[((size_t)c * 4 + k) * N + j];
  for (int t = trow[j]; t < trow[j + 1]; ++t) {
    const int i = tcol[t];
    const size_t e = tent[t];
    S[0] += val[4 * e] * z[i];
    S[1] += val[4 * e + 1] * z[i];
    S[2] += val[4 * e + 2] * z[N + i];
    S[3] += val[4 * e + 3] * z[N + i];
  }
  y[j] = 0.5 * z[j] + S[1] + 0.5 * z[N + j] - S[3];
  y[N + j] = -S[0] + eps_ratio * S[2];
}

}  // namespace

void launch_pack_strengths(hipStream_t s, int N, int nf, const double *geo,
                           const double *x, double *src64, float *src32) {
  hipLaunchKernelGGL(k_pack_strengths, dim3((N + 255) / 256), dim3(256), 0, s,
                     N, nf, geo, x, src64, src32);
  PBMP_HIP(hipGetLastError());
}

void launch_p2p_direct(hipStream_t s, bool fp64, int nf, int N, int Nt,
                       const double *src64, const float *src32,
                       const double *geo, const float *tgt32, double kappa,
                       int nchunk, double *part, bool floor_r2) {
  const int chunk = (N + nchunk - 1) / nchunk;
  if (fp64) {
    dim3 grid((Nt + kBlock - 1) / kBlock, nchunk);
    if (nf == 3)
      hipLaunchKernelGGL(k_p2p_f64<3>, grid, dim3(kBlock), 0, s, src64, N, geo,
                         Nt, chunk, kappa, part);
    else
      hipLaunchKernelGGL(k_p2p_f64<1>, grid, dim3(kBlock), 0, s, src64, N, geo,
                         Nt, chunk, kappa, part);
  } else {
    constexpr int TPT = 2;
    dim3 grid((Nt + kBlock * TPT - 1) / (kBlock * TPT), nchunk);
    const float kf = (float)kappa;
    const float nk = (float)(-kappa * 1.4426950408889634);
    const float4 *s4 = reinterpret_cast<const float4 *>(src32);
#define PBMP_P2P(NFV, FL)                                                      \
  hipLaunchKernelGGL((k_p2p_f32<NFV, TPT, FL>), grid, dim3(kBlock), 0, s, s4, N, \
                     tgt32, Nt, chunk, kf, nk, part)
    if (nf == 3 && floor_r2) PBMP_P2P(3, true);
    else if (nf == 3) PBMP_P2P(3, false);
    else if (floor_r2) PBMP_P2P(1, true);
    else PBMP_P2P(1, false);
#undef PBMP_P2P
  }
  PBMP_HIP(hipGetLastError());
}

void launch_finish(hipStream_t s, int N, int nchunk, const double *part,
                   const int *rowptr, const int *col, const double *val,
                   const double *x, double eps_ratio, double *y) {
  hipLaunchKernelGGL(k_finish, dim3((N + 255) / 256), dim3(256), 0, s, N,
                     nchunk, part, rowptr, col, val, x, eps_ratio, y);
  PBMP_HIP(hipGetLastError());
}

}  // namespace pbmp

namespace pbmp {
void launch_transpose(hipStream_t s, bool fp64, int nf, int N,
                      const double *src64, const float *src32,
                      const double *geo, const float *tgt32, const double *z,
                      double kappa, int nchunk, double *part,
                      const int *trow, const int *tcol, const int *tent,
                      const double *val, double eps_ratio, double *y) {
  const int chunk = (N + nchunk - 1) / nchunk;
  dim3 grid((N + kBlock - 1) / kBlock, nchunk);
  if (fp64)
    hipLaunchKernelGGL(k_p2p_transpose<double>, grid, dim3(kBlock), 0, s, N, nf,
                       src64, geo, geo, z, chunk, kappa, 0.0, part);
  else
    hipLaunchKernelGGL(k_p2p_transpose<float>, grid, dim3(kBlock), 0, s, N, nf,
                       src32, tgt32, geo, z, chunk, (float)kappa,
                       (float)(-kappa * 1.4426950408889634), part);
  PBMP_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_finish_transpose, dim3((N + 255) / 256), dim3(256), 0, s,
                     N, nchunk, part, trow, tcol, tent, val, z, eps_ratio, y);
  PBMP_HIP(hipGetLastError());
}
}  // namespace pbmp
