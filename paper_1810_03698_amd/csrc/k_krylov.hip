// FP64 vector kernels of the device GMRES (Saad-Schultz, restarted, right
// preconditioned with the 2x2 panel blocks of the singular entries).  All
// reductions are two-pass with a fixed order, so results are reproducible.
#include "kernels.hpp"

namespace pbmp {

namespace {

constexpr int kB = 256;

__global__ __launch_bounds__(kB) void k_mdot_partial(int n, const double *__restrict__ V,
                                                     size_t ld,
                                                     const double *__restrict__ w,
                                                     int per_block,
                                                     double *__restrict__ partial) {
  __shared__ double red[kB];
  const int k = blockIdx.y;
  const int b = blockIdx.x;
  const int i0 = b * per_block, i1 = min(n, i0 + per_block);
  const double *v = V + (size_t)k * ld;
  double acc = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kB) acc += v[i] * w[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(size_t)k * gridDim.x + b] = red[0];
}

__global__ void k_mdot_final(int nv, int nblk, const double *__restrict__ partial,
                             double *__restrict__ h) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nv) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[(size_t)k * nblk + b];
  h[k] = s;
}

__global__ void k_gemv_sub(int n, int nv, const double *__restrict__ V, size_t ld,
                           const double *__restrict__ h, double *__restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < nv; ++k) s += V[(size_t)k * ld + i] * h[k];
  w[i] -= s;
}

// The Arnoldi step's reductions without separate final passes: every
// block of the consuming kernel adds the k_mdot_partial block sums itself
// (nv * nblk values, in the order of k_mdot_final, so all blocks hold the
// same totals) and block 0 also stores them for the host.
constexpr int kMaxNV = 256;

__device__ inline void sum_partials(int nv, int nblk, const double *__restrict__ partial,
                                    double *h, double *__restrict__ hout) {
  for (int k = threadIdx.x; k < nv; k += blockDim.x) {
    const double *pk = partial + (size_t)k * nblk;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += pk[b];
    h[k] = s;
    if (blockIdx.x == 0) hout[k] = s;
  }
  __syncthreads();
}

// w -= V h with h summed from the partials (stored to hout by block 0)
__global__ __launch_bounds__(kB) void k_gemv_sub_p(int n, int nv, const double *__restrict__ V,
                                                   size_t ld, int nblk,
                                                   const double *__restrict__ partial,
                                                   double *__restrict__ hout,
                                                   double *__restrict__ w) {
  __shared__ double h[kMaxNV];
  sum_partials(nv, nblk, partial, h, hout);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < nv; ++k) s += V[(size_t)k * ld + i] * h[k];
  w[i] -= s;
}

// v = w / |w| with |w|^2 summed from the partials (stored to hout by block 0)
__global__ __launch_bounds__(kB) void k_scale_inv_sqrt_p(int n, int nblk,
                                                         const double *__restrict__ partial,
                                                         double *__restrict__ hout,
                                                         const double *__restrict__ w,
                                                         double *__restrict__ v) {
  __shared__ double h[1];
  sum_partials(1, nblk, partial, h, hout);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double q = h[0];
  v[i] = q > 0.0 ? w[i] / sqrt(q) : 0.0;
}

// v = w / sqrt(nrm2); a zero vector (Arnoldi breakdown) stays zero
__global__ void k_scale_inv_sqrt(int n, const double *__restrict__ w,
                                 const double *__restrict__ nrm2,
                                 double *__restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double q = *nrm2;
  v[i] = q > 0.0 ? w[i] / sqrt(q) : 0.0;
}

__global__ void k_axpy(int n, double a, const double *__restrict__ x,
                       double *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

__global__ void k_scale(int n, double a, const double *__restrict__ x,
                        double *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

__global__ void k_xmy(int n, const double *__restrict__ b,
                      const double *__restrict__ ax, double *__restrict__ r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r[i] = b[i] - ax[i];
}

// block [[1/2, -a], [1/2, e b]]^{-1} = 1/det [[e b, a], [-1/2, 1/2]],
// det = (e b + a) / 2
__device__ inline void block_solve(double a, double b, double e, double u1,
                                   double u2, double &z1, double &z2) {
  const double det = 0.5 * (e * b + a);
  z1 = (e * b * u1 + a * u2) / det;
  z2 = (-0.5 * u1 + 0.5 * u2) / det;
}

__global__ void k_precond(int N, const double *__restrict__ diag, double e,
                          const double *__restrict__ u, double *__restrict__ z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double z1, z2;
  block_solve(diag[i], diag[N + i], e, u[i], u[N + i], z1, z2);
  z[i] = z1;
  z[N + i] = z2;
}

// z = M^{-1} u (as k_precond) and the far-field strengths of z packed into
// the source records (as k_pack_strengths): the Arnoldi step's product
// input in one launch
__global__ void k_precond_pack(int N, int nf, const double *__restrict__ diag, double e,
                               const double *__restrict__ geo, const double *__restrict__ u,
                               double *__restrict__ z, double *__restrict__ src64,
                               float *__restrict__ src32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double z1, z2;
  block_solve(diag[i], diag[N + i], e, u[i], u[N + i], z1, z2);
  z[i] = z1;
  z[N + i] = z2;
  const double wA = geo[6 * N + i] * 0.07957747154594767 / nf;  // A / (4 pi nf)
  const double sv = wA * z2, sk = wA * z1;
  src64[16 * (size_t)i + 13] = sv;
  src64[16 * (size_t)i + 14] = sk;
  src32[16 * (size_t)i + 13] = (float)sv;
  src32[16 * (size_t)i + 14] = (float)sk;
}

__global__ void k_update_solution(int N, int nv, const double *__restrict__ V,
                                  size_t ld, const double *__restrict__ y,
                                  const double *__restrict__ diag, double e,
                                  double *__restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double u1 = 0.0, u2 = 0.0;
  for (int k = 0; k < nv; ++k) {
    u1 += V[(size_t)k * ld + i] * y[k];
    u2 += V[(size_t)k * ld + N + i] * y[k];
  }
  double z1, z2;
  block_solve(diag[i], diag[N + i], e, u1, u2, z1, z2);
  x[i] += z1;
  x[N + i] += z2;
}

__global__ void k_permute(int n, int blocks, const int *__restrict__ perm,
                          const double *__restrict__ in, double *__restrict__ out,
                          int gather) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * blocks) return;
  const int b = t / n, i = t % n;
  const size_t o = (size_t)b * n;
  if (gather)
    out[o + i] = in[o + perm[i]];
  else
    out[o + perm[i]] = in[o + i];
}

inline dim3 g1(int n) { return dim3((n + kB - 1) / kB); }

}  // namespace

void launch_mdot(hipStream_t s, int n, int nv, const double *V, size_t ld,
                 const double *w, double *partial, double *h) {
  const int per = 4096;
  const int nblk = (n + per - 1) / per;
  hipLaunchKernelGGL(k_mdot_partial, dim3(nblk, nv), dim3(kB), 0, s, n, V, ld,
                     w, per, partial);
  hipLaunchKernelGGL(k_mdot_final, dim3((nv + 63) / 64), dim3(64), 0, s, nv,
                     nblk, partial, h);
  PBMP_HIP(hipGetLastError());
}

int launch_mdot_partial(hipStream_t s, int n, int nv, const double *V, size_t ld,
                        const double *w, double *partial) {
  const int per = 4096;
  const int nblk = (n + per - 1) / per;
  hipLaunchKernelGGL(k_mdot_partial, dim3(nblk, nv), dim3(kB), 0, s, n, V, ld, w, per,
                     partial);
  PBMP_HIP(hipGetLastError());
  return nblk;
}

void launch_gemv_sub_p(hipStream_t s, int n, int nv, const double *V, size_t ld, int nblk,
                       const double *partial, double *hout, double *w) {
  if (nv > kMaxNV) throw Error(PBMP_EARG, "too many Krylov vectors");
  hipLaunchKernelGGL(k_gemv_sub_p, g1(n), dim3(kB), 0, s, n, nv, V, ld, nblk, partial, hout, w);
  PBMP_HIP(hipGetLastError());
}

void launch_scale_inv_sqrt_p(hipStream_t s, int n, int nblk, const double *partial,
                             double *hout, const double *w, double *v) {
  hipLaunchKernelGGL(k_scale_inv_sqrt_p, g1(n), dim3(kB), 0, s, n, nblk, partial, hout, w, v);
  PBMP_HIP(hipGetLastError());
}

void launch_gemv_sub(hipStream_t s, int n, int nv, const double *V, size_t ld,
                     const double *h, double *w) {
  hipLaunchKernelGGL(k_gemv_sub, g1(n), dim3(kB), 0, s, n, nv, V, ld, h, w);
  PBMP_HIP(hipGetLastError());
}

void launch_scale_inv_sqrt(hipStream_t s, int n, const double *w,
                           const double *nrm2, double *v) {
  hipLaunchKernelGGL(k_scale_inv_sqrt, g1(n), dim3(kB), 0, s, n, w, nrm2, v);
  PBMP_HIP(hipGetLastError());
}

void launch_axpy(hipStream_t s, int n, double a, const double *x, double *y) {
  hipLaunchKernelGGL(k_axpy, g1(n), dim3(kB), 0, s, n, a, x, y);
  PBMP_HIP(hipGetLastError());
}

void launch_scale(hipStream_t s, int n, double a, const double *x, double *y) {
  hipLaunchKernelGGL(k_scale, g1(n), dim3(kB), 0, s, n, a, x, y);
  PBMP_HIP(hipGetLastError());
}

void launch_xmy(hipStream_t s, int n, const double *b, const double *ax,
                double *r) {
  hipLaunchKernelGGL(k_xmy, g1(n), dim3(kB), 0, s, n, b, ax, r);
  PBMP_HIP(hipGetLastError());
}

void launch_precond(hipStream_t s, int N, const double *diag, double eps_ratio,
                    const double *u, double *z) {
  hipLaunchKernelGGL(k_precond, g1(N), dim3(kB), 0, s, N, diag, eps_ratio, u, z);
  PBMP_HIP(hipGetLastError());
}

void launch_precond_pack(hipStream_t s, int N, int nf, const double *diag, double eps_ratio,
                         const double *geo, const double *u, double *z, double *src64,
                         float *src32) {
  hipLaunchKernelGGL(k_precond_pack, g1(N), dim3(kB), 0, s, N, nf, diag, eps_ratio, geo, u, z,
                     src64, src32);
  PBMP_HIP(hipGetLastError());
}

void launch_update_solution(hipStream_t s, int N, int nv, const double *V,
                            size_t ld, const double *y, const double *diag,
                            double eps_ratio, double *x) {
  hipLaunchKernelGGL(k_update_solution, g1(N), dim3(kB), 0, s, N, nv, V, ld, y,
                     diag, eps_ratio, x);
  PBMP_HIP(hipGetLastError());
}

void launch_permute(hipStream_t s, int n, int blocks, const int *perm,
                    const double *in, double *out, bool gather) {
  hipLaunchKernelGGL(k_permute, g1(n * blocks), dim3(kB), 0, s, n, blocks, perm,
                     in, out, gather ? 1 : 0);
  PBMP_HIP(hipGetLastError());
}

namespace {
__global__ void k_add_strided(int n, double sign, const double *__restrict__ p, int stride,
                              double *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += sign * p[(size_t)stride * i];
}
}  // namespace

// y[i] += sign * p[stride * i]
void launch_add_strided(hipStream_t s, int n, double sign, const double *p, int stride,
                        double *y) {
  hipLaunchKernelGGL(k_add_strided, dim3((n + 255) / 256), dim3(256), 0, s, n, sign, p, stride,
                     y);
  PBMP_HIP(hipGetLastError());
}

}  // namespace pbmp
