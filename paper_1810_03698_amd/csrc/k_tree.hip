// Treecode product (section "The treecode algorithm"): Cartesian Taylor
// expansion of the kernels about box centres.
//
//   G(x, y_c + h) = sum_{|k|<=P} a_k(x) h^k,   a_k = (1/k!) D_y^k G(x, y_c)
//
// With D = x - y_c the coefficients follow the recurrences of Lindsay-Krasny
// (Laplace, G = 1/r) and Li-Johnston-Krasny (Yukawa, G = e^{-kr}/r, with
// auxiliary coefficients b_k of e^{-kr}); n = |k|:
//   n |D|^2 a_k = (2n-1) sum_i D_i a_{k-e_i} - (n-1) sum_i a_{k-2e_i}
//                 + kappa (sum_i D_i b_{k-e_i} - sum_i b_{k-2e_i}),
//   n b_k       = kappa (sum_i D_i a_{k-e_i} - sum_i a_{k-2e_i}),
// a_0 = e^{-k|D|}/|D|, b_0 = e^{-k|D|} (kappa = 0: Laplace).  Box moments
//   single layer  m_k  = sum_nodes s_V h^k,
//   double layer  mK_k = sum_nodes s_K sum_i k_i n_i h^{k-e_i}
// (the double-layer kernel is n.grad_y G) give V = sum a_k m_k and
// K = sum a_k mK_k.  Moments are formed at the leaves (P2M) and shifted up
// the tree (M2M, binomial expansion of (h + t)^k), in FP64.
#include <cmath>

#include "kernels.hpp"
#include "pair.hpp"
#include "runtime.hpp"

namespace pbmp {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;

// Multi-indices |k| <= P ordered by degree, then x exponent descending,
// then y exponent descending; m1/m2: positions of k - e_i and k - 2 e_i.
template <int P> struct Multi {
  static constexpr int n = (P + 1) * (P + 2) * (P + 3) / 6;
  int e[n][3];
  int m1[n][3];
  int m2[n][3];
  int deg[n];
  static constexpr int index(int i, int j, int l) {
    const int s = i + j + l;
    return s * (s + 1) * (s + 2) / 6 + (s - i) * (s - i + 1) / 2 + (s - i - j);
  }
  constexpr Multi() : e(), m1(), m2(), deg() {
    int k = 0;
    for (int s = 0; s <= P; ++s)
      for (int i = s; i >= 0; --i)
        for (int j = s - i; j >= 0; --j) {
          const int l = s - i - j;
          e[k][0] = i;
          e[k][1] = j;
          e[k][2] = l;
          deg[k] = s;
          const int ex[3] = {i, j, l};
          for (int d = 0; d < 3; ++d) {
            int a[3] = {ex[0], ex[1], ex[2]};
            a[d] -= 1;
            m1[k][d] = (a[d] >= 0) ? index(a[0], a[1], a[2]) : -1;
            a[d] -= 1;
            m2[k][d] = (a[d] >= 0) ? index(a[0], a[1], a[2]) : -1;
          }
          ++k;
        }
  }
};

inline int ncoef_of(int P) { return (P + 1) * (P + 2) * (P + 3) / 6; }

// blockIdx -> task: consecutive tasks (neighbouring target leaves, similar
// source lists) land on the same XCD so they share its L2.
__device__ inline int xcd_task(int ntasks) {
  const int per = (gridDim.x + 7) / 8;
  const int t = (blockIdx.x % 8) * per + blockIdx.x / 8;
  return t < ntasks ? t : -1;
}

// ---------------------------------------------------------------- P2M
// One block per leaf; thread k owns coefficient k.  exps [3*NC].
__global__ __launch_bounds__(64) void k_p2m(int NC, int nf,
                                            const int *__restrict__ leaves,
                                            const int *__restrict__ range,
                                            const double *__restrict__ center,
                                            const int *__restrict__ exps,
                                            const double *__restrict__ src,
                                            double *__restrict__ mom) {
  constexpr int kT = 32;
  __shared__ double sh[kT * 16];
  const int B = leaves[blockIdx.x];
  const int s0 = range[2 * B], s1 = range[2 * B + 1];
  const double cx = center[3 * B], cy = center[3 * B + 1], cz = center[3 * B + 2];
  for (int k0 = 0; k0 < NC; k0 += 64) {
    const int k = k0 + threadIdx.x;
    const bool on = k < NC;
    const int ex = on ? exps[3 * k] : 0, ey = on ? exps[3 * k + 1] : 0,
              ez = on ? exps[3 * k + 2] : 0;
    double m = 0.0, mk = 0.0;
    for (int jt = s0; jt < s1; jt += kT) {
      const int nj = min(kT, s1 - jt);
      __syncthreads();
      for (int e = threadIdx.x; e < nj * 16; e += 64) sh[e] = src[(size_t)jt * 16 + e];
      __syncthreads();
      if (!on) continue;
      for (int jj = 0; jj < nj; ++jj) {
        const double *r = sh + 16 * jj;
        for (int q = 0; q < nf; ++q) {
          const double h[3] = {r[3 * q] - cx, r[3 * q + 1] - cy, r[3 * q + 2] - cz};
          double px[9], py[9], pz[9];
          px[0] = py[0] = pz[0] = 1.0;
          for (int t = 1; t <= 8; ++t) {
            px[t] = px[t - 1] * h[0];
            py[t] = py[t - 1] * h[1];
            pz[t] = pz[t - 1] * h[2];
          }
          m += r[13] * px[ex] * py[ey] * pz[ez];
          double dk = 0.0;
          if (ex) dk += ex * r[9] * px[ex - 1] * py[ey] * pz[ez];
          if (ey) dk += ey * r[10] * px[ex] * py[ey - 1] * pz[ez];
          if (ez) dk += ez * r[11] * px[ex] * py[ey] * pz[ez - 1];
          mk += r[14] * dk;
        }
      }
    }
    if (on) {
      mom[(size_t)B * 2 * NC + k] = m;
      mom[(size_t)B * 2 * NC + NC + k] = mk;
    }
  }
}

// ---------------------------------------------------------------- M2M
__device__ inline double binom(int n, int k) {
  double c = 1.0;
  for (int i = 1; i <= k; ++i) c = c * (n - k + i) / i;
  return c;
}

__global__ __launch_bounds__(64) void k_m2m(int NC, const int *__restrict__ boxes,
                                            const int *__restrict__ child,
                                            const double *__restrict__ center,
                                            const int *__restrict__ exps,
                                            double *__restrict__ mom) {
  const int B = boxes[blockIdx.x];
  for (int k = threadIdx.x; k < NC; k += 64) {
    const int kx = exps[3 * k], ky = exps[3 * k + 1], kz = exps[3 * k + 2];
    double m = 0.0, mk = 0.0;
    for (int c = 0; c < 8; ++c) {
      const int C = child[8 * B + c];
      if (C < 0) break;
      const double t[3] = {center[3 * C] - center[3 * B], center[3 * C + 1] - center[3 * B + 1],
                           center[3 * C + 2] - center[3 * B + 2]};
      // (h + t)^k = sum_{j <= k} C(k, j) t^{k-j} h^j
      for (int jx = 0; jx <= kx; ++jx)
        for (int jy = 0; jy <= ky; ++jy)
          for (int jz = 0; jz <= kz; ++jz) {
            const int s = jx + jy + jz;
            const int jdx = s * (s + 1) * (s + 2) / 6 + (s - jx) * (s - jx + 1) / 2 + (s - jx - jy);
            const double w = binom(kx, jx) * binom(ky, jy) * binom(kz, jz) *
                             pow(t[0], kx - jx) * pow(t[1], ky - jy) * pow(t[2], kz - jz);
            m += w * mom[(size_t)C * 2 * NC + jdx];
            mk += w * mom[(size_t)C * 2 * NC + NC + jdx];
          }
    }
    mom[(size_t)B * 2 * NC + k] = m;
    mom[(size_t)B * 2 * NC + NC + k] = mk;
  }
}

__global__ void k_cast(size_t n, const double *__restrict__ a, float *__restrict__ b) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// ------------------------------------------------------------ P2P tasks
// One 64-lane block per task: targets [t0, t1) of a leaf (TPT per lane),
// sources = panels of the listed leaves, streamed through LDS.
constexpr int kTileT = 128;

template <class T, int NF, int TPT>
__device__ void p2p_task_body(const T *__restrict__ src, const T *__restrict__ tgt,
                              int N, int t0, int t1, const int *__restrict__ ranges,
                              int lb, int le, T kappa, T nk, int slot,
                              double *__restrict__ part, T *sh) {
  for (int tb = t0; tb < t1; tb += 64 * TPT) {
    T px[TPT], py[TPT], pz[TPT];
    int ti[TPT];
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
      ti[k] = tb + k * 64 + (int)threadIdx.x;
      const int tl = min(ti[k], t1 - 1);
      px[k] = tgt[tl];
      py[k] = tgt[N + tl];
      pz[k] = tgt[2 * N + tl];
    }
    double S[TPT][4];
#pragma unroll
    for (int k = 0; k < TPT; ++k)
      for (int c = 0; c < 4; ++c) S[k][c] = 0.0;
    for (int l = lb; l < le; ++l) {
      const int s0 = ranges[2 * l], s1 = ranges[2 * l + 1];
      for (int jt = s0; jt < s1; jt += kTileT) {
        const int nj = min(kTileT, s1 - jt);
        __syncthreads();
        for (int e = threadIdx.x; e < nj * 16; e += 64) sh[e] = src[(size_t)jt * 16 + e];
        __syncthreads();
        T a[TPT][4];
#pragma unroll
        for (int k = 0; k < TPT; ++k)
          for (int c = 0; c < 4; ++c) a[k][c] = T(0);
        for (int jj = 0; jj < nj; ++jj) {
          const T *r = sh + 16 * jj;
#pragma unroll
          for (int k = 0; k < TPT; ++k) {
            T t4[4];
            panel_terms<T>(r, NF, px[k], py[k], pz[k], kappa, nk, t4);
            const T vl = t4[0], vy = t4[2];
            a[k][0] += r[13] * vl;
            a[k][1] += r[14] * t4[1];
            a[k][2] += r[13] * vy;
            a[k][3] += r[14] * t4[3];
          }
        }
#pragma unroll
        for (int k = 0; k < TPT; ++k)
          for (int c = 0; c < 4; ++c) S[k][c] += (double)a[k][c];
      }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k)
      if (ti[k] < t1)
        for (int c = 0; c < 4; ++c) part[((size_t)slot * 4 + c) * N + ti[k]] = S[k][c];
  }
}

template <class T, int NF>
__global__ __launch_bounds__(64) void k_p2p_tasks(int ntask, const int *__restrict__ tasks,
                                                  const int *__restrict__ slots,
                                                  const int *__restrict__ ranges,
                                                  const T *__restrict__ src,
                                                  const T *__restrict__ tgt, int N,
                                                  T kappa, T nk, double *__restrict__ part) {
  __shared__ __align__(16) T sh[kTileT * 16];
  const int task = xcd_task(ntask);
  if (task < 0) return;
  const int t0 = tasks[4 * task], t1 = tasks[4 * task + 1];
  const int lb = tasks[4 * task + 2], le = tasks[4 * task + 3];
  const int slot = slots[task];
  const int tpt = min(5, (t1 - t0 + 63) / 64);
  switch (tpt) {
    case 1: p2p_task_body<T, NF, 1>(src, tgt, N, t0, t1, ranges, lb, le, kappa, nk, slot, part, sh); break;
    case 2: p2p_task_body<T, NF, 2>(src, tgt, N, t0, t1, ranges, lb, le, kappa, nk, slot, part, sh); break;
    case 3: p2p_task_body<T, NF, 3>(src, tgt, N, t0, t1, ranges, lb, le, kappa, nk, slot, part, sh); break;
    case 4: p2p_task_body<T, NF, 4>(src, tgt, N, t0, t1, ranges, lb, le, kappa, nk, slot, part, sh); break;
    default: p2p_task_body<T, NF, 5>(src, tgt, N, t0, t1, ranges, lb, le, kappa, nk, slot, part, sh); break;
  }
}

// ------------------------------------------------------------ M2P tasks
constexpr int kChunkBoxes = 32;

template <class T> __device__ inline T rsqrt_t(T x);
template <> __device__ inline float rsqrt_t<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ inline double rsqrt_t<double>(double x) { return 1.0 / sqrt(x); }
template <class T> __device__ inline T expneg_t(T nk, T kappa, T r);
template <> __device__ inline float expneg_t<float>(float nk, float, float r) {
  return __builtin_amdgcn_exp2f(nk * r);
}
template <> __device__ inline double expneg_t<double>(double, double kappa, double r) {
  return exp(-kappa * r);
}

template <class T, int P>
__global__ __launch_bounds__(64) void k_m2p_tasks(int ntask, const int *__restrict__ tasks,
                                                  const int *__restrict__ slots,
                                                  const int *__restrict__ boxes,
                                                  const double *__restrict__ center,
                                                  const T *__restrict__ mom,
                                                  const T *__restrict__ tgt, int N,
                                                  T kappa, T nk,
                                                  double *__restrict__ part) {
  constexpr Multi<P> mi{};
  constexpr int NC = Multi<P>::n;
  __shared__ T smom[kChunkBoxes * 2 * NC];
  __shared__ T scen[kChunkBoxes * 3];
  const int task = xcd_task(ntask);
  if (task < 0) return;
  const int t0 = tasks[4 * task], t1 = tasks[4 * task + 1];
  const int lb = tasks[4 * task + 2], le = tasks[4 * task + 3];
  const int slot = slots[task];
  const int nb = le - lb;
  for (int e = threadIdx.x; e < nb * 2 * NC; e += 64) {
    const int b = e / (2 * NC), c = e % (2 * NC);
    smom[e] = mom[(size_t)boxes[lb + b] * 2 * NC + c];
  }
  for (int e = threadIdx.x; e < nb * 3; e += 64) scen[e] = (T)center[3 * boxes[lb + e / 3] + e % 3];
  __syncthreads();
  for (int t = t0 + threadIdx.x; t < t1; t += 64) {
    const T x = tgt[t], y = tgt[N + t], z = tgt[2 * N + t];
    T acc[4] = {T(0), T(0), T(0), T(0)};
    for (int b = 0; b < nb; ++b) {
      const T D[3] = {x - scen[3 * b], y - scen[3 * b + 1], z - scen[3 * b + 2]};
      const T R2 = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
      const T ri = rsqrt_t<T>(R2);
      const T iR2 = ri * ri;
      const T ek = expneg_t<T>(nk, kappa, R2 * ri);
      T a[NC], ay[NC], by[NC];
      a[0] = ri;
      by[0] = ek;
      ay[0] = ek * ri;
#pragma unroll
      for (int k = 1; k < NC; ++k) {
        const int s = mi.deg[k];
        T S1 = T(0), S2 = T(0), Y1 = T(0), Y2 = T(0), B1 = T(0), B2 = T(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          if (mi.m1[k][d] >= 0) {
            S1 += D[d] * a[mi.m1[k][d]];
            Y1 += D[d] * ay[mi.m1[k][d]];
            B1 += D[d] * by[mi.m1[k][d]];
          }
          if (mi.m2[k][d] >= 0) {
            S2 += a[mi.m2[k][d]];
            Y2 += ay[mi.m2[k][d]];
            B2 += by[mi.m2[k][d]];
          }
        }
        const T c1 = T(2 * s - 1) / T(s), c2 = T(s - 1) / T(s);
        const T ks = kappa / T(s);
        a[k] = (c1 * S1 - c2 * S2) * iR2;
        by[k] = ks * (Y1 - Y2);
        ay[k] = (c1 * Y1 - c2 * Y2 + ks * (B1 - B2)) * iR2;
      }
      const T *m = smom + b * 2 * NC;
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        acc[0] += a[k] * m[k];
        acc[1] += a[k] * m[NC + k];
        acc[2] += ay[k] * m[k];
        acc[3] += ay[k] * m[NC + k];
      }
    }
    for (int c = 0; c < 4; ++c) part[((size_t)slot * 4 + c) * N + t] = (double)acc[c];
  }
}

__global__ void k_finish_slots(int N, const int *__restrict__ tslots,
                               const double *__restrict__ part,
                               const int *__restrict__ rowptr, const int *__restrict__ col,
                               const double *__restrict__ val, const double *__restrict__ x,
                               double eps_ratio, double *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double S[4] = {0.0, 0.0, 0.0, 0.0};
  const int ns = tslots[i];
  for (int c = 0; c < ns; ++c)
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

template <class T, int P>
void launch_m2p_p(Tree &t, hipStream_t s, const T *mom, const T *tgt, int N, T kappa,
                  T nk, double *part) {
  const int nb = ((t.n_m2p_tasks + 7) / 8) * 8;
  hipLaunchKernelGGL((k_m2p_tasks<T, P>), dim3(nb), dim3(64), 0, s, t.n_m2p_tasks,
                     t.d_m2p_task.p, t.d_m2p_slot.p, t.d_m2p_box.p, t.d_center.p, mom,
                     tgt, N, kappa, nk, part);
}

template <class T>
void launch_m2p(Tree &t, hipStream_t s, const T *mom, const T *tgt, int N, T kappa, T nk,
                double *part) {
  switch (t.prm.order) {
    case 1: launch_m2p_p<T, 1>(t, s, mom, tgt, N, kappa, nk, part); break;
    case 2: launch_m2p_p<T, 2>(t, s, mom, tgt, N, kappa, nk, part); break;
    case 3: launch_m2p_p<T, 3>(t, s, mom, tgt, N, kappa, nk, part); break;
    case 4: launch_m2p_p<T, 4>(t, s, mom, tgt, N, kappa, nk, part); break;
    case 5: launch_m2p_p<T, 5>(t, s, mom, tgt, N, kappa, nk, part); break;
    case 6: launch_m2p_p<T, 6>(t, s, mom, tgt, N, kappa, nk, part); break;
    default: throw Error(PBMP_EARG, "treecode order must be 1..6");
  }
}

}  // namespace

void tree_upload_exponents(Tree &t, hipStream_t s) {
  std::vector<int> ex;
  for (int d = 0; d <= t.prm.order; ++d)
    for (int i = d; i >= 0; --i)
      for (int j = d - i; j >= 0; --j) ex.insert(ex.end(), {i, j, d - i - j});
  t.d_monos.upload(ex.data(), ex.size(), s);
}

void tree_apply(Tree &t, hipStream_t s, bool fp64, int nf, int N, const double *geo,
                const double *src64, const float *src32, const float *tgt32,
                double kappa, double *part, KernelClock &clk) {
  const int NC = t.ncoef;
  hipEvent_t e0 = clk.on ? clk.begin(s) : nullptr;
  hipLaunchKernelGGL(k_p2m, dim3(t.nleaf), dim3(64), 0, s, NC, nf, t.d_leaves.p,
                     t.d_range.p, t.d_center.p, t.d_monos.p, src64, t.d_mom64.p);
  for (size_t l = 0; l + 1 < t.level_ptr.size(); ++l) {
    const int nb = t.level_ptr[l + 1] - t.level_ptr[l];
    if (nb > 0)
      hipLaunchKernelGGL(k_m2m, dim3(nb), dim3(64), 0, s, NC,
                         t.d_leaf_boxes.p + t.level_ptr[l], t.d_child.p, t.d_center.p,
                         t.d_monos.p, t.d_mom64.p);
  }
  if (!fp64) {
    const size_t n = (size_t)t.nbox * 2 * NC;
    hipLaunchKernelGGL(k_cast, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                       t.d_mom64.p, t.d_mom32.p);
  }
  PBMP_HIP(hipGetLastError());
  if (clk.on) clk.end(s, e0, KernelClock::P2M, 0.0);

  const float nk32 = (float)(-kappa * 1.4426950408889634);
  e0 = clk.on ? clk.begin(s) : nullptr;
  const int nbp = ((t.n_p2p_tasks + 7) / 8) * 8;
  if (fp64) {
    if (nf == 3)
      hipLaunchKernelGGL((k_p2p_tasks<double, 3>), dim3(nbp), dim3(64), 0, s, t.n_p2p_tasks,
                         t.d_p2p_task.p, t.d_p2p_slot.p, t.d_p2p_src.p, src64, geo, N,
                         kappa, 0.0, part);
    else
      hipLaunchKernelGGL((k_p2p_tasks<double, 1>), dim3(nbp), dim3(64), 0, s, t.n_p2p_tasks,
                         t.d_p2p_task.p, t.d_p2p_slot.p, t.d_p2p_src.p, src64, geo, N,
                         kappa, 0.0, part);
  } else {
    if (nf == 3)
      hipLaunchKernelGGL((k_p2p_tasks<float, 3>), dim3(nbp), dim3(64), 0, s, t.n_p2p_tasks,
                         t.d_p2p_task.p, t.d_p2p_slot.p, t.d_p2p_src.p, src32, tgt32, N,
                         (float)kappa, nk32, part);
    else
      hipLaunchKernelGGL((k_p2p_tasks<float, 1>), dim3(nbp), dim3(64), 0, s, t.n_p2p_tasks,
                         t.d_p2p_task.p, t.d_p2p_slot.p, t.d_p2p_src.p, src32, tgt32, N,
                         (float)kappa, nk32, part);
  }
  PBMP_HIP(hipGetLastError());
  if (clk.on) clk.end(s, e0, KernelClock::P2P, t.direct_pairs);

  if (t.n_m2p_tasks > 0 && !t.m2p_box.empty()) {
    e0 = clk.on ? clk.begin(s) : nullptr;
    if (fp64)
      launch_m2p<double>(t, s, t.d_mom64.p, geo, N, kappa, 0.0, part);
    else
      launch_m2p<float>(t, s, t.d_mom32.p, tgt32, N, (float)kappa, nk32, part);
    PBMP_HIP(hipGetLastError());
    if (clk.on) clk.end(s, e0, KernelClock::M2P, t.m2p_pairs);
  }
}

void launch_finish_slots(hipStream_t s, int N, const int *tslots, const double *part,
                         const int *rowptr, const int *col, const double *val,
                         const double *x, double eps_ratio, double *y) {
  hipLaunchKernelGGL(k_finish_slots, dim3((N + 255) / 256), dim3(256), 0, s, N, tslots,
                     part, rowptr, col, val, x, eps_ratio, y);
  PBMP_HIP(hipGetLastError());
}

}  // namespace pbmp
