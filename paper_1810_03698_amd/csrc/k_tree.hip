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

// binomial coefficients C(a, b), a, b <= 6
__constant__ double kBinom[7][7] = {
    {1, 0, 0, 0, 0, 0, 0},   {1, 1, 0, 0, 0, 0, 0},    {1, 2, 1, 0, 0, 0, 0},
    {1, 3, 3, 1, 0, 0, 0},   {1, 4, 6, 4, 1, 0, 0},    {1, 5, 10, 10, 5, 1, 0},
    {1, 6, 15, 20, 15, 6, 1}};

inline int ncoef_of(int P) { return (P + 1) * (P + 2) * (P + 3) / 6; }

// blockIdx -> task: consecutive tasks (neighbouring target leaves, similar
// source lists) land on the same XCD so they share its L2.
__device__ inline int xcd_task(int ntasks) {
  const int per = (gridDim.x + 7) / 8;
  const int t = (blockIdx.x % 8) * per + blockIdx.x / 8;
  return t < ntasks ? t : -1;
}

// ---------------------------------------------------------------- P2M
// One 256-lane block per leaf; every lane takes nodes of the leaf, builds
// all monomials h^k incrementally (each from its parent multi-index) and
// accumulates both moment sets in registers; then a wave reduction
// (shuffles) and an LDS reduction across the four waves.
template <int P>
__global__ __launch_bounds__(256) void k_p2m(int nf, const int *__restrict__ leaves,
                                             const int *__restrict__ range,
                                             const double *__restrict__ center,
                                             const double *__restrict__ src,
                                             double *__restrict__ mom) {
  constexpr Multi<P> mi{};
  constexpr int NC = Multi<P>::n;
  __shared__ double red[4][2 * NC];
  const int B = leaves[blockIdx.x];
  const int s0 = range[2 * B], s1 = range[2 * B + 1];
  const double c[3] = {center[3 * B], center[3 * B + 1], center[3 * B + 2]};
  double m[NC], mk[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) m[k] = mk[k] = 0.0;
  const int nnode = (s1 - s0) * nf;
  for (int g = threadIdx.x; g < nnode; g += 256) {
    const int j = s0 + g / nf, q = g % nf;
    const double *r = src + 16 * (size_t)j;
    const double h[3] = {r[3 * q] - c[0], r[3 * q + 1] - c[1], r[3 * q + 2] - c[2]};
    const double n[3] = {r[9], r[10], r[11]};
    const double sv = r[13], sk = r[14];
    double mono[NC];
    mono[0] = 1.0;
#pragma unroll
    for (int k = 1; k < NC; ++k) {
      const int d = mi.e[k][0] ? 0 : (mi.e[k][1] ? 1 : 2);
      mono[k] = mono[mi.m1[k][d]] * h[d];
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      m[k] += sv * mono[k];
      double dk = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d)
        if (mi.m1[k][d] >= 0) dk += mi.e[k][d] * n[d] * mono[mi.m1[k][d]];
      mk[k] += sk * dk;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    double a = m[k], b = mk[k];
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_down(a, off, 64);
      b += __shfl_down(b, off, 64);
    }
    if (lane == 0) {
      red[wave][k] = a;
      red[wave][NC + k] = b;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < 2 * NC; k += 256)
    mom[(size_t)B * 2 * NC + k] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
}

// ---------------------------------------------------------------- M2M
// (h + t)^k = sum_{j <= k} C(k, j) t^{k-j} h^j, t = child centre - parent
// centre; one block per box of a level (leaves return at once), one lane
// per coefficient.  The
// children's moments are staged in LDS first (one coalesced read), so the
// shift itself runs at LDS latency.
template <int P>
__global__ __launch_bounds__(64) void k_m2m(int base, const int *__restrict__ child,
                                            const double *__restrict__ center,
                                            double *__restrict__ mom) {
  constexpr Multi<P> mi{};
  constexpr int NC = Multi<P>::n;
  __shared__ double tp[8][3][P + 1];
  __shared__ double cm[8][2 * NC];
  __shared__ int cid[8];
  const int B = base + (int)blockIdx.x;
  if (threadIdx.x < 8) cid[threadIdx.x] = child[8 * B + threadIdx.x];
  __syncthreads();
  int nch = 0;
  for (int cc = 0; cc < 8; ++cc) nch += cid[cc] >= 0;
  if (nch == 0) return;  // a leaf: its moments come from P2M (uniform per block)
  if (threadIdx.x < 3 * nch) {
    const int cc = threadIdx.x / 3, d = threadIdx.x % 3;
    const double t = center[3 * cid[cc] + d] - center[3 * B + d];
    double p = 1.0;
    for (int e = 0; e <= P; ++e) {
      tp[cc][d][e] = p;
      p *= t;
    }
  }
  for (int e = threadIdx.x; e < nch * 2 * NC; e += 64) {
    const int cc = e / (2 * NC), k = e % (2 * NC);
    cm[cc][k] = mom[(size_t)cid[cc] * 2 * NC + k];
  }
  __syncthreads();
  for (int k = threadIdx.x; k < NC; k += 64) {
    const int kx = mi.e[k][0], ky = mi.e[k][1], kz = mi.e[k][2];
    double m = 0.0, mkk = 0.0;
    for (int cc = 0; cc < nch; ++cc) {
      for (int jx = 0; jx <= kx; ++jx) {
        const double wx = kBinom[kx][jx] * tp[cc][0][kx - jx];
        for (int jy = 0; jy <= ky; ++jy) {
          const double wxy = wx * kBinom[ky][jy] * tp[cc][1][ky - jy];
          for (int jz = 0; jz <= kz; ++jz) {
            const int jd = Multi<P>::index(jx, jy, jz);
            const double w = wxy * kBinom[kz][jz] * tp[cc][2][kz - jz];
            m += w * cm[cc][jd];
            mkk += w * cm[cc][NC + jd];
          }
        }
      }
    }
    mom[(size_t)B * 2 * NC + k] = m;
    mom[(size_t)B * 2 * NC + NC + k] = mkk;
  }
}

__global__ void k_cast(size_t n, const double *__restrict__ a, float *__restrict__ b) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// ------------------------------------------------------------ P2P tasks
// One 64-lane block per task: targets [t0, t1) of a leaf, sources = the
// task's panel sub-ranges, streamed through LDS.  Leaves are often much
// smaller than a wave, so the lanes are split into G groups of L = 64 / G:
// every group holds all targets (TPT per lane) and takes every G-th source
// panel of a tile; the groups' FP64 sums are added in LDS in a fixed order.
// G and TPT are chosen per task to use the most lanes.  The LDS tile is
// small and the groups' sums meet through lane shuffles, so a task holds
// 2 KB of LDS and many waves fit on a CU.
constexpr int kTileT = 32;
constexpr int kMaxTPT = 3;

struct LaneSplit {
  int G, L, tpt;
};

// G, L = 64 / G and targets per lane for nt targets: maximise the useful
// fraction G nt / (64 tpt) with tpt <= kMaxTPT (ties: fewer groups; a
// leaf of more than 64 kMaxTPT targets takes several passes with G = 1)
__device__ inline LaneSplit lane_split(int nt) {
  LaneSplit best{1, 64, min(kMaxTPT, (nt + 63) / 64)};
  float be = (float)nt / (64.0f * best.tpt * ((nt + 64 * best.tpt - 1) / (64 * best.tpt)));
  for (int G = 2; G <= 16; ++G) {
    const int L = 64 / G;
    const int tpt = (nt + L - 1) / L;
    if (tpt > kMaxTPT) continue;
    const float e = (float)(G * nt) / (64.0f * tpt);
    if (e > be) {
      be = e;
      best = LaneSplit{G, L, tpt};
    }
  }
  return best;
}

template <class T, int NF, int TPT, bool FLOOR>
__device__ void p2p_task_body(const T *__restrict__ src, const T *__restrict__ tgt,
                              int N, int t0, int t1, const int *__restrict__ ranges,
                              int lb, int le, T kappa, T nk, int slot,
                              double *__restrict__ part, T *sh, int G, int L) {
  const int lane = (int)threadIdx.x;
  const int gi = lane / L, li = lane - gi * L;
  const bool active = gi < G;
  for (int tb = t0; tb < t1; tb += L * TPT) {
    T px[TPT], py[TPT], pz[TPT];
    int ti[TPT];
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
      ti[k] = tb + k * L + li;
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
        for (int e = lane; e < nj * 16; e += 64) sh[e] = src[(size_t)jt * 16 + e];
        __syncthreads();
        T a[TPT][4];
#pragma unroll
        for (int k = 0; k < TPT; ++k)
          for (int c = 0; c < 4; ++c) a[k][c] = T(0);
        for (int jj = active ? gi : nj; jj < nj; jj += G) {
          const T *r = sh + 16 * jj;
#pragma unroll
          for (int k = 0; k < TPT; ++k) {
            if constexpr (sizeof(T) == 4) {
              // as the direct FP32 product: single layer per node with the
              // strength, double layer per panel through the shared n.R
              float kl = 0.f, A = 0.f, B = 0.f, d0[3] = {0.f, 0.f, 0.f};
#pragma unroll
              for (int q = 0; q < NF; ++q) {
                const float dx = px[k] - r[3 * q], dy = py[k] - r[3 * q + 1],
                            dz = pz[k] - r[3 * q + 2];
                if (q == 0) {
                  d0[0] = dx;
                  d0[1] = dy;
                  d0[2] = dz;
                }
                float ri, er;
                node_core<FLOOR>(dx, dy, dz, nk, ri, er);
                const float ri2 = ri * ri;
                a[k][0] = fmaf(r[13], ri, a[k][0]);
                a[k][2] = fmaf(r[13], er, a[k][2]);
                kl = fmaf(ri2, ri, kl);
                A = fmaf(er, ri2, A);
                B = fmaf(er, ri, B);
              }
              const float skn = r[14] * normal_dist(r[9], r[10], r[11], d0[0], d0[1], d0[2]);
              a[k][1] = fmaf(skn, kl, a[k][1]);
              a[k][3] = fmaf(skn, fmaf(kappa, B, A), a[k][3]);
            } else {
              T t4[4];
              panel_terms<T>(r, NF, px[k], py[k], pz[k], kappa, nk, t4);
              a[k][0] += r[13] * t4[0];
              a[k][1] += r[14] * t4[1];
              a[k][2] += r[13] * t4[2];
              a[k][3] += r[14] * t4[3];
            }
          }
        }
#pragma unroll
        for (int k = 0; k < TPT; ++k)
          for (int c = 0; c < 4; ++c) S[k][c] += (double)a[k][c];
      }
    }
    if (G > 1) {
      // group 0 adds the other groups' sums (lane li of group g is lane
      // li + g L); every lane takes part in the shuffles
#pragma unroll
      for (int k = 0; k < TPT; ++k)
        for (int c = 0; c < 4; ++c) {
          const double v = S[k][c];
          double acc = v;
          for (int g = 1; g < G; ++g) acc += __shfl(v, li + g * L, 64);
          S[k][c] = acc;
        }
    }
    if (gi == 0)
#pragma unroll
      for (int k = 0; k < TPT; ++k)
        if (ti[k] < t1)
          for (int c = 0; c < 4; ++c) part[((size_t)slot * 4 + c) * N + ti[k]] = S[k][c];
  }
}

template <class T, int NF, bool FLOOR>
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
  const LaneSplit ls = lane_split(t1 - t0);
  switch (ls.tpt) {
#define PBMP_BODY(K)                                                                          \
  p2p_task_body<T, NF, K, FLOOR>(src, tgt, N, t0, t1, ranges, lb, le, kappa, nk, slot, part, \
                                 sh, ls.G, ls.L)
    case 1: PBMP_BODY(1); break;
    case 2: PBMP_BODY(2); break;
    default: PBMP_BODY(3); break;
#undef PBMP_BODY
  }
}

// ------------------------------------------------------------ M2P tasks

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
  __shared__ T smom[kM2PChunkBoxes * 2 * NC];
  __shared__ T scen[kM2PChunkBoxes * 3];
  const int task = xcd_task(ntask);
  if (task < 0) return;
  const int t0 = tasks[4 * task], t1 = tasks[4 * task + 1];
  const int lb = tasks[4 * task + 2], le = tasks[4 * task + 3];
  const int slot = slots[task];
  const int nb = le - lb;
  const int nt = t1 - t0;
  for (int e = threadIdx.x; e < nb * 2 * NC; e += 64) {
    const int b = e / (2 * NC), c = e % (2 * NC);
    smom[e] = mom[(size_t)boxes[lb + b] * 2 * NC + c];
  }
  for (int e = threadIdx.x; e < nb * 3; e += 64) scen[e] = (T)center[3 * boxes[lb + e / 3] + e % 3];
  // lanes in G groups of L = 64 / G: a group takes every G-th box for all
  // targets; G maximises the useful fraction nt nb / (64 ceil(nt/L) ceil(nb/G))
  int G = 1;
  {
    float be = 0.0f;
    for (int g = 1; g <= 16; ++g) {
      const int L = 64 / g;
      const float e = (float)nt * nb / (64.0f * ((nt + L - 1) / L) * ((nb + g - 1) / g));
      if (e > be) {
        be = e;
        G = g;
      }
    }
  }
  const int L = 64 / G;
  const int gi = (int)threadIdx.x / L, li = (int)threadIdx.x - gi * L;
  const bool active = gi < G;
  __syncthreads();
  const int iters = (nt + L - 1) / L;
  for (int it = 0; it < iters; ++it) {
    const int t = t0 + it * L + li;
    const int tl = min(t, t1 - 1);
    const T x = tgt[tl], y = tgt[N + tl], z = tgt[2 * N + tl];
    T acc[4] = {T(0), T(0), T(0), T(0)};
    for (int b = active ? gi : nb; b < nb; b += G) {
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
    double sum[4] = {(double)acc[0], (double)acc[1], (double)acc[2], (double)acc[3]};
    if (G > 1)
      for (int c = 0; c < 4; ++c) {
        const double v = sum[c];
        for (int g = 1; g < G; ++g) sum[c] += __shfl(v, li + g * L, 64);
      }
    if (gi == 0 && t < t1)
      for (int c = 0; c < 4; ++c) part[((size_t)slot * 4 + c) * N + t] = sum[c];
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

template <int P> void launch_moments_p(Tree &t, hipStream_t s, int nf, const double *src64) {
  hipLaunchKernelGGL(k_p2m<P>, dim3(t.nleaf), dim3(256), 0, s, nf, t.d_leaves.p, t.d_range.p,
                     t.d_center.p, src64, t.d_mom64.p);
  // levels bottom-up; the deepest level holds leaves only
  for (int l = t.depth - 1; l >= 0; --l) {
    const int nb = t.level_start[l + 1] - t.level_start[l];
    if (nb > 0)
      hipLaunchKernelGGL(k_m2m<P>, dim3(nb), dim3(64), 0, s, t.level_start[l], t.d_child.p,
                         t.d_center.p, t.d_mom64.p);
  }
}

void launch_moments(Tree &t, hipStream_t s, int nf, const double *src64) {
  switch (t.prm.order) {
    case 1: launch_moments_p<1>(t, s, nf, src64); break;
    case 2: launch_moments_p<2>(t, s, nf, src64); break;
    case 3: launch_moments_p<3>(t, s, nf, src64); break;
    case 4: launch_moments_p<4>(t, s, nf, src64); break;
    case 5: launch_moments_p<5>(t, s, nf, src64); break;
    case 6: launch_moments_p<6>(t, s, nf, src64); break;
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
                double kappa, double *part, KernelClock &clk, bool floor_r2) {
  const int NC = t.ncoef;
  hipEvent_t e0 = clk.on ? clk.begin(s) : nullptr;
  launch_moments(t, s, nf, src64);
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
#define PBMP_TP(TT, NFV, FL, SRC, TGT, KAP, NK)                                          \
  hipLaunchKernelGGL((k_p2p_tasks<TT, NFV, FL>), dim3(nbp), dim3(64), 0, s, t.n_p2p_tasks, \
                     t.d_p2p_task.p, t.d_p2p_slot.p, t.d_p2p_src.p, SRC, TGT, N, KAP, NK,  \
                     part)
  if (fp64) {
    if (nf == 3) PBMP_TP(double, 3, true, src64, geo, kappa, 0.0);
    else PBMP_TP(double, 1, true, src64, geo, kappa, 0.0);
  } else {
    const float kf = (float)kappa;
    if (nf == 3 && floor_r2) PBMP_TP(float, 3, true, src32, tgt32, kf, nk32);
    else if (nf == 3) PBMP_TP(float, 3, false, src32, tgt32, kf, nk32);
    else if (floor_r2) PBMP_TP(float, 1, true, src32, tgt32, kf, nk32);
    else PBMP_TP(float, 1, false, src32, tgt32, kf, nk32);
  }
#undef PBMP_TP
  PBMP_HIP(hipGetLastError());
  if (clk.on) clk.end(s, e0, KernelClock::P2P, t.direct_pairs);

  if (t.n_m2p_tasks > 0 && t.n_m2p_entries > 0) {
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
