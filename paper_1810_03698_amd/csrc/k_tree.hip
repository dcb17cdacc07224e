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
// (the double-layer kernel is n.grad_y G) give V = sum_{|k|<=P} a_k m_k and
// K = sum_{|k|<=P+1} a_k mK_k: the double-layer moment of degree |k| holds
// h^(|k|-1), so its series is carried one degree further and both layers
// are truncated at degree P in h.  Moments are formed in FP64: those of the
// leaves from their nodes, those of the accepted boxes above the leaves
// from the leaf moments by exact binomial shifts.
#include <cmath>

#include <type_traits>

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
  int p1[n][3];  // position of k + e_i (-1 beyond degree P)
  int deg[n];
  static constexpr int index(int i, int j, int l) {
    const int s = i + j + l;
    return s * (s + 1) * (s + 2) / 6 + (s - i) * (s - i + 1) / 2 + (s - i - j);
  }
  constexpr Multi() : e(), m1(), m2(), p1(), deg() {
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
            a[d] += 3;
            p1[k][d] = (s < P) ? index(a[0], a[1], a[2]) : -1;
          }
          ++k;
        }
  }
};

constexpr double kInv4PiT = 0.07957747154594767;

inline int ncoef_of(int P) { return (P + 1) * (P + 2) * (P + 3) / 6; }

// coefficient counts of order P: NV single-layer terms (|k| <= P), NK
// double-layer terms (|k| <= P + 1); a box's moments are [NV | NK]
template <int P> struct Orders {
  static constexpr int NV = Multi<P>::n;
  static constexpr int NK = Multi<P + 1>::n;
  static constexpr int NM = NV + NK;
};

// blockIdx -> task: consecutive tasks (neighbouring target leaves, similar
// source lists) land on the same XCD so they share its L2.
__device__ inline int xcd_task(int ntasks) {
  const int per = (gridDim.x + 7) / 8;
  const int t = (blockIdx.x % 8) * per + blockIdx.x / 8;
  return t < ntasks ? t : -1;
}

// ---------------------------------------------------------------- P2M
// Moments of every leaf straight from its nodes (every box is a contiguous
// panel range): one block (one wave by default) per task, a task being a
// leaf's panels [s0, s1) or a slice of at most mom_chunk_panels(P) of them.
// Every lane takes nodes, builds all monomials h^k incrementally (each from
// its parent multi-index) and accumulates both moment sets in registers; a
// wave reduction (shuffles), and an LDS reduction across waves when a block
// has several, give the task's partial moments, and k_mom_reduce adds a
// leaf's slices in a fixed order.  The accepted boxes above the leaves then
// take their moments from the leaves' by exact shifts (k_shift_tasks): two
// short launches instead of walking every box's nodes, whose long tasks and
// few waves left the direct form latency-bound.
#ifndef PBMP_P2M_THREADS
#define PBMP_P2M_THREADS 64
#endif
constexpr int kP2MThreads = PBMP_P2M_THREADS;
constexpr int kP2MTile = 64;  // panels per LDS tile (64 and 192 nodes: multiples of 64)
static_assert(kP2MThreads % 64 == 0 && kP2MTile % kP2MThreads == 0, "P2M tiling");

// direct: every leaf is one task, so the task's sums are the leaf's moments
// and go straight to mom64 (and mom32 when not null) instead of part
template <int P>
__global__ __launch_bounds__(kP2MThreads) void k_p2m_tasks(int nf, const int *__restrict__ tasks,
                                                   const double *__restrict__ center,
                                                   const double *__restrict__ src,
                                                   double *__restrict__ part, int direct,
                                                   double *__restrict__ mom64,
                                                   float *__restrict__ mom32) {
  constexpr Multi<P> mi{};
  constexpr Multi<P + 1> miK{};
  constexpr int NC = Orders<P>::NV, NK = Orders<P>::NK, NM = Orders<P>::NM;
  constexpr int NW = kP2MThreads / 64;
  __shared__ double red[NW][NM];
  const int B = tasks[3 * blockIdx.x];
  const int s0 = tasks[3 * blockIdx.x + 1], s1 = tasks[3 * blockIdx.x + 2];
  const double c[3] = {center[3 * B], center[3 * B + 1], center[3 * B + 2]};
  double m[NC], mk[NK];
#pragma unroll
  for (int k = 0; k < NC; ++k) m[k] = 0.0;
#pragma unroll
  for (int k = 0; k < NK; ++k) mk[k] = 0.0;
  // the slice's panel records pass through LDS in tiles of kP2MTile
  // (coalesced loads, all issued together); records padded to 17 doubles
  // against bank conflicts.  A tile holds a multiple of 64 nodes, so every
  // lane takes the same nodes in the same order as without staging.
  __shared__ double sh[kP2MTile * 17];
  for (int jt = s0; jt < s1; jt += kP2MTile) {
    const int nj = min(kP2MTile, s1 - jt);
    __syncthreads();
    {
      // 16-byte loads, two in flight per round (a plain copy loop waits for
      // each load before its store)
      constexpr int U = kP2MTile * 8 / kP2MThreads, Bk = 2;
      typedef double d2 __attribute__((ext_vector_type(2)));
      const d2 *s2 = reinterpret_cast<const d2 *>(src + (size_t)jt * 16);
#pragma unroll
      for (int u0 = 0; u0 < U; u0 += Bk) {
        d2 buf[Bk];
#pragma unroll
        for (int u = 0; u < Bk; ++u) {
          const int e = threadIdx.x + (u0 + u) * kP2MThreads;
          if (e < nj * 8) buf[u] = s2[e];
        }
#pragma unroll
        for (int u = 0; u < Bk; ++u) {
          const int e = threadIdx.x + (u0 + u) * kP2MThreads;
          if (e < nj * 8) {
            double *d = sh + 17 * (e >> 3) + 2 * (e & 7);
            d[0] = buf[u].x;
            d[1] = buf[u].y;
          }
        }
      }
    }
    __syncthreads();
    for (int g = threadIdx.x; g < nj * nf; g += kP2MThreads) {
      const int q = g % nf;
      const double *r = sh + 17 * (g / nf);
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
      for (int k = 0; k < NC; ++k) m[k] += sv * mono[k];
      // double layer to degree P + 1 (its monomials h^(k - e_d) have
      // degree <= P; a multi-index has the same position in both tables)
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        double dk = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d)
          if (miK.m1[k][d] >= 0) dk += miK.e[k][d] * n[d] * mono[miK.m1[k][d]];
        mk[k] += sk * dk;
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    double a = k < NC ? m[k] : mk[k - NC];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
    if (lane == 0) red[wave][k] = a;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < NM; k += kP2MThreads) {
    double v = red[0][k];
    for (int w = 1; w < NW; ++w) v += red[w][k];
    if (direct) {
      mom64[(size_t)B * NM + k] = v;
      if (mom32) mom32[(size_t)B * NM + k] = (float)v;
    } else {
      part[(size_t)blockIdx.x * NM + k] = v;
    }
  }
}

// mom[B] = sum of the partial moments of B's slices, in slice order
// (mom32: the FP32 copy the mixed-precision M2P reads, or null; boxes with
// fewer than min_tasks tasks are skipped: not this pass's, or written by
// their single task)
__global__ void k_mom_reduce(int nbox, int ncoef2, const int *__restrict__ first,
                             const int *__restrict__ count, const double *__restrict__ part,
                             double *__restrict__ mom, float *__restrict__ mom32,
                             int min_tasks) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nbox * ncoef2) return;
  const int B = e / ncoef2, k = e % ncoef2;
  const int t0 = first[B], nt = count[B];
  if (nt == 0 || nt < min_tasks) return;
  double v = 0.0;
  for (int t = t0; t < t0 + nt; ++t) v += part[(size_t)t * ncoef2 + k];
  mom[e] = v;
  if (mom32) mom32[e] = (float)v;
}

// Moments of the accepted boxes with children from the leaf moments: with
// d = c_L - c_B, (h + d)^k = sum_{j <= k} C(k, j) d^(k-j) h^j, and the
// double-layer moments (n . grad_h) h^k shift with the same coefficients,
// so m_k(B) = sum over the leaves L under B of sum_{j <= k} C(k, j)
// d^(k-j) m_j(L), for both moment sets.  One wave per task (a run of at
// most kShiftLeaves of a box's leaves): the moments of all the run's
// leaves and the monomials of their d are staged in LDS with every load
// issued together, then each lane owns coefficients k and walks its terms
// (j, k - j, C(k, j)) from a table, leaf by leaf in order.
constexpr int kShiftThreads = 64;

template <int P>
__global__ __launch_bounds__(kShiftThreads) void k_shift_tasks(
    const int *__restrict__ tasks, const int *__restrict__ leaves,
    const double *__restrict__ center, const int *__restrict__ monos,
    const int *__restrict__ toff, const int *__restrict__ tjq,
    const double *__restrict__ tc, double *__restrict__ mom, float *__restrict__ mom32,
    const int *__restrict__ count, double *__restrict__ part) {
  // single-layer moments k < NC, double-layer k < NK (the terms of a
  // coefficient reach only coefficients of lower or equal degree, so one
  // table of degree P + 1 serves both)
  constexpr int NC = Orders<P>::NV, NK = Orders<P>::NK, NM = Orders<P>::NM;
  constexpr int R = (NK + kShiftThreads - 1) / kShiftThreads;
  __shared__ double sm[kShiftLeaves * NM], sd[kShiftLeaves * NK];
  __shared__ int sL[kShiftLeaves];
  const int B = tasks[3 * blockIdx.x];
  const int la = tasks[3 * blockIdx.x + 1];
  const int nl = tasks[3 * blockIdx.x + 2] - la;
  const double cB[3] = {center[3 * B], center[3 * B + 1], center[3 * B + 2]};
  __shared__ double sdl[kShiftLeaves * 3];
  if (threadIdx.x < nl) {
    const int L = leaves[la + threadIdx.x];
    sL[threadIdx.x] = L;
    for (int c = 0; c < 3; ++c) sdl[3 * threadIdx.x + c] = center[3 * L + c] - cB[c];
  }
  __syncthreads();
  // moments with eight loads in flight per lane
  for (int e0 = threadIdx.x; e0 < nl * NM; e0 += 8 * kShiftThreads) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * kShiftThreads;
      if (e < nl * NM) v[u] = mom[(size_t)sL[e / NM] * NM + e % NM];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * kShiftThreads;
      if (e < nl * NM) sm[e] = v[u];
    }
  }
  for (int e = threadIdx.x; e < nl * NK; e += kShiftThreads) {
    const int l = e / NK, k = e % NK;
    double v = 1.0;
    for (int c = 0; c < 3; ++c)
      for (int u = 0; u < monos[3 * k + c]; ++u) v *= sdl[3 * l + c];
    sd[e] = v;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int k = threadIdx.x + r * kShiftThreads;
    if (k >= NK) continue;
    const bool hasV = k < NC;
    const int t0 = toff[k], t1 = toff[k + 1];
    // terms outer (one table read each), leaves inner; per-leaf sums in
    // registers are added in leaf order at the end
    double v[kShiftLeaves], w[kShiftLeaves];
#pragma unroll
    for (int l = 0; l < kShiftLeaves; ++l) v[l] = w[l] = 0.0;
    for (int t = t0; t < t1; ++t) {
      const int j = tjq[2 * t], q = tjq[2 * t + 1];
      const double ct = tc[t];
#pragma unroll
      for (int l = 0; l < kShiftLeaves; ++l) {
        if (l < nl) {
          const double c = ct * sd[l * NK + q];
          if (hasV) v[l] += c * sm[l * NM + j];
          w[l] += c * sm[l * NM + NC + j];
        }
      }
    }
    double aV = 0.0, aK = 0.0;
#pragma unroll
    for (int l = 0; l < kShiftLeaves; ++l) {
      if (l < nl) {
        aV += v[l];
        aK += w[l];
      }
    }
    if (count[B] == 1) {  // the box's only task: its moments
      if (hasV) mom[(size_t)B * NM + k] = aV;
      mom[(size_t)B * NM + NC + k] = aK;
      if (mom32) {
        if (hasV) mom32[(size_t)B * NM + k] = (float)aV;
        mom32[(size_t)B * NM + NC + k] = (float)aK;
      }
    } else {
      if (hasV) part[(size_t)blockIdx.x * NM + k] = aV;
      part[(size_t)blockIdx.x * NM + NC + k] = aK;
    }
  }
}


// ------------------------------------------------------------ P2P tasks
// One 64-lane block per task: targets [t0, t1) of a leaf, sources = the
// task's panel sub-ranges, streamed through LDS.  Leaves are often much
// smaller than a wave, so the lanes are split into G groups of L = 64 / G:
// every group holds all targets (TPT per lane) and takes every G-th source
// panel of a tile; group 0 adds the other groups' FP64 sums through lane
// shuffles in a fixed order.  G and TPT are chosen per task to use the most
// lanes.  Tile, TPT bound and the use of groups are compile-time settings
// (the defaults were the fastest measured; M2P runs without groups).
constexpr int kTileT = PBMP_P2P_TILE;
constexpr int kMaxTPT = PBMP_P2P_MAXTPT;

// Copies nj (<= MAXREC) records of 16 T from global memory to LDS in
// 16-byte accesses, every load of the lane issued before the first store
// (a plain copy loop waits for each load before its store).
template <class T, int MAXREC>
__device__ __forceinline__ void stage_records(const T *__restrict__ src, T *sh, int nj,
                                              int lane) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  typedef double d2 __attribute__((ext_vector_type(2)));
  using V = typename std::conditional<sizeof(T) == 4, f4, d2>::type;
  constexpr int PER = 16 * (int)sizeof(T) / 16;  // 16-byte units per record
  constexpr int U = (MAXREC * PER + 63) / 64;
  const V *s = reinterpret_cast<const V *>(src);
  V *d = reinterpret_cast<V *>(sh);
  constexpr int B = 2;  // loads in flight per round (registers of the caller stay free)
  const int n = nj * PER;
#pragma unroll
  for (int u0 = 0; u0 < U; u0 += B) {
    V buf[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int e = lane + 64 * (u0 + u);
      if (u0 + u < U && e < n) buf[u] = s[e];
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int e = lane + 64 * (u0 + u);
      if (u0 + u < U && e < n) d[e] = buf[u];
    }
  }
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
        stage_records<T, kTileT>(src + (size_t)jt * 16, sh, nj, lane);
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
#if PBMP_P2P_MAXTPT >= 4
    case 3: PBMP_BODY(3); break;
    case 4: PBMP_BODY(4); break;
    default: PBMP_BODY(kMaxTPT); break;
#else
    default: PBMP_BODY(3); break;
#endif
#undef PBMP_BODY
  }
}

// ------------------------------------------------------------ M2P tasks

template <class T> __device__ inline T rsqrt_t(T x);
template <> __device__ inline float rsqrt_t<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ inline double rsqrt_t<double>(double x) { return rsqrt_fp64(x); }
template <class T> __device__ inline T expneg_t(T nk, T kappa, T r);
template <> __device__ inline float expneg_t<float>(float nk, float, float r) {
  return __builtin_amdgcn_exp2f(nk * r);
}
template <> __device__ inline double expneg_t<double>(double, double kappa, double r) {
  return exp_fp64(-kappa * r);
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
  constexpr Multi<P + 1> mi{};
  constexpr int NC = Orders<P>::NV, NK = Orders<P>::NK, NM = Orders<P>::NM;
  __shared__ T smom[kM2PChunkBoxes * NM];
  __shared__ T scen[kM2PChunkBoxes * 3];
  const int task = xcd_task(ntask);
  if (task < 0) return;
  const int t0 = tasks[4 * task], t1 = tasks[4 * task + 1];
  const int lb = tasks[4 * task + 2], le = tasks[4 * task + 3];
  const int slot = slots[task];
  const int nb = le - lb;
  const int nt = t1 - t0;
  // box ids first, then the moments with eight loads in flight per lane
  __shared__ int sbox[kM2PChunkBoxes];
  if (threadIdx.x < nb) sbox[threadIdx.x] = boxes[lb + threadIdx.x];
  __syncthreads();
  for (int e0 = threadIdx.x; e0 < nb * NM; e0 += 8 * 64) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + 64 * u;
      if (e < nb * NM) v[u] = mom[(size_t)sbox[e / NM] * NM + e % NM];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + 64 * u;
      if (e < nb * NM) smom[e] = v[u];
    }
  }
  for (int e = threadIdx.x; e < nb * 3; e += 64) scen[e] = (T)center[3 * sbox[e / 3] + e % 3];
  // optionally lanes in G groups of L = 64 / G (PBMP_M2P_GROUPS): a group
  // takes every G-th box for all targets, G maximising the useful fraction
  // nt nb / (64 ceil(nt/L) ceil(nb/G)); off by default (measured slower)
  int G = 1;
  {
    float be = 0.0f;
    for (int g = 1; g <= 16 * PBMP_M2P_GROUPS; ++g) {
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
      const T *m = smom + b * NM;
      // coefficients degree by degree, each contracted as soon as it is
      // formed (single layer k < NC, double layer k < NK), so that only the
      // two previous degrees stay live for the recurrence
      T a[NK], ay[NK], by[NK];
      a[0] = ri;
      by[0] = ek;
      ay[0] = ek * ri;
      acc[0] += a[0] * m[0];
      acc[1] += a[0] * m[NC];
      acc[2] += ay[0] * m[0];
      acc[3] += ay[0] * m[NC];
#pragma unroll
      for (int k = 1; k < NK; ++k) {
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
        if (k < NC) {
          acc[0] += a[k] * m[k];
          acc[2] += ay[k] * m[k];
        }
        acc[1] += a[k] * m[NC + k];
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

// y = A x from the far-field slots and the near/self corrections.  Four
// lanes per row (a wave takes 16 rows): lane u of a row sums the row's slots
// u, u + 4, ... and its correction entries u, u + 4, ..., so that the
// four lanes read neighbouring entries together and a launch holds four
// times as many waves to hide the latency of the scattered reads of x;
// the lanes' sums are then added in a fixed order (lane shuffles).
constexpr int kFinLanes = 4;
constexpr int kFinBlock = 256;

__global__ __launch_bounds__(kFinBlock) void k_finish_slots(
    int N, const int *__restrict__ tslots, const double *__restrict__ part,
    const int *__restrict__ rowptr, const int *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ x, double eps_ratio,
    double *__restrict__ y) {
  const int t = blockIdx.x * kFinBlock + (int)threadIdx.x;
  const int i = t / kFinLanes, u = t % kFinLanes;
  const bool live = i < N;
  const int il = live ? i : N - 1;
  double S[4] = {0.0, 0.0, 0.0, 0.0};
  const int ns = tslots[il];
  for (int c = u; c < ns; c += kFinLanes)
#pragma unroll
    for (int k = 0; k < 4; ++k) S[k] += part[((size_t)c * 4 + k) * N + il];
  const int e1 = rowptr[il + 1];
  for (int e = rowptr[il] + u; e < e1; e += kFinLanes) {
    const int j = col[e];
    const double ph = x[j], dp = x[N + j];
    const double *v = val + 4 * (size_t)e;
    S[0] += v[0] * dp;
    S[1] += v[1] * ph;
    S[2] += v[2] * dp;
    S[3] += v[3] * ph;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    S[k] += __shfl_xor(S[k], 1, kFinLanes);
    S[k] += __shfl_xor(S[k], 2, kFinLanes);
  }
  if (!live || u != 0) return;
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

template <int P>
void launch_moments_p(Tree &t, hipStream_t s, int nf, const double *src64, float *mom32) {
  constexpr int NM = Orders<P>::NM;
  if (t.n_mom_tasks == 0) return;
  const int direct = t.n_mom_tasks == t.nleaf;  // no leaf split into slices
  hipLaunchKernelGGL(k_p2m_tasks<P>, dim3(t.n_mom_tasks), dim3(kP2MThreads), 0, s, nf,
                     t.d_mom_task.p, t.d_center.p, src64, t.d_mom_part.p, direct, t.d_mom64.p,
                     mom32);
  const int n = t.nbox * NM;
  if (!direct)
    hipLaunchKernelGGL(k_mom_reduce, dim3((n + 255) / 256), dim3(256), 0, s, t.nbox, NM,
                       t.d_mom_first.p, t.d_mom_count.p, t.d_mom_part.p, t.d_mom64.p, mom32, 1);
  if (t.n_shift_tasks > 0) {
    hipLaunchKernelGGL(k_shift_tasks<P>, dim3(t.n_shift_tasks), dim3(kShiftThreads), 0, s,
                       t.d_shift_task.p, t.d_leaves.p, t.d_center.p, t.d_monos.p,
                       t.d_shift_toff.p, t.d_shift_tjq.p, t.d_shift_tc.p, t.d_mom64.p, mom32,
                       t.d_shift_count.p, t.d_shift_part.p);
    if (t.shift_multi)
      hipLaunchKernelGGL(k_mom_reduce, dim3((n + 255) / 256), dim3(256), 0, s, t.nbox, NM,
                         t.d_shift_first.p, t.d_shift_count.p, t.d_shift_part.p, t.d_mom64.p,
                         mom32, 2);
  }
}

// moments in FP64, and their FP32 copy when mom32 is not null
void launch_moments(Tree &t, hipStream_t s, int nf, const double *src64, float *mom32) {
  switch (t.prm.order) {
    case 1: launch_moments_p<1>(t, s, nf, src64, mom32); break;
    case 2: launch_moments_p<2>(t, s, nf, src64, mom32); break;
    case 3: launch_moments_p<3>(t, s, nf, src64, mom32); break;
    case 4: launch_moments_p<4>(t, s, nf, src64, mom32); break;
    case 5: launch_moments_p<5>(t, s, nf, src64, mom32); break;
    case 6: launch_moments_p<6>(t, s, nf, src64, mom32); break;
    default: throw Error(PBMP_EARG, "treecode order must be 1..6");
  }
}


// ===================================================== transposed product
// A^T z for the adjoint solve, the exact transpose of the treecode product
// above: P2P^T runs the forward P2P pairs with sources on lanes; M2P^T
// gathers, for every accepted box B, local coefficients
//   L_B,k = sum over the targets i of the leaves that accepted B of z_i a_k(x_i - c_B)
// (Laplace coefficients with the first component of z, Yukawa with the
// second); L2P evaluates at every node y the expansions of all boxes that
// contain it, h = y - c_B,
//   V^T: sum_k L_k h^k,   K^T: n . grad_h sum_k L_k h^k,
// the transpose of forming every box's moments from its nodes.

template <class T, int NF, int SPT>
__device__ void p2pT_body(const T *__restrict__ src, const T *__restrict__ tgt,
                          const double *__restrict__ z, const double *__restrict__ geo, int N,
                          int s0, int s1, const int *__restrict__ ranges, int lb, int le,
                          T kappa, T nk, int slot, double *__restrict__ part, T *sh, int G,
                          int L) {
  const int lane = (int)threadIdx.x;
  const int gi = lane / L, li = lane - gi * L;
  const bool active = gi < G;
  for (int sb = s0; sb < s1; sb += L * SPT) {
    T rec[SPT][16];
    int sj[SPT];
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
      sj[k] = sb + k * L + li;
      const int jl = min(sj[k], s1 - 1);
      for (int c = 0; c < 16; ++c) rec[k][c] = src[16 * (size_t)jl + c];
    }
    double S[SPT][4];
#pragma unroll
    for (int k = 0; k < SPT; ++k)
      for (int c = 0; c < 4; ++c) S[k][c] = 0.0;
    for (int l = lb; l < le; ++l) {
      const int a0 = ranges[2 * l], a1 = ranges[2 * l + 1];
      for (int it = a0; it < a1; it += 64) {
        const int nt = min(64, a1 - it);
        __syncthreads();
        if (lane < nt) {
          const int i = it + lane;
          sh[5 * lane] = tgt[i];
          sh[5 * lane + 1] = tgt[N + i];
          sh[5 * lane + 2] = tgt[2 * N + i];
          sh[5 * lane + 3] = (T)z[i];
          sh[5 * lane + 4] = (T)z[N + i];
        }
        __syncthreads();
        T a[SPT][4];
#pragma unroll
        for (int k = 0; k < SPT; ++k)
          for (int c = 0; c < 4; ++c) a[k][c] = T(0);
        for (int e = active ? gi : nt; e < nt; e += G) {
          const T *r = sh + 5 * e;
#pragma unroll
          for (int k = 0; k < SPT; ++k) {
            T t4[4];
            panel_terms<T>(rec[k], NF, r[0], r[1], r[2], kappa, nk, t4);
            a[k][0] += r[3] * t4[0];
            a[k][1] += r[3] * t4[1];
            a[k][2] += r[4] * t4[2];
            a[k][3] += r[4] * t4[3];
          }
        }
#pragma unroll
        for (int k = 0; k < SPT; ++k)
          for (int c = 0; c < 4; ++c) S[k][c] += (double)a[k][c];
      }
    }
    if (G > 1) {
#pragma unroll
      for (int k = 0; k < SPT; ++k)
        for (int c = 0; c < 4; ++c) {
          const double v = S[k][c];
          double acc = v;
          for (int g = 1; g < G; ++g) acc += __shfl(v, li + g * L, 64);
          S[k][c] = acc;
        }
    }
    if (gi == 0)
#pragma unroll
      for (int k = 0; k < SPT; ++k)
        if (sj[k] < s1) {
          const double wA = geo[6 * (size_t)N + sj[k]] * kInv4PiT / NF;
          for (int c = 0; c < 4; ++c) part[((size_t)slot * 4 + c) * N + sj[k]] = wA * S[k][c];
        }
  }
}

template <class T, int NF>
__global__ __launch_bounds__(64) void k_p2pT_tasks(int ntask, const int *__restrict__ tasks,
                                                   const int *__restrict__ range,
                                                   const int *__restrict__ subs,
                                                   const T *__restrict__ src,
                                                   const T *__restrict__ tgt,
                                                   const double *__restrict__ z,
                                                   const double *__restrict__ geo, int N,
                                                   T kappa, T nk, double *__restrict__ part) {
  __shared__ T sh[64 * 5];
  const int task = xcd_task(ntask);
  if (task < 0) return;
  const int B = tasks[4 * task], lb = tasks[4 * task + 1], le = tasks[4 * task + 2];
  const int slot = tasks[4 * task + 3];
  const int s0 = range[2 * B], s1 = range[2 * B + 1];
  // split for the sources (at most two panels per lane: records stay in registers)
  const int ns = s1 - s0;
  int G = 1, spt = min(2, (ns + 63) / 64);
  float be = (float)ns / (64.0f * spt * ((ns + 64 * spt - 1) / (64 * spt)));
  for (int g = 2; g <= 16; ++g) {
    const int L = 64 / g, tp = (ns + L - 1) / L;
    if (tp > 2) continue;
    const float e = (float)(g * ns) / (64.0f * tp);
    if (e > be) {
      be = e;
      G = g;
      spt = tp;
    }
  }
  if (spt == 1)
    p2pT_body<T, NF, 1>(src, tgt, z, geo, N, s0, s1, subs, lb, le, kappa, nk, slot, part, sh,
                        G, 64 / G);
  else
    p2pT_body<T, NF, 2>(src, tgt, z, geo, N, s0, s1, subs, lb, le, kappa, nk, slot, part, sh,
                        G, 64 / G);
}

// M2P^T: per task (box B, target sub-ranges) the partial local coefficients
// of one kernel family (YUK: Yukawa with z2, else Laplace with z1)
template <class T, int P, bool YUK>
__global__ __launch_bounds__(64) void k_m2pT_tasks(int ntask, const int *__restrict__ tasks,
                                                   const int *__restrict__ subs,
                                                   const double *__restrict__ center,
                                                   const T *__restrict__ tgt,
                                                   const double *__restrict__ z, int N,
                                                   T kappa, T nk, double *__restrict__ Lpart) {
  // local coefficients to degree P + 1 (the double layer's transpose
  // reaches them; the single layer's uses those of degree <= P)
  constexpr Multi<P + 1> mi{};
  constexpr int NC = Orders<P>::NK;
  const int task = xcd_task(ntask);
  if (task < 0) return;
  const int B = tasks[4 * task], lb = tasks[4 * task + 1], le = tasks[4 * task + 2];
  const T cx = (T)center[3 * B], cy = (T)center[3 * B + 1], cz = (T)center[3 * B + 2];
  T acc[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) acc[k] = T(0);
  for (int l = lb; l < le; ++l) {
    const int a0 = subs[2 * l], a1 = subs[2 * l + 1];
    for (int t = a0 + (int)threadIdx.x; t < a1; t += 64) {
      const T D[3] = {tgt[t] - cx, tgt[N + t] - cy, tgt[2 * N + t] - cz};
      const T R2 = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
      const T ri = rsqrt_t<T>(R2);
      const T iR2 = ri * ri;
      if (!YUK) {
        const T w = (T)z[t];
        T a[NC];
        a[0] = ri;
#pragma unroll
        for (int k = 1; k < NC; ++k) {
          const int s = mi.deg[k];
          T S1 = T(0), S2 = T(0);
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            if (mi.m1[k][d] >= 0) S1 += D[d] * a[mi.m1[k][d]];
            if (mi.m2[k][d] >= 0) S2 += a[mi.m2[k][d]];
          }
          a[k] = (T(2 * s - 1) / T(s) * S1 - T(s - 1) / T(s) * S2) * iR2;
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[k] += w * a[k];
      } else {
        const T w = (T)z[N + t];
        const T ek = expneg_t<T>(nk, kappa, R2 * ri);
        T ay[NC], by[NC];
        by[0] = ek;
        ay[0] = ek * ri;
#pragma unroll
        for (int k = 1; k < NC; ++k) {
          const int s = mi.deg[k];
          T Y1 = T(0), Y2 = T(0), B1 = T(0), B2 = T(0);
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            if (mi.m1[k][d] >= 0) {
              Y1 += D[d] * ay[mi.m1[k][d]];
              B1 += D[d] * by[mi.m1[k][d]];
            }
            if (mi.m2[k][d] >= 0) {
              Y2 += ay[mi.m2[k][d]];
              B2 += by[mi.m2[k][d]];
            }
          }
          const T ks = kappa / T(s);
          by[k] = ks * (Y1 - Y2);
          ay[k] = (T(2 * s - 1) / T(s) * Y1 - T(s - 1) / T(s) * Y2 + ks * (B1 - B2)) * iR2;
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[k] += w * ay[k];
      }
    }
  }
  // wave sums in FP64, lane 0 writes
  double *out = Lpart + (size_t)task * 2 * NC + (YUK ? NC : 0);
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    double v = (double)acc[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (threadIdx.x == 0) out[k] = v;
  }
}

// L_B = sum of the partials of B's tasks (fixed order); zero without tasks
__global__ void k_l_reduce(int nbox, int ncoef2, const int *__restrict__ count,
                           const int *__restrict__ off, const double *__restrict__ Lpart,
                           double *__restrict__ Lb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nbox * ncoef2) return;
  const int B = e / ncoef2, k = e % ncoef2;
  double v = 0.0;
  const int t0 = off[B], nt = count[2 * B + 1];
  for (int t = t0; t < t0 + nt; ++t) v += Lpart[(size_t)t * ncoef2 + k];
  Lb[e] = v;
}

// L2P at the leaves: every node takes the local expansions of all boxes
// on its leaf's path to the root, each about its own centre (the direct
// counterpart of shifting them down level by level), lanes over the leaf's
// panels, FP64.  Boxes that no leaf accepted carry zero coefficients and
// are skipped.
constexpr int kMaxChain = 24;

template <int P, int NF>
__global__ __launch_bounds__(64) void k_l2p(const int *__restrict__ leaves,
                                            const int *__restrict__ range,
                                            const int *__restrict__ parent,
                                            const int *__restrict__ ntask,
                                            const double *__restrict__ center,
                                            const double *__restrict__ Lb,
                                            const double *__restrict__ src64,
                                            const double *__restrict__ geo,
                                            const int *__restrict__ tslotsT, int N,
                                            double *__restrict__ part) {
  constexpr Multi<P> mi{};
  constexpr Multi<P + 1> miK{};
  constexpr int NC = Orders<P>::NV, NK = Orders<P>::NK;
  __shared__ double lp[kMaxChain][2 * NK];
  __shared__ double lc[kMaxChain][3];
  __shared__ int chain[kMaxChain];
  __shared__ int nchain;
  const int B = leaves[blockIdx.x];
  if (threadIdx.x == 0) {
    int n = 0;
    for (int a = B; a >= 0 && n < kMaxChain; a = parent[a])
      if (ntask[2 * a + 1] > 0) chain[n++] = a;
    nchain = n;
  }
  __syncthreads();
  const int nc = nchain;
  for (int e = threadIdx.x; e < nc * 2 * NK; e += 64) {
    const int a = e / (2 * NK), k = e % (2 * NK);
    lp[a][k] = Lb[(size_t)chain[a] * 2 * NK + k];
  }
  for (int e = threadIdx.x; e < nc * 3; e += 64) lc[e / 3][e % 3] = center[3 * chain[e / 3] + e % 3];
  __syncthreads();
  for (int j = range[2 * B] + (int)threadIdx.x; j < range[2 * B + 1]; j += 64) {
    const double *r = src64 + 16 * (size_t)j;
    const double n[3] = {r[9], r[10], r[11]};
    double out[4] = {0.0, 0.0, 0.0, 0.0};
    for (int a = 0; a < nc; ++a) {
      for (int q = 0; q < NF; ++q) {
        const double h[3] = {r[3 * q] - lc[a][0], r[3 * q + 1] - lc[a][1],
                             r[3 * q + 2] - lc[a][2]};
        double mono[NC];
        mono[0] = 1.0;
#pragma unroll
        for (int k = 1; k < NC; ++k) {
          const int d = mi.e[k][0] ? 0 : (mi.e[k][1] ? 1 : 2);
          mono[k] = mono[mi.m1[k][d]] * h[d];
        }
#pragma unroll
        for (int k = 0; k < NK; ++k) {
          double dn = 0.0;
#pragma unroll
          for (int d = 0; d < 3; ++d)
            if (miK.m1[k][d] >= 0) dn += miK.e[k][d] * n[d] * mono[miK.m1[k][d]];
          if (k < NC) {
            out[0] += lp[a][k] * mono[k];
            out[2] += lp[a][NK + k] * mono[k];
          }
          out[1] += lp[a][k] * dn;
          out[3] += lp[a][NK + k] * dn;
        }
      }
    }
    const double wA = geo[6 * (size_t)N + j] * kInv4PiT / NF;
    const int slot = tslotsT[j] - 1;
    for (int k = 0; k < 4; ++k) part[((size_t)slot * 4 + k) * N + j] = wA * out[k];
  }
}

// (A^T z) from the transposed partial slots, the transposed near/self
// correction and the identity terms
__global__ void k_finish_T_slots(int N, const int *__restrict__ tslotsT,
                                 const double *__restrict__ part, const int *__restrict__ trow,
                                 const int *__restrict__ tcol, const int *__restrict__ tent,
                                 const double *__restrict__ val, const double *__restrict__ z,
                                 double eps_ratio, double *__restrict__ y) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double S[4] = {0.0, 0.0, 0.0, 0.0};
  const int ns = tslotsT[j];
  for (int c = 0; c < ns; ++c)
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

template <class T, int P>
void tree_T_far(Tree &t, hipStream_t s, int nf, int N, const double *geo,
                const double *src64, const T *src, const T *tgt, const double *z, T kappa,
                T nk, double *part) {
  constexpr int NK = Orders<P>::NK;
  // P2P^T
  const int nbp = ((t.n_p2pT_tasks + 7) / 8) * 8;
  if (nf == 3)
    hipLaunchKernelGGL((k_p2pT_tasks<T, 3>), dim3(nbp), dim3(64), 0, s, t.n_p2pT_tasks,
                       t.d_p2pT_task.p, t.d_range.p, t.d_p2pT_sub.p, src, tgt, z, geo, N,
                       kappa, nk, part);
  else
    hipLaunchKernelGGL((k_p2pT_tasks<T, 1>), dim3(nbp), dim3(64), 0, s, t.n_p2pT_tasks,
                       t.d_p2pT_task.p, t.d_range.p, t.d_p2pT_sub.p, src, tgt, z, geo, N,
                       kappa, nk, part);
  // M2P^T, per-box sums, L2L down the levels, L2P at the leaves
  t.d_Lpart.reserve((size_t)std::max(1, t.n_m2pT_tasks) * 2 * NK);
  t.d_L.reserve((size_t)t.nbox * 2 * NK);
  if (t.n_m2pT_tasks > 0) {
    const int nbm = ((t.n_m2pT_tasks + 7) / 8) * 8;
    hipLaunchKernelGGL((k_m2pT_tasks<T, P, false>), dim3(nbm), dim3(64), 0, s,
                       t.n_m2pT_tasks, t.d_m2pT_task.p, t.d_m2pT_sub.p, t.d_center.p, tgt, z,
                       N, kappa, nk, t.d_Lpart.p);
    hipLaunchKernelGGL((k_m2pT_tasks<T, P, true>), dim3(nbm), dim3(64), 0, s,
                       t.n_m2pT_tasks, t.d_m2pT_task.p, t.d_m2pT_sub.p, t.d_center.p, tgt, z,
                       N, kappa, nk, t.d_Lpart.p);
  }
  const int nl = t.nbox * 2 * NK;
  hipLaunchKernelGGL(k_l_reduce, dim3((nl + 255) / 256), dim3(256), 0, s, t.nbox, 2 * NK,
                     t.d_m2pT_count.p, t.d_m2pT_off.p, t.d_Lpart.p, t.d_L.p);
  if (nf == 3)
    hipLaunchKernelGGL((k_l2p<P, 3>), dim3(t.nleaf), dim3(64), 0, s, t.d_leaves.p,
                       t.d_range.p, t.d_parent.p, t.d_m2pT_count.p, t.d_center.p, t.d_L.p,
                       src64, geo, t.d_tslotsT.p, N, part);
  else
    hipLaunchKernelGGL((k_l2p<P, 1>), dim3(t.nleaf), dim3(64), 0, s, t.d_leaves.p,
                       t.d_range.p, t.d_parent.p, t.d_m2pT_count.p, t.d_center.p, t.d_L.p,
                       src64, geo, t.d_tslotsT.p, N, part);
  PBMP_HIP(hipGetLastError());
}

template <class T>
void tree_T_far_p(Tree &t, hipStream_t s, int nf, int N, const double *geo,
                  const double *src64, const T *src, const T *tgt, const double *z, T kappa,
                  T nk, double *part) {
  switch (t.prm.order) {
    case 1: tree_T_far<T, 1>(t, s, nf, N, geo, src64, src, tgt, z, kappa, nk, part); break;
    case 2: tree_T_far<T, 2>(t, s, nf, N, geo, src64, src, tgt, z, kappa, nk, part); break;
    case 3: tree_T_far<T, 3>(t, s, nf, N, geo, src64, src, tgt, z, kappa, nk, part); break;
    case 4: tree_T_far<T, 4>(t, s, nf, N, geo, src64, src, tgt, z, kappa, nk, part); break;
    case 5: tree_T_far<T, 5>(t, s, nf, N, geo, src64, src, tgt, z, kappa, nk, part); break;
    case 6: tree_T_far<T, 6>(t, s, nf, N, geo, src64, src, tgt, z, kappa, nk, part); break;
    default: throw Error(PBMP_EARG, "treecode order must be 1..6");
  }
}


// ======================================================= mesh adjoint
// Far-field part of the gradient of lambda . A x with respect to the
// collocation points c_i (target side) and to the far nodes y_g, normals n_j
// and areas A_j (source side), with the same octree, lists and expansions
// as the treecode product, so that the vertex gradient costs what a
// product costs.  Per target i the form is
//   l1_i (S_KL - S_VL) + l2_i (eps S_VY - S_KY)
// (the strengths s_V, s_K of the forward solution packed in the records).
// Exact derivatives of the discrete treecode operator with the expansion
// centres held fixed: direct pairs through op_pair; an accepted box's
// expansion, differentiated in the target, d/dx_i a_k(x - c) =
// -(k_i + 1) a_{k + e_i} (coefficients to degree P + 2); in the sources, the
// local expansions L_k = sum_i lambda_i a_k(x_i - c) of every box on a
// leaf's path (as in the transposed product) differentiated in the node
// h = y - c: the node's share of the form is
//   s_K n.grad_h P_K(h) + s_V P_V(h),
//   P_K = sum_{|k|<=P+1} (L^L_k - L^Y_k) h^k,  P_V = sum_{|k|<=P} (eps L^Y_k - L^L_k) h^k,
// with gradients in h, in n and in the area (the strengths are linear in A).

// target side, direct pairs: per forward P2P task, g_i = d/dc_i of the form
// over the task's source panels; partial slots [slot][4][N] (components 0..2)
template <int NF>
__global__ __launch_bounds__(64) void k_p2p_grad_tasks(int ntask, const int *__restrict__ tasks,
                                                       const int *__restrict__ slots,
                                                       const int *__restrict__ ranges,
                                                       const double *__restrict__ src64,
                                                       const double *__restrict__ geo,
                                                       const double *__restrict__ lam, int N,
                                                       double kappa, double eps_ratio,
                                                       double *__restrict__ part) {
  constexpr int kTileG = 64;
  __shared__ __align__(16) double sh[kTileG * 16];
  const int task = xcd_task(ntask);
  if (task < 0) return;
  const int t0 = tasks[4 * task], t1 = tasks[4 * task + 1];
  const int lb = tasks[4 * task + 2], le = tasks[4 * task + 3];
  const int slot = slots[task];
  const int lane = (int)threadIdx.x;
  for (int tb = t0; tb < t1; tb += 64) {
    const int t = tb + lane, tl = min(t, t1 - 1);
    const double c[3] = {geo[tl], geo[N + tl], geo[2 * N + tl]};
    const double l1 = lam[tl], l2 = eps_ratio * lam[N + tl], l2k = lam[N + tl];
    double g[3] = {0.0, 0.0, 0.0};
    for (int l = lb; l < le; ++l) {
      const int s0 = ranges[2 * l], s1 = ranges[2 * l + 1];
      for (int jt = s0; jt < s1; jt += kTileG) {
        const int nj = min(kTileG, s1 - jt);
        __syncthreads();
        stage_records<double, kTileG>(src64 + (size_t)jt * 16, sh, nj, lane);
        __syncthreads();
        for (int jj = 0; jj < nj; ++jj) {
          const double *r = sh + 16 * jj;
#pragma unroll
          for (int q = 0; q < NF; ++q) {
            const double R[3] = {c[0] - r[3 * q], c[1] - r[3 * q + 1], c[2] - r[3 * q + 2]};
            double gR[3], gn[3];
            op_pair(R, r + 9, kappa, l1 * r[14], l1 * r[13], l2k * r[14], l2 * r[13], gR, gn);
            for (int d = 0; d < 3; ++d) g[d] += gR[d];
          }
        }
      }
    }
    if (t < t1)
      for (int d = 0; d < 3; ++d) part[((size_t)slot * 4 + d) * N + t] = g[d];
  }
}

// target side, expansions: per forward M2P task (FP64 moments),
// d/dx of sum_k a_k m_k = - sum_k (k_d + 1) a_{k + e_d} m_k
template <int P>
__global__ __launch_bounds__(64) void k_m2p_grad_tasks(int ntask, const int *__restrict__ tasks,
                                                       const int *__restrict__ slots,
                                                       const int *__restrict__ boxes,
                                                       const double *__restrict__ center,
                                                       const double *__restrict__ mom,
                                                       const double *__restrict__ geo,
                                                       const double *__restrict__ lam, int N,
                                                       double kappa, double eps_ratio,
                                                       double *__restrict__ part) {
  constexpr Multi<P + 2> mi{};
  constexpr int NC = Orders<P>::NV, NK = Orders<P>::NK, NM = Orders<P>::NM;
  constexpr int NG = Multi<P + 2>::n;
  __shared__ double smom[kM2PChunkBoxes * NM];
  __shared__ double scen[kM2PChunkBoxes * 3];
  __shared__ int sbox[kM2PChunkBoxes];
  const int task = xcd_task(ntask);
  if (task < 0) return;
  const int t0 = tasks[4 * task], t1 = tasks[4 * task + 1];
  const int lb = tasks[4 * task + 2], le = tasks[4 * task + 3];
  const int slot = slots[task];
  const int nb = le - lb;
  if (threadIdx.x < nb) sbox[threadIdx.x] = boxes[lb + threadIdx.x];
  __syncthreads();
  for (int e = threadIdx.x; e < nb * NM; e += 64) smom[e] = mom[(size_t)sbox[e / NM] * NM + e % NM];
  for (int e = threadIdx.x; e < nb * 3; e += 64) scen[e] = center[3 * sbox[e / 3] + e % 3];
  __syncthreads();
  for (int tb = t0; tb < t1; tb += 64) {
    const int t = tb + (int)threadIdx.x, tl = min(t, t1 - 1);
    const double x[3] = {geo[tl], geo[N + tl], geo[2 * N + tl]};
    const double l1 = lam[tl], l2 = lam[N + tl];
    double g[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < nb; ++b) {
      const double D[3] = {x[0] - scen[3 * b], x[1] - scen[3 * b + 1], x[2] - scen[3 * b + 2]};
      const double R2 = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
      const double ri = rsqrt_fp64(R2), iR2 = ri * ri;
      const double ek = exp_fp64(-kappa * R2 * ri);
      double a[NG], ay[NG], by[NG];
      a[0] = ri;
      by[0] = ek;
      ay[0] = ek * ri;
#pragma unroll
      for (int k = 1; k < NG; ++k) {
        const int sd = mi.deg[k];
        double S1 = 0, S2 = 0, Y1 = 0, Y2 = 0, B1 = 0, B2 = 0;
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
        const double c1 = double(2 * sd - 1) / sd, c2 = double(sd - 1) / sd, ks = kappa / sd;
        a[k] = (c1 * S1 - c2 * S2) * iR2;
        by[k] = ks * (Y1 - Y2);
        ay[k] = (c1 * Y1 - c2 * Y2 + ks * (B1 - B2)) * iR2;
      }
      const double *m = smom + b * NM;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double vl = 0, kl = 0, vy = 0, ky = 0;
#pragma unroll
        for (int k = 0; k < NK; ++k) {
          const int kp = mi.p1[k][d];
          const double w = -double(mi.e[k][d] + 1);
          if (k < NC) {
            vl += w * a[kp] * m[k];
            vy += w * ay[kp] * m[k];
          }
          kl += w * a[kp] * m[NC + k];
          ky += w * ay[kp] * m[NC + k];
        }
        g[d] += l1 * (kl - vl) + l2 * (eps_ratio * vy - ky);
      }
    }
    if (t < t1)
      for (int d = 0; d < 3; ++d) part[((size_t)slot * 4 + d) * N + t] = g[d];
  }
}

// gc_i = sum of the target's forward slots
__global__ void k_grad_slots_reduce(int N, int ncomp, int stride, const int *__restrict__ nslots,
                                    int extra, const double *__restrict__ part,
                                    double *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int ns = nslots[i] + extra;
  for (int c = 0; c < ncomp; ++c) {
    double v = 0.0;
    for (int sl = 0; sl < ns; ++sl) v += part[((size_t)sl * stride + c) * N + i];
    out[(size_t)ncomp * i + c] = v;
  }
}

// gy (3 per node), gn, gA of a panel = sum of its transposed slots
__global__ void k_grad_src_reduce(int N, const int *__restrict__ nslots,
                                  const double *__restrict__ part, double *__restrict__ gy,
                                  double *__restrict__ gn, double *__restrict__ gA) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const int ns = nslots[j];
  double v[13];
  for (int c = 0; c < 13; ++c) v[c] = 0.0;
  for (int sl = 0; sl < ns; ++sl)
    for (int c = 0; c < 13; ++c) v[c] += part[((size_t)sl * 13 + c) * N + j];
  for (int c = 0; c < 9; ++c) gy[9 * (size_t)j + c] = v[c];
  for (int c = 0; c < 3; ++c) gn[3 * (size_t)j + c] = v[9 + c];
  gA[j] = v[12];
}

// source side, direct pairs: per P2P^T task (sources of one leaf on the
// lanes, the task's targets through LDS), per source panel the 13 values
// d/dy_q (3 per node), d/dn (3), d/dA (1); slots [slot][13][N]
constexpr int kGradT = 13;

template <int NF>
__global__ __launch_bounds__(64) void k_p2pT_grad_tasks(int ntask, const int *__restrict__ tasks,
                                                        const int *__restrict__ range,
                                                        const int *__restrict__ subs,
                                                        const double *__restrict__ src64,
                                                        const double *__restrict__ geo,
                                                        const double *__restrict__ lam, int N,
                                                        double kappa, double eps_ratio,
                                                        double *__restrict__ part) {
  __shared__ double sh[64 * 5];
  const int task = xcd_task(ntask);
  if (task < 0) return;
  const int B = tasks[4 * task], lb = tasks[4 * task + 1], le = tasks[4 * task + 2];
  const int slot = tasks[4 * task + 3];
  const int s0 = range[2 * B], s1 = range[2 * B + 1];
  const int lane = (int)threadIdx.x;
  for (int sb = s0; sb < s1; sb += 64) {
    const int j = sb + lane, jl = min(j, s1 - 1);
    double rec[15];
    for (int c = 0; c < 15; ++c) rec[c] = src64[16 * (size_t)jl + c];
    double acc[kGradT];
    for (int c = 0; c < kGradT; ++c) acc[c] = 0.0;
    for (int l = lb; l < le; ++l) {
      const int a0 = subs[2 * l], a1 = subs[2 * l + 1];
      for (int it = a0; it < a1; it += 64) {
        const int nt = min(64, a1 - it);
        __syncthreads();
        if (lane < nt) {
          const int i = it + lane;
          sh[5 * lane] = geo[i];
          sh[5 * lane + 1] = geo[N + i];
          sh[5 * lane + 2] = geo[2 * N + i];
          sh[5 * lane + 3] = lam[i];
          sh[5 * lane + 4] = lam[N + i];
        }
        __syncthreads();
        for (int e = 0; e < nt; ++e) {
          const double *r = sh + 5 * e;
#pragma unroll
          for (int q = 0; q < NF; ++q) {
            const double R[3] = {r[0] - rec[3 * q], r[1] - rec[3 * q + 1], r[2] - rec[3 * q + 2]};
            double gR[3], gn[3];
            const double f = op_pair(R, rec + 9, kappa, r[3] * rec[14], r[3] * rec[13],
                                     r[4] * rec[14], eps_ratio * r[4] * rec[13], gR, gn);
            for (int d = 0; d < 3; ++d) {
              acc[3 * q + d] -= gR[d];
              acc[9 + d] += gn[d];
            }
            acc[12] += f;
          }
        }
      }
    }
    if (j < s1) {
      const double iA = 1.0 / geo[6 * (size_t)N + j];
      acc[12] *= iA;
      for (int c = 0; c < kGradT; ++c) part[((size_t)slot * kGradT + c) * N + j] = acc[c];
    }
  }
}

// source side, expansions: at every node the local expansions of the
// boxes on its leaf's path to the root (FP64 L from the M2P^T kernels with
// z = lambda); slot tslotsT[j] - 1
template <int P, int NF>
__global__ __launch_bounds__(64) void k_l2p_grad(const int *__restrict__ leaves,
                                                 const int *__restrict__ range,
                                                 const int *__restrict__ parent,
                                                 const int *__restrict__ ntask,
                                                 const double *__restrict__ center,
                                                 const double *__restrict__ Lb,
                                                 const double *__restrict__ src64,
                                                 const double *__restrict__ geo,
                                                 const int *__restrict__ tslotsT, int N,
                                                 double eps_ratio, double *__restrict__ part) {
  constexpr Multi<P> mi{};
  constexpr Multi<P + 1> miK{};
  constexpr int NC = Orders<P>::NV, NK = Orders<P>::NK;
  __shared__ double lp[kMaxChain][2 * NK];
  __shared__ double lc[kMaxChain][3];
  __shared__ int chain[kMaxChain];
  __shared__ int nchain;
  const int B = leaves[blockIdx.x];
  if (threadIdx.x == 0) {
    int n = 0;
    for (int a = B; a >= 0 && n < kMaxChain; a = parent[a])
      if (ntask[2 * a + 1] > 0) chain[n++] = a;
    nchain = n;
  }
  __syncthreads();
  const int nc = nchain;
  for (int e = threadIdx.x; e < nc * 2 * NK; e += 64) {
    const int a = e / (2 * NK), k = e % (2 * NK);
    lp[a][k] = Lb[(size_t)chain[a] * 2 * NK + k];
  }
  for (int e = threadIdx.x; e < nc * 3; e += 64) lc[e / 3][e % 3] = center[3 * chain[e / 3] + e % 3];
  __syncthreads();
  for (int j = range[2 * B] + (int)threadIdx.x; j < range[2 * B + 1]; j += 64) {
    const double *r = src64 + 16 * (size_t)j;
    const double n[3] = {r[9], r[10], r[11]};
    const double sv = r[13], sk = r[14];
    double acc[kGradT];
    for (int c = 0; c < kGradT; ++c) acc[c] = 0.0;
    for (int a = 0; a < nc; ++a) {
      for (int q = 0; q < NF; ++q) {
        const double h[3] = {r[3 * q] - lc[a][0], r[3 * q + 1] - lc[a][1], r[3 * q + 2] - lc[a][2]};
        double mono[NC];
        mono[0] = 1.0;
#pragma unroll
        for (int k = 1; k < NC; ++k) {
          const int d = mi.e[k][0] ? 0 : (mi.e[k][1] ? 1 : 2);
          mono[k] = mono[mi.m1[k][d]] * h[d];
        }
        double pv = 0.0, gv[3] = {0, 0, 0}, gk[3] = {0, 0, 0};
        double hk[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
        for (int k = 0; k < NK; ++k) {
          const double cK = lp[a][k] - lp[a][NK + k];
          if (k < NC) {
            const double cV = eps_ratio * lp[a][NK + k] - lp[a][k];
            pv += cV * mono[k];
#pragma unroll
            for (int d = 0; d < 3; ++d)
              if (mi.m1[k][d] >= 0) gv[d] += cV * mi.e[k][d] * mono[mi.m1[k][d]];
          }
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const int k1 = miK.m1[k][d];
            if (k1 < 0) continue;
            gk[d] += cK * miK.e[k][d] * mono[k1];
#pragma unroll
            for (int e = 0; e < 3; ++e) {
              const int k2 = miK.m1[k1][e];
              if (k2 < 0) continue;
              hk[d][e] += cK * miK.e[k][d] * miK.e[k1][e] * mono[k2];
            }
          }
        }
        const double qk = n[0] * gk[0] + n[1] * gk[1] + n[2] * gk[2];
        for (int e = 0; e < 3; ++e) {
          const double hn = n[0] * hk[0][e] + n[1] * hk[1][e] + n[2] * hk[2][e];
          acc[3 * q + e] += sk * hn + sv * gv[e];
          acc[9 + e] += sk * gk[e];
        }
        acc[12] += sk * qk + sv * pv;
      }
    }
    const double iA = 1.0 / geo[6 * (size_t)N + j];
    acc[12] *= iA;
    const int slot = tslotsT[j] - 1;
    for (int c = 0; c < kGradT; ++c) part[((size_t)slot * kGradT + c) * N + j] = acc[c];
  }
}

template <int P>
void tree_mesh_adjoint_far_p(Tree &t, hipStream_t s, int nf, int N, const double *geo,
                             const double *src64, const double *lam, double kappa,
                             double eps_ratio, double *part, double *partT, double *gc,
                             double *gy, double *gn, double *gA) {
  constexpr int NK = Orders<P>::NK;
  // target side: direct pairs and expansions into the forward slots
  const int nbp = ((t.n_p2p_tasks + 7) / 8) * 8;
  if (nf == 3)
    hipLaunchKernelGGL(k_p2p_grad_tasks<3>, dim3(nbp), dim3(64), 0, s, t.n_p2p_tasks,
                       t.d_p2p_task.p, t.d_p2p_slot.p, t.d_p2p_src.p, src64, geo, lam, N,
                       kappa, eps_ratio, part);
  else
    hipLaunchKernelGGL(k_p2p_grad_tasks<1>, dim3(nbp), dim3(64), 0, s, t.n_p2p_tasks,
                       t.d_p2p_task.p, t.d_p2p_slot.p, t.d_p2p_src.p, src64, geo, lam, N,
                       kappa, eps_ratio, part);
  if (t.n_m2p_tasks > 0 && t.n_m2p_entries > 0) {
    const int nbm = ((t.n_m2p_tasks + 7) / 8) * 8;
    hipLaunchKernelGGL((k_m2p_grad_tasks<P>), dim3(nbm), dim3(64), 0, s, t.n_m2p_tasks,
                       t.d_m2p_task.p, t.d_m2p_slot.p, t.d_m2p_box.p, t.d_center.p,
                       t.d_mom64.p, geo, lam, N, kappa, eps_ratio, part);
  }
  hipLaunchKernelGGL(k_grad_slots_reduce, dim3((N + 255) / 256), dim3(256), 0, s, N, 3, 4,
                     t.d_tslots.p, 0, part, gc);
  // source side: transposed direct pairs, local expansions at the nodes
  const int nbt = ((t.n_p2pT_tasks + 7) / 8) * 8;
  if (nf == 3)
    hipLaunchKernelGGL(k_p2pT_grad_tasks<3>, dim3(nbt), dim3(64), 0, s, t.n_p2pT_tasks,
                       t.d_p2pT_task.p, t.d_range.p, t.d_p2pT_sub.p, src64, geo, lam, N,
                       kappa, eps_ratio, partT);
  else
    hipLaunchKernelGGL(k_p2pT_grad_tasks<1>, dim3(nbt), dim3(64), 0, s, t.n_p2pT_tasks,
                       t.d_p2pT_task.p, t.d_range.p, t.d_p2pT_sub.p, src64, geo, lam, N,
                       kappa, eps_ratio, partT);
  t.d_Lpart.reserve((size_t)std::max(1, t.n_m2pT_tasks) * 2 * NK);
  t.d_L.reserve((size_t)t.nbox * 2 * NK);
  if (t.n_m2pT_tasks > 0) {
    const int nbm = ((t.n_m2pT_tasks + 7) / 8) * 8;
    hipLaunchKernelGGL((k_m2pT_tasks<double, P, false>), dim3(nbm), dim3(64), 0, s,
                       t.n_m2pT_tasks, t.d_m2pT_task.p, t.d_m2pT_sub.p, t.d_center.p, geo, lam,
                       N, kappa, 0.0, t.d_Lpart.p);
    hipLaunchKernelGGL((k_m2pT_tasks<double, P, true>), dim3(nbm), dim3(64), 0, s,
                       t.n_m2pT_tasks, t.d_m2pT_task.p, t.d_m2pT_sub.p, t.d_center.p, geo, lam,
                       N, kappa, 0.0, t.d_Lpart.p);
  }
  const int nl = t.nbox * 2 * NK;
  hipLaunchKernelGGL(k_l_reduce, dim3((nl + 255) / 256), dim3(256), 0, s, t.nbox, 2 * NK,
                     t.d_m2pT_count.p, t.d_m2pT_off.p, t.d_Lpart.p, t.d_L.p);
  if (nf == 3)
    hipLaunchKernelGGL((k_l2p_grad<P, 3>), dim3(t.nleaf), dim3(64), 0, s, t.d_leaves.p,
                       t.d_range.p, t.d_parent.p, t.d_m2pT_count.p, t.d_center.p, t.d_L.p,
                       src64, geo, t.d_tslotsT.p, N, eps_ratio, partT);
  else
    hipLaunchKernelGGL((k_l2p_grad<P, 1>), dim3(t.nleaf), dim3(64), 0, s, t.d_leaves.p,
                       t.d_range.p, t.d_parent.p, t.d_m2pT_count.p, t.d_center.p, t.d_L.p,
                       src64, geo, t.d_tslotsT.p, N, eps_ratio, partT);
  hipLaunchKernelGGL(k_grad_src_reduce, dim3((N + 255) / 256), dim3(256), 0, s, N,
                     t.d_tslotsT.p, partT, gy, gn, gA);
  PBMP_HIP(hipGetLastError());
}

}  // namespace

void tree_upload_exponents(Tree &t, hipStream_t s) {
  std::vector<int> ex;
  for (int d = 0; d <= t.prm.order + 1; ++d)
    for (int i = d; i >= 0; --i)
      for (int j = d - i; j >= 0; --j) ex.insert(ex.end(), {i, j, d - i - j});
  t.d_monos.upload(ex.data(), ex.size(), s);
  // shift terms per coefficient k: (j, k - j, C(k, j)) for every j <= k
  auto index = [](int i, int j, int l) {
    const int d = i + j + l;
    return d * (d + 1) * (d + 2) / 6 + (d - i) * (d - i + 1) / 2 + (d - i - j);
  };
  auto binom = [](int n, int r) {
    double c = 1.0;
    for (int u = 1; u <= r; ++u) c = c * (n - r + u) / u;
    return c;
  };
  const int nc = (int)ex.size() / 3;
  std::vector<int> off(nc + 1, 0), jq;
  std::vector<double> c;
  for (int k = 0; k < nc; ++k) {
    const int kx = ex[3 * k], ky = ex[3 * k + 1], kz = ex[3 * k + 2];
    for (int jx = 0; jx <= kx; ++jx)
      for (int jy = 0; jy <= ky; ++jy)
        for (int jz = 0; jz <= kz; ++jz) {
          jq.push_back(index(jx, jy, jz));
          jq.push_back(index(kx - jx, ky - jy, kz - jz));
          c.push_back(binom(kx, jx) * binom(ky, jy) * binom(kz, jz));
        }
    off[k + 1] = (int)c.size();
  }
  t.d_shift_toff.upload(off.data(), off.size(), s);
  t.d_shift_tjq.upload(jq.data(), jq.size(), s);
  t.d_shift_tc.upload(c.data(), c.size(), s);
}

void tree_apply(Tree &t, hipStream_t s, bool fp64, int nf, int N, const double *geo,
                const double *src64, const float *src32, const float *tgt32,
                double kappa, double *part, KernelClock &clk, bool floor_r2) {
  hipEvent_t e0 = clk.on ? clk.begin(s) : nullptr;
  launch_moments(t, s, nf, src64, fp64 ? nullptr : t.d_mom32.p);
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
  const int rows_per_block = kFinBlock / kFinLanes;
  hipLaunchKernelGGL(k_finish_slots, dim3((N + rows_per_block - 1) / rows_per_block),
                     dim3(kFinBlock), 0, s, N, tslots, part, rowptr, col, val, x, eps_ratio, y);
  PBMP_HIP(hipGetLastError());
}

void tree_mesh_adjoint_far(Tree &t, hipStream_t s, int nf, int N, const double *geo,
                           const double *src64, const double *lam, double kappa,
                           double eps_ratio, double *part, double *partT, double *gc,
                           double *gy, double *gn, double *gA) {
  switch (t.prm.order) {
#define PBMP_MA(P)                                                                          \
  case P:                                                                                   \
    tree_mesh_adjoint_far_p<P>(t, s, nf, N, geo, src64, lam, kappa, eps_ratio, part, partT, \
                               gc, gy, gn, gA);                                             \
    break;
    PBMP_MA(1)
    PBMP_MA(2)
    PBMP_MA(3)
    PBMP_MA(4)
    PBMP_MA(5)
    PBMP_MA(6)
#undef PBMP_MA
    default: throw Error(PBMP_EARG, "treecode order must be 1..6");
  }
}

void tree_apply_transpose(Tree &t, hipStream_t s, bool fp64, int nf, int N, const double *geo,
                          const double *src64, const float *src32, const float *tgt32,
                          const double *z, double kappa, double *part, const int *trow,
                          const int *tcol, const int *tent, const double *val, double eps_ratio,
                          double *y) {
  if (fp64)
    tree_T_far_p<double>(t, s, nf, N, geo, src64, src64, geo, z, kappa, 0.0, part);
  else
    tree_T_far_p<float>(t, s, nf, N, geo, src64, src32, tgt32, z, (float)kappa,
                        (float)(-kappa * 1.4426950408889634), part);
  hipLaunchKernelGGL(k_finish_T_slots, dim3((N + 255) / 256), dim3(256), 0, s, N,
                     t.d_tslotsT.p, part, trow, tcol, tent, val, z, eps_ratio, y);
  PBMP_HIP(hipGetLastError());
}

}  // namespace pbmp
