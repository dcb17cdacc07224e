// On-device construction of the treecode's octree and interaction lists
// (section "The treecode algorithm").
//
//  1. Panels are ordered by the Morton key of their centroid on a 2^21 grid
//     over the bounding cube (radix sort of the 63-bit keys, stable, so ties
//     keep the caller's order); every octree cell is then a contiguous range.
//  2. The octree is built level by level: in every box of the current level
//     that holds more than `leaf` panels, a child starts wherever the next
//     three key bits (the octant one level down) change.  A scan of those
//     flags numbers the children, so box ids run level by level and, within
//     a level, in key order; the target leaves are listed in key order.
//  3. Box geometry: the expansion centre is the midpoint of the bounding box
//     of the box's far nodes, R_B the largest node distance from it, R_T the
//     largest centroid distance.
//  4. Lists per target leaf T, descending from the root: box B is accepted
//     for M2P when |c_B - c_T| - R_T > 0 and R_B < theta (|c_B - c_T| - R_T);
//     a leaf that fails goes to the P2P list; other boxes are opened.  A
//     counting pass sizes everything, scans give offsets, and a second pass
//     writes the lists, the P2P tasks (the leaf's source panels cut into
//     chunks, as sub-ranges, sized so that every task carries about the same
//     number of target-source pairs), the M2P tasks (likewise) and the
//     partial-sum slot of every task.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>
#include <cmath>
#include <vector>

#include "runtime.hpp"

namespace pbmp {

namespace {

constexpr int kLevels = 21;
constexpr int kStack = 8 * (kLevels + 1);

// 21 bits -> every third bit
__device__ inline uint64_t spread3_d(uint64_t x) {
  x &= 0x1fffffull;
  x = (x | x << 32) & 0x1f00000000ffffull;
  x = (x | x << 16) & 0x1f0000ff0000ffull;
  x = (x | x << 8) & 0x100f00f00f00f00full;
  x = (x | x << 4) & 0x10c30c30c30c30c3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}

// centroids (caller's order) of the triangles, SoA
__global__ void k_user_centroids(int N, const double *__restrict__ verts,
                                 const int *__restrict__ tri, double *__restrict__ c) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const double *A = verts + 3 * tri[3 * j], *B = verts + 3 * tri[3 * j + 1],
               *C = verts + 3 * tri[3 * j + 2];
  for (int d = 0; d < 3; ++d) c[(size_t)d * N + j] = (A[d] + B[d] + C[d]) / 3.0;
}

// bounding box of the centroids: one block, box[0..5] = lo xyz, hi xyz
__global__ __launch_bounds__(1024) void k_bbox(int N, const double *__restrict__ c,
                                               double *__restrict__ box) {
  __shared__ double red[6][1024];
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int j = threadIdx.x; j < N; j += 1024)
    for (int d = 0; d < 3; ++d) {
      const double v = c[(size_t)d * N + j];
      lo[d] = fmin(lo[d], v);
      hi[d] = fmax(hi[d], v);
    }
  for (int d = 0; d < 3; ++d) {
    red[d][threadIdx.x] = lo[d];
    red[3 + d][threadIdx.x] = hi[d];
  }
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int d = 0; d < 3; ++d) {
        red[d][threadIdx.x] = fmin(red[d][threadIdx.x], red[d][threadIdx.x + w]);
        red[3 + d][threadIdx.x] = fmax(red[3 + d][threadIdx.x], red[3 + d][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) box[threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_morton_keys(int N, const double *__restrict__ c, const double *__restrict__ box,
                              uint64_t *__restrict__ key, int *__restrict__ idx) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const double ext = fmax(fmax(fmax(box[3] - box[0], box[4] - box[1]), box[5] - box[2]), 1e-12);
  uint64_t k = 0;
  for (int d = 0; d < 3; ++d) {
    const double u = (c[(size_t)d * N + j] - box[d]) / ext;
    const double g = fmin(2097151.0, fmax(0.0, floor(u * 2097152.0)));
    k |= spread3_d((uint64_t)g) << (2 - d);
  }
  key[j] = k;
  idx[j] = j;
}

// ---- level-by-level octree --------------------------------------------
struct Boxes {
  int *start, *end, *level, *parent, *first, *nchild;
};

__global__ void k_root(Boxes b, int N, int *__restrict__ owner) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    b.start[0] = 0;
    b.end[0] = N;
    b.level[0] = 0;
    b.parent[0] = -1;
    b.first[0] = -1;
    b.nchild[0] = 0;
  }
  if (i < N) owner[i] = 0;
}

// flag[i] = 1 where a child cell (level l+1) starts inside a box of level l
// that is split
__global__ void k_mark(int N, int l, int leaf, const uint64_t *__restrict__ key,
                       const int *__restrict__ owner, Boxes b, int *__restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int B = owner[i];
  int f = 0;
  if (b.level[B] == l && b.end[B] - b.start[B] > leaf && l < kLevels) {
    const int sh = 3 * (kLevels - 1 - l);
    f = (i == b.start[B]) || (((key[i] >> sh) & 7ull) != ((key[i - 1] >> sh) & 7ull));
  }
  flag[i] = f;
}

__global__ void k_emit(int N, int l, int base, const int *__restrict__ flag,
                       const int *__restrict__ idx, const int *__restrict__ owner, Boxes b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N || !flag[i]) return;
  const int k = base + idx[i], P = owner[i];
  b.start[k] = i;
  b.level[k] = l + 1;
  b.parent[k] = P;
  b.first[k] = -1;
  b.nchild[k] = 0;
  if (i == b.start[P]) b.first[P] = k;
}

__global__ void k_ends(int base, int nnew, Boxes b) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nnew) return;
  const int k = base + t, P = b.parent[k];
  const bool last = (t + 1 == nnew) || b.parent[k + 1] != P;
  b.end[k] = last ? b.end[P] : b.start[k + 1];
  if (last) b.nchild[P] = k - b.first[P] + 1;
}

__global__ void k_owner(int N, int l, int base, const int *__restrict__ flag,
                        const int *__restrict__ idx, Boxes b, int *__restrict__ owner) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int B = owner[i];
  if (b.level[B] == l && b.nchild[B] > 0) owner[i] = base + idx[i] + flag[i] - 1;
}

// leaves in key order (the order of their panel ranges): a panel that
// starts its leaf flags it; the leaf containing panel i is owner[i]
__global__ void k_leaf_flags(int N, const int *__restrict__ owner, Boxes b,
                             int *__restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) flag[i] = b.start[owner[i]] == i;
}

__global__ void k_leaf_list(int N, const int *__restrict__ flag, const int *__restrict__ idx,
                            const int *__restrict__ owner, int *__restrict__ leaves) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N && flag[i]) leaves[idx[i]] = owner[i];
}

// ranges and the 8-wide child table in the layout of the product kernels
__global__ void k_pack_boxes(int nbox, Boxes b, int *__restrict__ range,
                             int *__restrict__ child) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nbox) return;
  range[2 * k] = b.start[k];
  range[2 * k + 1] = b.end[k];
  for (int c = 0; c < 8; ++c) child[8 * k + c] = c < b.nchild[k] ? b.first[k] + c : -1;
}

// ---- box geometry: one wave per box -------------------------------------
__device__ inline double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__global__ __launch_bounds__(64) void k_box_geometry(int nbox, int nf, int N, Boxes b,
                                                     const double *__restrict__ src64,
                                                     const double *__restrict__ geo,
                                                     double *__restrict__ center,
                                                     double *__restrict__ radius) {
  const int B = blockIdx.x;
  const int s0 = b.start[B], s1 = b.end[B];
  const int n = (s1 - s0) * nf;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int g = threadIdx.x; g < n; g += 64) {
    const double *y = src64 + 16 * (size_t)(s0 + g / nf) + 3 * (g % nf);
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], y[d]);
      hi[d] = fmax(hi[d], y[d]);
    }
  }
  double c[3];
  for (int d = 0; d < 3; ++d) c[d] = 0.5 * (wave_min(lo[d]) + wave_max(hi[d]));
  double rb = 0.0, rt = 0.0;
  for (int g = threadIdx.x; g < n; g += 64) {
    const double *y = src64 + 16 * (size_t)(s0 + g / nf) + 3 * (g % nf);
    double r2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double t = y[d] - c[d];
      r2 += t * t;
    }
    rb = fmax(rb, r2);
  }
  for (int j = s0 + (int)threadIdx.x; j < s1; j += 64) {
    double r2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double t = geo[(size_t)d * N + j] - c[d];
      r2 += t * t;
    }
    rt = fmax(rt, r2);
  }
  rb = wave_max(rb);
  rt = wave_max(rt);
  if (threadIdx.x == 0) {
    for (int d = 0; d < 3; ++d) center[3 * B + d] = c[d];
    radius[2 * B] = sqrt(rb);
    radius[2 * B + 1] = sqrt(rt);
  }
}

// ---- interaction lists -------------------------------------------------
// Sources per task for a leaf of nt targets when every task should carry
// about `work` target-source pairs: the launches are short, so the longest
// task sets their duration and tasks of equal work keep every wave busy to
// the end.
constexpr int kMinChunk = 32, kMaxChunk = 4096;
__device__ inline int task_chunk(int work, int nt, int lo, int hi) {
  return min(hi, max(lo, work / max(1, nt)));
}

struct ListOut {
  // counting pass: per leaf [8]: n_m2p, n_p2p, n_sub, n_ptask, n_mtask,
  // p2p panels, targets, spare
  int *count;
  // filling pass (offsets = exclusive scans of the counts)
  const int *off_m2p, *off_p2p, *off_sub, *off_ptask, *off_mtask;
  int *m2p_box, *p2p_box, *sub, *ptask, *pslot, *mtask, *mslot;
  int *slots_of_box;
};

// P2P task of one source run [sb, se) of sub-ranges over the leaf's
// targets, writing slot `slot`
__device__ inline void emit_p2p(const ListOut &out, int at, int slot, int t0, int t1, int sb,
                                int se) {
  int *tk = out.ptask + 4 * at;
  tk[0] = t0;
  tk[1] = t1;
  tk[2] = sb;
  tk[3] = se;
  out.pslot[at] = slot;
}

template <bool FILL>
__global__ void k_lists(int nleaf, const int *__restrict__ leaves, Boxes b,
                        const double *__restrict__ center, const double *__restrict__ radius,
                        double theta, int chunk, int mchunk, ListOut out) {
  const int li = blockIdx.x * blockDim.x + threadIdx.x;
  if (li >= nleaf) return;
  const int T = leaves[li];
  const double cT[3] = {center[3 * T], center[3 * T + 1], center[3 * T + 2]};
  const double RT = radius[2 * T + 1];
  const int t0 = b.start[T], t1 = b.end[T];
  // equal work per task: chunk and mchunk arrive as target-source pairs per
  // task and become sources per task for this leaf's size
  chunk = task_chunk(chunk, t1 - t0, kMinChunk, kMaxChunk);
  mchunk = task_chunk(mchunk, t1 - t0, 1, kM2PChunkBoxes);
  int nm = 0, np = 0, nsub = 0, ntask = 0, nemit = 0, cnt = 0, panels = 0;
  int om = 0, op = 0, os = 0, ot = 0, firstsub = 0;
  if (FILL) {
    om = out.off_m2p[li];
    op = out.off_p2p[li];
    os = out.off_sub[li];
    ot = out.off_ptask[li];
    firstsub = os;
  }
  int stack[kStack];
  int top = 0;
  stack[top++] = 0;
  while (top > 0) {
    const int B = stack[--top];
    double d2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double t = center[3 * B + d] - cT[d];
      d2 += t * t;
    }
    const double sep = sqrt(d2) - RT;
    if (sep > 0.0 && radius[2 * B] < theta * sep) {
      if (FILL) out.m2p_box[om + nm] = B;
      ++nm;
    } else if (b.nchild[B] == 0) {
      if (FILL) out.p2p_box[op + np] = B;
      ++np;
      int s0 = b.start[B];
      const int s1 = b.end[B];
      panels += s1 - s0;
      while (s0 < s1) {
        const int take = min(s1 - s0, chunk - cnt);
        if (FILL) {
          out.sub[2 * (os + nsub)] = s0;
          out.sub[2 * (os + nsub) + 1] = s0 + take;
        }
        ++nsub;
        s0 += take;
        cnt += take;
        if (cnt == chunk) {
          if (FILL) {
            emit_p2p(out, ot + nemit, ntask, t0, t1, firstsub, os + nsub);
            firstsub = os + nsub;
          }
          ++nemit;
          ++ntask;
          cnt = 0;
        }
      }
    } else {
      for (int c = b.nchild[B] - 1; c >= 0; --c) stack[top++] = b.first[B] + c;
    }
  }
  if (cnt > 0) {
    if (FILL) emit_p2p(out, ot + nemit, ntask, t0, t1, firstsub, os + nsub);
    ++nemit;
    ++ntask;
  }
  const int nmt = (nm + mchunk - 1) / mchunk;
  if (FILL) {
    const int omt = out.off_mtask[li];
    for (int k = 0; k < nmt; ++k) {
      int *tk = out.mtask + 4 * (omt + k);
      tk[0] = t0;
      tk[1] = t1;
      tk[2] = om + k * mchunk;
      tk[3] = om + min((k + 1) * mchunk, nm);
      out.mslot[omt + k] = ntask + k;
    }
    out.slots_of_box[T] = ntask + nmt;
  } else {
    int *c = out.count + 8 * (size_t)li;
    c[0] = nm;
    c[1] = np;
    c[2] = nsub;
    c[3] = nemit;
    c[4] = nmt;
    c[5] = panels;
    c[6] = t1 - t0;
    c[7] = ntask;
  }
}

__global__ void k_column(int n, const int *__restrict__ count, int c, int *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = count[8 * (size_t)i + c];
}

__global__ void k_column2(int n, const int *__restrict__ count, int c, int *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = count[2 * (size_t)i + c];
}

__global__ void k_target_slots(int N, const int *__restrict__ owner,
                               const int *__restrict__ slots_of_box, int *__restrict__ tsl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) tsl[i] = slots_of_box[owner[i]];
}


// ---- transposed lists (for the adjoint product) -------------------------
// entries of a per-leaf CSR list as (box, leaf index) pairs
__global__ void k_expand_pairs(int nleaf, const int *__restrict__ ptr,
                               const int *__restrict__ box, int *__restrict__ key,
                               int *__restrict__ val) {
  const int li = blockIdx.x * blockDim.x + threadIdx.x;
  if (li >= nleaf) return;
  for (int e = ptr[li]; e < ptr[li + 1]; ++e) {
    key[e] = box[e];
    val[e] = li;
  }
}

// CSR over boxes from pairs sorted by box: [first[b], last[b])
__global__ void k_runs(int n, const int *__restrict__ key, int *__restrict__ first,
                       int *__restrict__ last) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  if (e == 0 || key[e] != key[e - 1]) first[key[e]] = e;
  if (e == n - 1 || key[e] != key[e + 1]) last[key[e]] = e + 1;
}

__global__ void k_fill_int(int n, int v, int *__restrict__ a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// Tasks of the transposed products.  For every box B (one thread), its
// transposed list (the target leaves that hold B, in leaf order) is cut into
// chunks of at most `chunk` target panels, stored as target sub-ranges.
// count[b] = (sub-ranges, tasks); the filling pass writes
// task = (box, sub begin, sub end, slot) and the sub-ranges.
template <bool FILL>
__global__ void k_tasks_T(int nbox, const int *__restrict__ first, const int *__restrict__ last,
                          const int *__restrict__ val, const int *__restrict__ leaves, Boxes b,
                          int chunk, bool per_source, int *__restrict__ count,
                          const int *__restrict__ off_sub,
                          const int *__restrict__ off_task, int *__restrict__ sub,
                          int *__restrict__ task) {
  const int B = blockIdx.x * blockDim.x + threadIdx.x;
  if (B >= nbox) return;
  // equal work per task (P2P^T: the box's own panels times the targets)
  if (per_source) chunk = task_chunk(chunk, b.end[B] - b.start[B], kMinChunk, kMaxChunk);
  int nsub = 0, ntask = 0, cnt = 0, os = 0, ot = 0, firstsub = 0;
  if (FILL) {
    os = off_sub[B];
    ot = off_task[B];
    firstsub = os;
  }
  for (int e = first[B]; e < last[B]; ++e) {
    const int T = leaves[val[e]];
    int s0 = b.start[T];
    const int s1 = b.end[T];
    while (s0 < s1) {
      const int take = min(s1 - s0, chunk - cnt);
      if (FILL) {
        sub[2 * (os + nsub)] = s0;
        sub[2 * (os + nsub) + 1] = s0 + take;
      }
      ++nsub;
      s0 += take;
      cnt += take;
      if (cnt == chunk) {
        if (FILL) {
          int *tk = task + 4 * (ot + ntask);
          tk[0] = B;
          tk[1] = firstsub;
          tk[2] = os + nsub;
          tk[3] = ntask;
          firstsub = os + nsub;
        }
        ++ntask;
        cnt = 0;
      }
    }
  }
  if (cnt > 0) {
    if (FILL) {
      int *tk = task + 4 * (ot + ntask);
      tk[0] = B;
      tk[1] = firstsub;
      tk[2] = os + nsub;
      tk[3] = ntask;
    }
    ++ntask;
  }
  if (!FILL) {
    count[2 * B] = nsub;
    count[2 * B + 1] = ntask;
  }
}

// per panel: number of transposed slots of its leaf (P2P^T tasks + 1)
__global__ void k_source_slots(int N, const int *__restrict__ owner,
                               const int *__restrict__ count, int *__restrict__ tsl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) tsl[i] = count[2 * owner[i] + 1] + 1;
}


// ---- moment tasks --------------------------------------------------------
__global__ void k_need_moments(int n, const int *__restrict__ m2p_box, int *__restrict__ need) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) need[m2p_box[e]] = 1;  // every writer stores the same value
}

// node tasks for the moments of every leaf (the inputs of every shift)
__global__ void k_mom_counts(int nbox, Boxes b, int chunk, int *__restrict__ count) {
  const int B = blockIdx.x * blockDim.x + threadIdx.x;
  if (B < nbox) count[B] = b.nchild[B] == 0 ? (b.end[B] - b.start[B] + chunk - 1) / chunk : 0;
}

__global__ void k_leaf_starts(int nleaf, const int *__restrict__ leaves, Boxes b,
                              int *__restrict__ ls) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < nleaf) ls[l] = b.start[leaves[l]];
}

__device__ inline int lower_bound_int(const int *a, int n, int v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// shift tasks of every accepted box with children: its leaves (a
// contiguous run of the key-ordered leaves, those starting inside its
// panel range) in runs of at most `chunk`
__global__ void k_shift_counts(int nbox, const int *__restrict__ need, Boxes b,
                               const int *__restrict__ ls, int nleaf, int chunk,
                               int *__restrict__ range, int *__restrict__ count) {
  const int B = blockIdx.x * blockDim.x + threadIdx.x;
  if (B >= nbox) return;
  const int l0 = lower_bound_int(ls, nleaf, b.start[B]);
  const int l1 = lower_bound_int(ls, nleaf, b.end[B]);
  range[2 * B] = l0;
  range[2 * B + 1] = l1;
  count[B] = (need[B] && b.nchild[B] > 0) ? (l1 - l0 + chunk - 1) / chunk : 0;
}

__global__ void k_shift_fill(int nbox, const int *__restrict__ first,
                             const int *__restrict__ count, const int *__restrict__ range,
                             int chunk, int *__restrict__ task) {
  const int B = blockIdx.x * blockDim.x + threadIdx.x;
  if (B >= nbox) return;
  for (int k = 0; k < count[B]; ++k) {
    int *tk = task + 3 * (first[B] + k);
    tk[0] = B;
    tk[1] = range[2 * B] + k * chunk;
    tk[2] = min(range[2 * B + 1], range[2 * B] + (k + 1) * chunk);
  }
}

__global__ void k_mom_fill(int nbox, const int *__restrict__ first,
                           const int *__restrict__ count, Boxes b, int chunk,
                           int *__restrict__ task) {
  const int B = blockIdx.x * blockDim.x + threadIdx.x;
  if (B >= nbox) return;
  for (int k = 0; k < count[B]; ++k) {
    int *tk = task + 3 * (first[B] + k);
    tk[0] = B;
    tk[1] = b.start[B] + k * chunk;
    tk[2] = min(b.end[B], b.start[B] + (k + 1) * chunk);
  }
}

inline dim3 grid_for(size_t n, int b = 256) { return dim3((unsigned)((n + b - 1) / b)); }

// exclusive scan of n ints on the device; returns the total
int exclusive_scan_total(hipStream_t s, const int *in, int *out, int n, Dbuf<char> &tmp) {
  if (n <= 0) return 0;
  size_t bytes = 0;
  PBMP_HIP(rocprim::exclusive_scan(nullptr, bytes, in, out, 0, (size_t)n,
                                   rocprim::plus<int>(), s));
  tmp.reserve(std::max<size_t>(bytes, 1));
  PBMP_HIP(rocprim::exclusive_scan(tmp.p, bytes, in, out, 0, (size_t)n,
                                   rocprim::plus<int>(), s));
  int last[2];
  PBMP_HIP(hipMemcpyAsync(&last[0], out + n - 1, sizeof(int), hipMemcpyDeviceToHost, s));
  PBMP_HIP(hipMemcpyAsync(&last[1], in + n - 1, sizeof(int), hipMemcpyDeviceToHost, s));
  PBMP_HIP(hipStreamSynchronize(s));
  return last[0] + last[1];
}

}  // namespace

void morton_order_device(hipStream_t s, int N, const double *verts, const int *tri_user,
                         int *perm, uint64_t *key_sorted) {
  Dbuf<double> cen, box;
  Dbuf<uint64_t> key;
  Dbuf<int> idx;
  Dbuf<char> tmp;
  cen.alloc(3 * (size_t)N);
  box.alloc(6);
  key.alloc(N);
  idx.alloc(N);
  hipLaunchKernelGGL(k_user_centroids, grid_for(N), dim3(256), 0, s, N, verts, tri_user, cen.p);
  hipLaunchKernelGGL(k_bbox, dim3(1), dim3(1024), 0, s, N, cen.p, box.p);
  hipLaunchKernelGGL(k_morton_keys, grid_for(N), dim3(256), 0, s, N, cen.p, box.p, key.p, idx.p);
  PBMP_HIP(hipGetLastError());
  size_t bytes = 0;
  PBMP_HIP(rocprim::radix_sort_pairs(nullptr, bytes, key.p, key_sorted, idx.p, perm, (size_t)N,
                                     0, 63, s));
  tmp.alloc(std::max<size_t>(bytes, 1));
  PBMP_HIP(rocprim::radix_sort_pairs(tmp.p, bytes, key.p, key_sorted, idx.p, perm, (size_t)N, 0,
                                     63, s));
  PBMP_HIP(hipStreamSynchronize(s));
}

void Tree::build_device(int N, int nf, const uint64_t *key, const double *geo,
                        const double *src64, hipStream_t s) {
  stream_ = s;
  ncoef = (prm.order + 1) * (prm.order + 2) * (prm.order + 3) / 6;
  ncoefK = (prm.order + 2) * (prm.order + 3) * (prm.order + 4) / 6;
  nmom = ncoef + ncoefK;
  Dbuf<int> owner, flag, idx;
  Dbuf<char> tmp;
  owner.alloc(N);
  flag.alloc(N);
  idx.alloc(N);
  // box arrays with room to grow
  int cap = std::max(64, 2 * N / std::max(1, prm.leaf) + 64);
  auto alloc_boxes = [&](int c) {
    Dbuf<int> *arr[6] = {&d_start, &d_end, &d_level, &d_parent, &d_first, &d_nchild};
    for (Dbuf<int> *a : arr) {
      Dbuf<int> nb;
      nb.alloc(c);
      if (a->n) PBMP_HIP(hipMemcpyAsync(nb.p, a->p, sizeof(int) * a->n,
                                        hipMemcpyDeviceToDevice, s));
      PBMP_HIP(hipStreamSynchronize(s));
      a->swap(nb);
    }
  };
  d_start.release();
  d_end.release();
  d_level.release();
  d_parent.release();
  d_first.release();
  d_nchild.release();
  alloc_boxes(cap);
  auto view = [&]() {
    return Boxes{d_start.p, d_end.p, d_level.p, d_parent.p, d_first.p, d_nchild.p};
  };
  hipLaunchKernelGGL(k_root, grid_for(N), dim3(256), 0, s, view(), N, owner.p);
  nbox = 1;
  depth = 0;
  level_start.assign({0, 1});
  for (int l = 0; l < kLevels; ++l) {
    hipLaunchKernelGGL(k_mark, grid_for(N), dim3(256), 0, s, N, l, prm.leaf, key, owner.p,
                       view(), flag.p);
    const int nnew = exclusive_scan_total(s, flag.p, idx.p, N, tmp);
    if (nnew == 0) break;
    if (nbox + nnew > cap) {
      cap = std::max(2 * cap, nbox + nnew + 64);
      alloc_boxes(cap);
    }
    hipLaunchKernelGGL(k_emit, grid_for(N), dim3(256), 0, s, N, l, nbox, flag.p, idx.p,
                       owner.p, view());
    hipLaunchKernelGGL(k_ends, grid_for(nnew), dim3(256), 0, s, nbox, nnew, view());
    hipLaunchKernelGGL(k_owner, grid_for(N), dim3(256), 0, s, N, l, nbox, flag.p, idx.p,
                       view(), owner.p);
    PBMP_HIP(hipGetLastError());
    nbox += nnew;
    depth = l + 1;
    level_start.push_back(nbox);
  }
  // leaves in key order: target leaves (and so tasks) that follow each
  // other are neighbours in space, and the tasks that one XCD takes share
  // their sources in its L2
  hipLaunchKernelGGL(k_leaf_flags, grid_for(N), dim3(256), 0, s, N, owner.p, view(), flag.p);
  nleaf = exclusive_scan_total(s, flag.p, idx.p, N, tmp);
  d_leaves.alloc(nleaf);
  hipLaunchKernelGGL(k_leaf_list, grid_for(N), dim3(256), 0, s, N, flag.p, idx.p, owner.p,
                     d_leaves.p);
  d_range.alloc(2 * (size_t)nbox);
  d_child.alloc(8 * (size_t)nbox);
  hipLaunchKernelGGL(k_pack_boxes, grid_for(nbox), dim3(256), 0, s, nbox, view(), d_range.p,
                     d_child.p);
  // geometry
  d_center.alloc(3 * (size_t)nbox);
  d_radius.alloc(2 * (size_t)nbox);
  hipLaunchKernelGGL(k_box_geometry, dim3(nbox), dim3(64), 0, s, nbox, nf, N, view(), src64,
                     geo, d_center.p, d_radius.p);
  PBMP_HIP(hipGetLastError());
  // lists: count, scan, fill
  Dbuf<int> cnt, col, off[5];
  cnt.alloc(8 * (size_t)nleaf);
  col.alloc(nleaf);
  ListOut lo{};
  lo.count = cnt.p;
  hipLaunchKernelGGL(k_lists<false>, grid_for(nleaf, 64), dim3(64), 0, s, nleaf, d_leaves.p,
                     view(), d_center.p, d_radius.p, prm.theta, kP2PTaskWork,
                     kM2PTaskWork, lo);
  PBMP_HIP(hipGetLastError());
  int tot[5];
  for (int c = 0; c < 5; ++c) {
    off[c].alloc(nleaf + 1);
    hipLaunchKernelGGL(k_column, grid_for(nleaf), dim3(256), 0, s, nleaf, cnt.p, c, col.p);
    tot[c] = exclusive_scan_total(s, col.p, off[c].p, nleaf, tmp);
    PBMP_HIP(hipMemcpyAsync(off[c].p + nleaf, &tot[c], sizeof(int), hipMemcpyHostToDevice, s));
    PBMP_HIP(hipStreamSynchronize(s));
  }
  n_m2p_entries = tot[0];
  n_p2p_entries = tot[1];
  n_p2p_tasks = tot[3];
  n_m2p_tasks = tot[4];
  d_m2p_box.alloc(std::max(1, tot[0]));
  d_p2p_box.alloc(std::max(1, tot[1]));
  d_p2p_src.alloc(2 * (size_t)std::max(1, tot[2]));
  d_p2p_task.alloc(4 * (size_t)std::max(1, tot[3]));
  d_p2p_slot.alloc(std::max(1, tot[3]));
  d_m2p_task.alloc(4 * (size_t)std::max(1, tot[4]));
  d_m2p_slot.alloc(std::max(1, tot[4]));
  Dbuf<int> slots_of_box;
  slots_of_box.alloc(nbox);
  lo.off_m2p = off[0].p;
  lo.off_p2p = off[1].p;
  lo.off_sub = off[2].p;
  lo.off_ptask = off[3].p;
  lo.off_mtask = off[4].p;
  lo.m2p_box = d_m2p_box.p;
  lo.p2p_box = d_p2p_box.p;
  lo.sub = d_p2p_src.p;
  lo.ptask = d_p2p_task.p;
  lo.pslot = d_p2p_slot.p;
  lo.mtask = d_m2p_task.p;
  lo.mslot = d_m2p_slot.p;
  lo.slots_of_box = slots_of_box.p;
  hipLaunchKernelGGL(k_lists<true>, grid_for(nleaf, 64), dim3(64), 0, s, nleaf, d_leaves.p,
                     view(), d_center.p, d_radius.p, prm.theta, kP2PTaskWork,
                     kM2PTaskWork, lo);
  d_tslots.alloc(N);
  hipLaunchKernelGGL(k_target_slots, grid_for(N), dim3(256), 0, s, N, owner.p, slots_of_box.p,
                     d_tslots.p);
  PBMP_HIP(hipGetLastError());
  d_m2p_ptr.alloc(nleaf + 1);
  d_p2p_ptr.alloc(nleaf + 1);
  PBMP_HIP(hipMemcpyAsync(d_m2p_ptr.p, off[0].p, sizeof(int) * (nleaf + 1),
                          hipMemcpyDeviceToDevice, s));
  PBMP_HIP(hipMemcpyAsync(d_p2p_ptr.p, off[1].p, sizeof(int) * (nleaf + 1),
                          hipMemcpyDeviceToDevice, s));
  // transposed lists and tasks (adjoint product): P2P^T per source leaf,
  // M2P^T per accepted box
  build_transposed(N, owner.p, tmp);
  // per-product work counts and the largest slot count (host bookkeeping
  // for launches and counters)
  std::vector<int> h(8 * (size_t)nleaf);
  cnt.download(h.data(), h.size(), s);
  PBMP_HIP(hipStreamSynchronize(s));
  direct_pairs = m2p_pairs = 0.0;
  max_slots = 0;
  for (int k = 0; k < nleaf; ++k) {
    const int *c = &h[8 * (size_t)k];
    direct_pairs += (double)c[6] * c[5] * nf;
    m2p_pairs += (double)c[6] * c[0];
    max_slots = std::max(max_slots, c[7] + c[4]);
  }
  // moment tasks for the boxes that some leaf accepts
  {
    Dbuf<int> need;
    need.alloc(nbox);
    hipLaunchKernelGGL(k_fill_int, grid_for(nbox), dim3(256), 0, s, nbox, 0, need.p);
    if (n_m2p_entries > 0)
      hipLaunchKernelGGL(k_need_moments, grid_for(n_m2p_entries), dim3(256), 0, s,
                         n_m2p_entries, d_m2p_box.p, need.p);
    d_mom_count.alloc(nbox);
    d_mom_first.alloc(nbox);
    hipLaunchKernelGGL(k_mom_counts, grid_for(nbox), dim3(256), 0, s, nbox, view(),
                       mom_chunk_panels(prm.order), d_mom_count.p);
    n_mom_tasks = exclusive_scan_total(s, d_mom_count.p, d_mom_first.p, nbox, tmp);
    d_mom_task.alloc(3 * (size_t)std::max(1, n_mom_tasks));
    hipLaunchKernelGGL(k_mom_fill, grid_for(nbox), dim3(256), 0, s, nbox, d_mom_first.p,
                       d_mom_count.p, view(), mom_chunk_panels(prm.order), d_mom_task.p);
    d_mom_part.alloc((size_t)std::max(1, n_mom_tasks) * nmom);
    // shifts of the leaf moments to the accepted boxes above them
    Dbuf<int> ls, range;
    ls.alloc(std::max(1, nleaf));
    range.alloc(2 * (size_t)nbox);
    hipLaunchKernelGGL(k_leaf_starts, grid_for(nleaf), dim3(256), 0, s, nleaf, d_leaves.p,
                       view(), ls.p);
    d_shift_count.alloc(nbox);
    d_shift_first.alloc(nbox);
    hipLaunchKernelGGL(k_shift_counts, grid_for(nbox), dim3(256), 0, s, nbox, need.p, view(),
                       ls.p, nleaf, kShiftLeaves, range.p, d_shift_count.p);
    n_shift_tasks = exclusive_scan_total(s, d_shift_count.p, d_shift_first.p, nbox, tmp);
    {
      std::vector<int> hc(nbox);
      d_shift_count.download(hc.data(), nbox, s);
      PBMP_HIP(hipStreamSynchronize(s));
      shift_multi = std::any_of(hc.begin(), hc.end(), [](int c) { return c > 1; });
    }
    d_shift_task.alloc(3 * (size_t)std::max(1, n_shift_tasks));
    hipLaunchKernelGGL(k_shift_fill, grid_for(nbox), dim3(256), 0, s, nbox, d_shift_first.p,
                       d_shift_count.p, range.p, kShiftLeaves, d_shift_task.p);
    d_shift_part.alloc((size_t)std::max(1, n_shift_tasks) * nmom);
    PBMP_HIP(hipStreamSynchronize(s));
    PBMP_HIP(hipGetLastError());
  }
  d_mom64.alloc((size_t)nbox * nmom);
  d_mom32.alloc((size_t)nbox * nmom);
  PBMP_HIP(hipMemsetAsync(d_mom64.p, 0, sizeof(double) * nbox * nmom, s));
  tree_upload_exponents(*this, s);
  PBMP_HIP(hipStreamSynchronize(s));
}

void Tree::build_transposed(int N, const int *owner, Dbuf<char> &tmp) {
  hipStream_t s = stream_;
  auto view = [&]() {
    return Boxes{d_start.p, d_end.p, d_level.p, d_parent.p, d_first.p, d_nchild.p};
  };
  auto one = [&](const Dbuf<int> &ptr, const Dbuf<int> &box, int n, int chunk, bool per_source,
                 Dbuf<int> &tsub,
                 Dbuf<int> &ttask, Dbuf<int> &cnt_out, Dbuf<int> &off_task, int &ntasks) {
    Dbuf<int> key, val, skey, sval, first, last, col, off_sub;
    const int m = std::max(1, n);
    key.alloc(m);
    val.alloc(m);
    skey.alloc(m);
    sval.alloc(m);
    first.alloc(nbox);
    last.alloc(nbox);
    hipLaunchKernelGGL(k_fill_int, grid_for(nbox), dim3(256), 0, s, nbox, 0, first.p);
    hipLaunchKernelGGL(k_fill_int, grid_for(nbox), dim3(256), 0, s, nbox, 0, last.p);
    if (n > 0) {
      hipLaunchKernelGGL(k_expand_pairs, grid_for(nleaf), dim3(256), 0, s, nleaf, ptr.p, box.p,
                         key.p, val.p);
      size_t bytes = 0;
      unsigned bits = 1;
      while ((1u << bits) < (unsigned)nbox) ++bits;
      PBMP_HIP(rocprim::radix_sort_pairs(nullptr, bytes, key.p, skey.p, val.p, sval.p,
                                         (size_t)n, 0, bits, s));
      tmp.reserve(std::max<size_t>(bytes, 1));
      PBMP_HIP(rocprim::radix_sort_pairs(tmp.p, bytes, key.p, skey.p, val.p, sval.p,
                                         (size_t)n, 0, bits, s));
      hipLaunchKernelGGL(k_runs, grid_for(n), dim3(256), 0, s, n, skey.p, first.p, last.p);
    }
    cnt_out.alloc(2 * (size_t)nbox);
    hipLaunchKernelGGL(k_tasks_T<false>, grid_for(nbox, 64), dim3(64), 0, s, nbox, first.p,
                       last.p, sval.p, d_leaves.p, view(), chunk, per_source, cnt_out.p, nullptr,
                       nullptr,
                       nullptr, nullptr);
    col.alloc(nbox);
    off_sub.alloc(nbox);
    off_task.alloc(nbox);
    hipLaunchKernelGGL(k_column2, grid_for(nbox), dim3(256), 0, s, nbox, cnt_out.p, 0, col.p);
    const int nsub = exclusive_scan_total(s, col.p, off_sub.p, nbox, tmp);
    hipLaunchKernelGGL(k_column2, grid_for(nbox), dim3(256), 0, s, nbox, cnt_out.p, 1, col.p);
    ntasks = exclusive_scan_total(s, col.p, off_task.p, nbox, tmp);
    tsub.alloc(2 * (size_t)std::max(1, nsub));
    ttask.alloc(4 * (size_t)std::max(1, ntasks));
    hipLaunchKernelGGL(k_tasks_T<true>, grid_for(nbox, 64), dim3(64), 0, s, nbox, first.p,
                       last.p, sval.p, d_leaves.p, view(), chunk, per_source, nullptr, off_sub.p,
                       off_task.p, tsub.p, ttask.p);
    PBMP_HIP(hipGetLastError());
    PBMP_HIP(hipStreamSynchronize(s));
  };
  Dbuf<int> p2pT_off;
  one(d_p2p_ptr, d_p2p_box, n_p2p_entries, kP2PTaskWork, true, d_p2pT_sub, d_p2pT_task,
      d_p2pT_count, p2pT_off, n_p2pT_tasks);
  one(d_m2p_ptr, d_m2p_box, n_m2p_entries, kM2PTChunkTargets, false, d_m2pT_sub, d_m2pT_task,
      d_m2pT_count, d_m2pT_off, n_m2pT_tasks);
  d_tslotsT.alloc(N);
  hipLaunchKernelGGL(k_source_slots, grid_for(N), dim3(256), 0, s, N, owner, d_p2pT_count.p,
                     d_tslotsT.p);
  PBMP_HIP(hipGetLastError());
  // largest slot count of a source panel
  std::vector<int> h(2 * (size_t)nbox);
  d_p2pT_count.download(h.data(), h.size(), s);
  PBMP_HIP(hipStreamSynchronize(s));
  max_slots_T = 1;
  for (int b = 0; b < nbox; ++b) max_slots_T = std::max(max_slots_T, h[2 * b + 1] + 1);
}

}  // namespace pbmp
