// Octree over the panels (internal Morton order) for the treecode product,
// built on the device (k_treebuild.hip).
#pragma once

#include <vector>

#include "common.hpp"

namespace pbmp {

// P2P tasks: source tile in LDS, targets per lane bound, lane groups on/off
#ifndef PBMP_P2P_TILE
#define PBMP_P2P_TILE 128
#endif
#ifndef PBMP_P2P_MAXTPT
#define PBMP_P2P_MAXTPT 5
#endif
#ifndef PBMP_P2P_GROUPS
#define PBMP_P2P_GROUPS 1
#endif
#ifndef PBMP_M2P_GROUPS
#define PBMP_M2P_GROUPS 0
#endif

struct LaneSplit {
  int G, L, tpt;
};

// Lanes of a one-wave P2P task for nt targets: G groups of L = 64 / G lanes,
// tpt targets per lane, maximising the useful fraction G nt / (64 tpt) with
// tpt <= PBMP_P2P_MAXTPT (ties: fewer groups; more than 64 * MAXTPT
// targets take several passes with G = 1)
__host__ __device__ inline LaneSplit lane_split(int nt) {
  const int t1 = (nt + 63) / 64;
  LaneSplit best{1, 64, t1 < PBMP_P2P_MAXTPT ? t1 : PBMP_P2P_MAXTPT};
  float be = (float)nt / (64.0f * best.tpt * ((nt + 64 * best.tpt - 1) / (64 * best.tpt)));
  for (int G = 2; G <= 16 * PBMP_P2P_GROUPS; ++G) {
    const int L = 64 / G;
    const int tpt = (nt + L - 1) / L;
    if (tpt > PBMP_P2P_MAXTPT) continue;
    const float e = (float)(G * nt) / (64.0f * tpt);
    if (e > be) {
      be = e;
      best = LaneSplit{G, L, tpt};
    }
  }
  return best;
}

// boxes per M2P task (one task's moments are staged in LDS)
#ifndef PBMP_M2P_CHUNK
#define PBMP_M2P_CHUNK 16
#endif
constexpr int kM2PChunkBoxes = PBMP_M2P_CHUNK;
// work per task, in target-source pairs: a leaf of nt targets gets tasks of
// about kP2PTaskWork / nt source panels (P2P) and kM2PTaskWork / nt boxes
// (M2P, at most kM2PChunkBoxes), so that tasks take about the same time
#ifndef PBMP_P2P_WORK
#define PBMP_P2P_WORK 12288
#endif
#ifndef PBMP_M2P_WORK
#define PBMP_M2P_WORK 1024
#endif
constexpr int kP2PTaskWork = PBMP_P2P_WORK;
constexpr int kM2PTaskWork = PBMP_M2P_WORK;
// panels per moment task
// Panels per moment task: one wave per task, so a slice bounds the nodes a
// lane walks; higher orders carry a longer wave reduction per task and
// take longer slices (measured fastest: 512 up to P = 4, 1024 above).
#ifdef PBMP_MOM_CHUNK
inline int mom_chunk_panels(int) { return PBMP_MOM_CHUNK; }
#else
inline int mom_chunk_panels(int order) { return order <= 4 ? 512 : 1024; }
#endif
// leaves per shift task (moments of the boxes above the leaves)
constexpr int kShiftLeaves = 16;
// target panels per M2P^T task (adjoint product)
constexpr int kM2PTChunkTargets = 512;

struct TreeParams {
  double theta = 0.5;
  int order = 4;
  int leaf = 300;
};

class Tree {
 public:
  TreeParams prm;
  // coefficient counts: ncoef = C(P+3, 3) single-layer terms (|k| <= P),
  // ncoefK = C(P+4, 3) double-layer terms (|k| <= P + 1: the double-layer
  // moment of degree |k| holds h^(|k|-1), so both layers reach degree P in
  // h); moments and local coefficients of a box are [ncoef | ncoefK]
  int nbox = 0, nleaf = 0, ncoef = 0, ncoefK = 0, nmom = 0, depth = 0;
  std::vector<int> level_start;  // boxes of level l are [level_start[l], level_start[l+1])
  // tasks and list sizes
  int n_p2p_tasks = 0, n_m2p_tasks = 0, max_slots = 0;
  int n_m2p_entries = 0, n_p2p_entries = 0;
  double direct_pairs = 0.0, m2p_pairs = 0.0;  // per product (nodes / boxes)

  // boxes (ids level by level, key order within a level)
  Dbuf<int> d_start, d_end, d_level, d_parent, d_first, d_nchild;
  Dbuf<int> d_range;      // [2*nbox] start, end
  Dbuf<int> d_child;      // [8*nbox] child ids (-1 none)
  Dbuf<double> d_center;  // [3*nbox] expansion centres
  Dbuf<double> d_radius;  // [2*nbox] R_B (far nodes), R_T (centroids)
  Dbuf<int> d_leaves;     // [nleaf] leaf box ids (the target leaves)
  // lists per target leaf (CSR over the leaf index)
  Dbuf<int> d_m2p_ptr, d_m2p_box;  // accepted boxes
  Dbuf<int> d_p2p_ptr, d_p2p_box;  // leaves summed directly
  // tasks
  Dbuf<int> d_p2p_task;   // [4*n] t0, t1, sub-range begin, end
  Dbuf<int> d_p2p_slot;
  Dbuf<int> d_p2p_src;    // source sub-ranges of the P2P tasks: [2*len] start, end
  Dbuf<int> d_m2p_task;   // [4*n] t0, t1, list begin, end
  Dbuf<int> d_m2p_slot;
  Dbuf<int> d_tslots;     // [N] number of slots of the target's leaf
  // transposed (adjoint) product: P2P^T tasks per source leaf and M2P^T
  // tasks per accepted box, each over target sub-ranges;
  // task = (box, sub begin, sub end, slot)
  Dbuf<int> d_p2pT_sub, d_p2pT_task, d_p2pT_count;  // count[2*box] = (subs, tasks)
  Dbuf<int> d_m2pT_sub, d_m2pT_task, d_m2pT_count, d_m2pT_off;  // off: first task of a box
  Dbuf<int> d_tslotsT;    // [N] transposed slots of the panel's leaf (tasks + 1)
  int n_p2pT_tasks = 0, n_m2pT_tasks = 0, max_slots_T = 1;
  Dbuf<double> d_Lpart, d_L;  // local coefficients: per M2P^T task, per box [2][ncoefK]
  // moment tasks: the panels of every leaf in slices of at most
  // mom_chunk_panels(P); task = (box, s0, s1); a box's slices are consecutive
  int n_mom_tasks = 0;
  Dbuf<int> d_mom_task, d_mom_first, d_mom_count;
  Dbuf<double> d_mom_part;  // [n_mom_tasks][nmom]
  // shift tasks: the leaves under an accepted box with children in runs of
  // at most kShiftLeaves; task = (box, first leaf index, end leaf index)
  int n_shift_tasks = 0;
  bool shift_multi = false;  // some box has several shift tasks
  Dbuf<int> d_shift_task, d_shift_first, d_shift_count;
  Dbuf<double> d_shift_part;  // [n_shift_tasks][nmom]
  Dbuf<int> d_shift_toff, d_shift_tjq;  // per coefficient k: terms [toff[k], toff[k+1]), (j, k-j)
  Dbuf<double> d_shift_tc;              // C(k, j) of each term
  Dbuf<double> d_mom64;   // [nbox][nmom]
  Dbuf<float> d_mom32;    // [nbox][nmom]
  Dbuf<int> d_monos;      // [3*ncoefK] exponents up to degree P + 1

  // Build from the Morton keys of the panels in internal (sorted) order,
  // the centroids (geo SoA) and far nodes (src64 records), all on device.
  void build_device(int N, int nf, const uint64_t *key, const double *geo,
                    const double *src64, hipStream_t s);

 private:
  hipStream_t stream_ = nullptr;
  void build_transposed(int N, const int *owner, Dbuf<char> &tmp);
};

// Morton order of the panels on the device: perm[i] = caller's index of the
// i-th panel, key_sorted[i] its key (tri_user: the caller's triangles)
void morton_order_device(hipStream_t s, int N, const double *verts, const int *tri_user,
                         int *perm, uint64_t *key_sorted);

// upload the multi-index exponent table of the chosen order (d_monos)
void tree_upload_exponents(Tree &t, hipStream_t s);

}  // namespace pbmp
