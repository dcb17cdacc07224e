// Octree over the panels (internal Morton order) for the treecode product.
#pragma once

#include <vector>

#include "common.hpp"

namespace pbmp {

// boxes per M2P task (one task's moments are staged in LDS)
constexpr int kM2PChunkBoxes = 32;

struct TreeParams {
  double theta = 0.5;
  int order = 4;
  int leaf = 300;
};

class Tree {
 public:
  TreeParams prm;
  int nbox = 0, nleaf = 0, ncoef = 0, depth = 0;
  // host topology
  std::vector<int> start, end, parent, level, first_child, nchild;
  std::vector<double> center, radius, tradius;  // [3*nbox], [nbox], [nbox]
  std::vector<int> leaves;                      // box ids of leaves
  // interaction lists per target leaf (CSR over leaf index)
  std::vector<int> p2p_ptr, p2p_src;  // source leaf box ids
  std::vector<int> m2p_ptr, m2p_box;  // accepted boxes
  // tasks
  int n_p2p_tasks = 0, n_m2p_tasks = 0, max_slots = 0;
  double direct_pairs = 0.0, m2p_pairs = 0.0;  // per product (nodes / boxes)

  // device data
  Dbuf<double> d_center;  // [3*nbox]
  Dbuf<int> d_range;      // [2*nbox] start, end
  Dbuf<int> d_p2p_task;   // [4*n] t0, t1, list begin, list end (+ slot below)
  Dbuf<int> d_p2p_slot;
  Dbuf<int> d_p2p_src;    // source sub-ranges of the P2P tasks: [2*len] start, end
  Dbuf<int> d_m2p_task;
  Dbuf<int> d_m2p_slot;
  Dbuf<int> d_m2p_box;
  Dbuf<int> d_tslots;     // [N] number of slots of the target's leaf
  Dbuf<int> d_leaves;     // leaf box ids
  Dbuf<int> d_leaf_boxes; // boxes with moments needed, by level (bottom-up)
  std::vector<int> level_ptr;  // CSR of d_leaf_boxes per level
  Dbuf<int> d_child;      // [8*nbox] child ids (-1 none)
  Dbuf<double> d_mom64;   // [nbox][2][ncoef]
  Dbuf<float> d_mom32;    // [nbox][2][ncoef]
  Dbuf<int> d_monos;      // [3*ncoef] exponents

  // Build from Morton-sorted panel centroids and far-field nodes (host data).
  void build(int N, const double *cen /*SoA 3N*/, int nf,
             const std::vector<double> &nodes /*[N][nf][3]*/, hipStream_t s);
};

// upload the multi-index exponent table of the chosen order (d_monos)
void tree_upload_exponents(Tree &t, hipStream_t s);

}  // namespace pbmp
