// Read-back of the device-built octree and interaction lists (inspection
// and tests).
#include <algorithm>

#include "runtime.hpp"

namespace pbmp {

void Runtime::tree_export(int64_t counts[4], int32_t *perm, int32_t *box_range,
                          int32_t *box_level, double *box_centre, double *box_radius,
                          int32_t *leaf_box, int32_t *m2p_ptr, int32_t *m2p_box,
                          int32_t *p2p_ptr, int32_t *p2p_box) const {
  PBMP_REQUIRE(tree_active_ && tree_, PBMP_ESTATE, "no treecode octree on this context");
  const Tree &t = *tree_;
  if (counts) {
    counts[0] = t.nbox;
    counts[1] = t.nleaf;
    counts[2] = t.n_m2p_entries;
    counts[3] = t.n_p2p_entries;
  }
  if (perm) std::copy(perm_.begin(), perm_.end(), perm);
  if (box_range) t.d_range.download(box_range, 2 * (size_t)t.nbox, s_);
  if (box_level) t.d_level.download(box_level, t.nbox, s_);
  if (box_centre) t.d_center.download(box_centre, 3 * (size_t)t.nbox, s_);
  if (box_radius) t.d_radius.download(box_radius, 2 * (size_t)t.nbox, s_);
  if (leaf_box) t.d_leaves.download(leaf_box, t.nleaf, s_);
  if (m2p_ptr) t.d_m2p_ptr.download(m2p_ptr, t.nleaf + 1, s_);
  if (m2p_box) t.d_m2p_box.download(m2p_box, t.n_m2p_entries, s_);
  if (p2p_ptr) t.d_p2p_ptr.download(p2p_ptr, t.nleaf + 1, s_);
  if (p2p_box) t.d_p2p_box.download(p2p_box, t.n_p2p_entries, s_);
  PBMP_HIP(hipStreamSynchronize(s_));
}

}  // namespace pbmp
