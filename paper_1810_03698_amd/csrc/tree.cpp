// Octree, interaction lists and work decomposition of the treecode
// (section "The treecode algorithm").  Panels arrive sorted by the Morton key
// of their centroid in the bounding cube, so every octree cell is a
// contiguous range of panels; a cell is split while it holds more than
// `leaf` panels.  Sources are the far-field nodes of the panels, targets the
// centroids.  For every target leaf T and box B the acceptance criterion
//     R_B < theta * (|c_B - c_T| - R_T)
// (R_B: largest distance from the box centre to its nodes, R_T: largest
// distance from the target leaf centre to its targets) guarantees the
// paper's per-target criterion R_B / |x - c_B| < theta for every target x of
// T.  Accepted boxes go to T's M2P list; leaves that fail it to its P2P list.
#include <algorithm>
#include <cmath>
#include <functional>

#include "runtime.hpp"

namespace pbmp {

namespace {
#ifndef PBMP_P2P_CHUNK
#define PBMP_P2P_CHUNK 256
#endif
// source panels per P2P task: leaf ranges are cut at this size so that no
// task is much longer than the others (the launch is short enough for the
// longest task to set its duration)
constexpr int kP2PChunkPanels = PBMP_P2P_CHUNK;
}  // namespace

void Tree::build(int N, const double *cen, int nf,
                 const std::vector<double> &nodes, hipStream_t s) {
  (void)nodes;
  ncoef = (prm.order + 1) * (prm.order + 2) * (prm.order + 3) / 6;
  // ---- topology from Morton keys (recomputed with the same cube as the
  // panel ordering: per-axis minimum, largest extent)
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int j = 0; j < N; ++j)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], cen[d * N + j]);
      hi[d] = std::max(hi[d], cen[d * N + j]);
    }
  const double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-12});
  std::vector<uint32_t> q(3 * (size_t)N);
  for (int j = 0; j < N; ++j)
    for (int d = 0; d < 3; ++d) {
      const double u = (cen[d * N + j] - lo[d]) / ext;
      q[3 * j + d] = (uint32_t)std::min(2097151.0, std::max(0.0, u * 2097152.0));
    }
  auto octant = [&](int j, int lvl) {  // child index at depth lvl (1-based)
    const int sh = 21 - lvl;
    return (int)(((q[3 * j] >> sh) & 1) << 2 | ((q[3 * j + 1] >> sh) & 1) << 1 |
                 ((q[3 * j + 2] >> sh) & 1));
  };
  start.clear(); end.clear(); parent.clear(); level.clear();
  first_child.clear(); nchild.clear(); leaves.clear();
  std::vector<int> child_ids;
  std::function<int(int, int, int, int)> make = [&](int a, int b, int lvl, int par) -> int {
    const int id = (int)start.size();
    start.push_back(a);
    end.push_back(b);
    parent.push_back(par);
    level.push_back(lvl);
    first_child.push_back(-1);
    nchild.push_back(0);
    depth = std::max(depth, lvl);
    if (b - a <= prm.leaf || lvl >= 21) {
      leaves.push_back(id);
      return id;
    }
    // children: contiguous runs of equal octant (keys are sorted)
    std::vector<std::pair<int, int>> runs;
    int r0 = a;
    for (int j = a + 1; j <= b; ++j)
      if (j == b || octant(j, lvl + 1) != octant(r0, lvl + 1)) {
        runs.push_back({r0, j});
        r0 = j;
      }
    std::vector<int> kids;
    for (auto &r : runs) kids.push_back(make(r.first, r.second, lvl + 1, id));
    first_child[id] = (int)child_ids.size();
    nchild[id] = (int)kids.size();
    child_ids.insert(child_ids.end(), kids.begin(), kids.end());
    return id;
  };
  depth = 0;
  make(0, N, 0, -1);
  nbox = (int)start.size();
  nleaf = (int)leaves.size();
  // ---- geometry of the boxes
  center.assign(3 * (size_t)nbox, 0.0);
  radius.assign(nbox, 0.0);
  tradius.assign(nbox, 0.0);
  for (int b = 0; b < nbox; ++b) {
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (int j = start[b]; j < end[b]; ++j)
      for (int qn = 0; qn < nf; ++qn)
        for (int d = 0; d < 3; ++d) {
          const double v = nodes[(3 * (size_t)j + qn) * 3 + d];
          mn[d] = std::min(mn[d], v);
          mx[d] = std::max(mx[d], v);
        }
    for (int d = 0; d < 3; ++d) center[3 * b + d] = 0.5 * (mn[d] + mx[d]);
    double rb = 0.0, rt = 0.0;
    for (int j = start[b]; j < end[b]; ++j) {
      for (int qn = 0; qn < nf; ++qn) {
        double r2 = 0.0;
        for (int d = 0; d < 3; ++d) {
          const double t = nodes[(3 * (size_t)j + qn) * 3 + d] - center[3 * b + d];
          r2 += t * t;
        }
        rb = std::max(rb, r2);
      }
      double r2 = 0.0;
      for (int d = 0; d < 3; ++d) {
        const double t = cen[d * N + j] - center[3 * b + d];
        r2 += t * t;
      }
      rt = std::max(rt, r2);
    }
    radius[b] = std::sqrt(rb);
    tradius[b] = std::sqrt(rt);
  }
  // ---- interaction lists per target leaf
  p2p_ptr.assign(1, 0);
  m2p_ptr.assign(1, 0);
  p2p_src.clear();
  m2p_box.clear();
  direct_pairs = m2p_pairs = 0.0;
  std::vector<int> stack;
  for (int li = 0; li < nleaf; ++li) {
    const int T = leaves[li];
    stack.assign(1, 0);
    while (!stack.empty()) {
      const int B = stack.back();
      stack.pop_back();
      double d2 = 0.0;
      for (int d = 0; d < 3; ++d) {
        const double t = center[3 * B + d] - center[3 * T + d];
        d2 += t * t;
      }
      const double sep = std::sqrt(d2) - tradius[T];
      if (sep > 0.0 && radius[B] < prm.theta * sep) {
        m2p_box.push_back(B);
        m2p_pairs += (double)(end[T] - start[T]);
      } else if (nchild[B] == 0) {
        p2p_src.push_back(B);
        direct_pairs += (double)(end[T] - start[T]) * (end[B] - start[B]) * nf;
      } else {
        for (int c = nchild[B] - 1; c >= 0; --c) stack.push_back(child_ids[first_child[B] + c]);
      }
    }
    p2p_ptr.push_back((int)p2p_src.size());
    m2p_ptr.push_back((int)m2p_box.size());
  }
  // ---- tasks: (t0, t1, list begin, list end) and the partial slot each
  // writes; slots of a target leaf are 0..n-1 in a fixed order
  std::vector<int> pt, ps, mt, ms, tsl(N, 0), srcr;
  max_slots = 0;
  for (int li = 0; li < nleaf; ++li) {
    const int T = leaves[li];
    int slot = 0;
    // the leaf's source panels, in list order, cut into tasks of at most
    // kP2PChunkPanels panels; a task lists its source sub-ranges
    int first = (int)(srcr.size() / 2), cnt = 0;
    auto close_task = [&]() {
      pt.insert(pt.end(), {start[T], end[T], first, (int)(srcr.size() / 2)});
      ps.push_back(slot++);
      first = (int)(srcr.size() / 2);
      cnt = 0;
    };
    for (int a = p2p_ptr[li]; a < p2p_ptr[li + 1]; ++a) {
      int s0 = start[p2p_src[a]];
      const int s1 = end[p2p_src[a]];
      while (s0 < s1) {
        const int take = std::min(s1 - s0, kP2PChunkPanels - cnt);
        srcr.insert(srcr.end(), {s0, s0 + take});
        s0 += take;
        cnt += take;
        if (cnt == kP2PChunkPanels) close_task();
      }
    }
    if (cnt > 0) close_task();
    for (int c = m2p_ptr[li]; c < m2p_ptr[li + 1]; c += kM2PChunkBoxes) {
      mt.insert(mt.end(), {start[T], end[T], c, std::min(c + kM2PChunkBoxes, m2p_ptr[li + 1])});
      ms.push_back(slot++);
    }
    for (int j = start[T]; j < end[T]; ++j) tsl[j] = slot;
    max_slots = std::max(max_slots, slot);
  }
  n_p2p_tasks = (int)ps.size();
  n_m2p_tasks = (int)ms.size();
  if (srcr.empty()) srcr.assign(2, 0);
  std::vector<int> range(2 * (size_t)nbox), child(8 * (size_t)nbox, -1);
  for (int b = 0; b < nbox; ++b) {
    range[2 * b] = start[b];
    range[2 * b + 1] = end[b];
    for (int c = 0; c < nchild[b]; ++c) child[8 * b + c] = child_ids[first_child[b] + c];
  }
  // boxes by level, deepest first: leaves get P2M, inner boxes M2M
  level_ptr.assign(1, 0);
  std::vector<int> order;
  for (int l = depth; l >= 0; --l) {
    for (int b = 0; b < nbox; ++b)
      if (level[b] == l && nchild[b] > 0) order.push_back(b);
    level_ptr.push_back((int)order.size());
  }
  if (order.empty()) order.push_back(0);
  if (pt.empty()) pt.assign(4, 0), ps.assign(1, 0);
  if (mt.empty()) mt.assign(4, 0), ms.assign(1, 0);
  std::vector<int> mb(m2p_box);
  if (mb.empty()) mb.push_back(0);
  d_center.upload(center.data(), center.size(), s);
  d_range.upload(range.data(), range.size(), s);
  d_child.upload(child.data(), child.size(), s);
  d_p2p_task.upload(pt.data(), pt.size(), s);
  d_p2p_slot.upload(ps.data(), ps.size(), s);
  d_p2p_src.upload(srcr.data(), srcr.size(), s);
  d_m2p_task.upload(mt.data(), mt.size(), s);
  d_m2p_slot.upload(ms.data(), ms.size(), s);
  d_m2p_box.upload(mb.data(), mb.size(), s);
  d_tslots.upload(tsl.data(), tsl.size(), s);
  d_leaf_boxes.upload(order.data(), order.size(), s);
  std::vector<int> lv(leaves);
  d_leaves.upload(lv.data(), lv.size(), s);
  d_mom64.alloc((size_t)nbox * 2 * ncoef);
  d_mom32.alloc((size_t)nbox * 2 * ncoef);
  tree_upload_exponents(*this, s);
  PBMP_HIP(hipStreamSynchronize(s));
}

}  // namespace pbmp
