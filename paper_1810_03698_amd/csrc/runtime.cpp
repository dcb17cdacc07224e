// Host runtime of the pbmp library: mesh and site preparation, the
// boundary-integral operator, device GMRES, the induced-dipole loops and the
// solvation energy (sections "The boundary element method", "Self-consistent
// induced field", "Calculation of the solvation energy").
#include "runtime.hpp"

#include <algorithm>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>

namespace pbmp {

double coulomb_kcal() {
  const double e = 1.602176634e-19, NA = 6.02214076e23, eps0 = 8.8541878128e-12;
  return e * e * NA / (4.0 * M_PI * eps0 * 1e-10 * 4184.0);
}

double debye_per_e_ang() {
  const double e = 1.602176634e-19, c = 299792458.0;
  return e * 1e-10 * c / 1e-21;
}

namespace {

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) {
  return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

template <class T>
std::vector<T> fetch(const T *p, size_t n, int where, hipStream_t s) {
  std::vector<T> h(n);
  if (n == 0) return h;
  PBMP_REQUIRE(p != nullptr, PBMP_EARG, "null input pointer");
  if (where == PBMP_DEVICE) {
    PBMP_HIP(hipMemcpyAsync(h.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, s));
    PBMP_HIP(hipStreamSynchronize(s));
  } else {
    std::memcpy(h.data(), p, n * sizeof(T));
  }
  return h;
}

bool finite_all(const std::vector<double> &v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

// Uniform-grid neighbour search: for every query point q_l, the panels j
// with |q_l - c_j| < radius(l, j) (strict).  The grid cell is at least the
// largest radius.
struct Grid {
  double lo[3], h;
  int64_t dims[3];
  std::vector<int64_t> key;  // sorted cell key per slot
  std::vector<int> idx;      // panel id per slot
  void build(const std::vector<double> &cen, int N, double cell) {
    for (int d = 0; d < 3; ++d) {
      double mn = 1e300, mx = -1e300;
      for (int j = 0; j < N; ++j) {
        mn = std::min(mn, cen[d * N + j]);
        mx = std::max(mx, cen[d * N + j]);
      }
      lo[d] = mn;
      dims[d] = std::max<int64_t>(1, (int64_t)std::floor((mx - mn) / cell) + 1);
    }
    h = cell;
    std::vector<std::pair<int64_t, int>> kv(N);
    for (int j = 0; j < N; ++j) kv[j] = {cell_key(cen[j], cen[N + j], cen[2 * N + j]), j};
    std::sort(kv.begin(), kv.end());
    key.resize(N);
    idx.resize(N);
    for (int j = 0; j < N; ++j) {
      key[j] = kv[j].first;
      idx[j] = kv[j].second;
    }
  }
  int64_t coord(double x, int d) const {
    int64_t c = (int64_t)std::floor((x - lo[d]) / h);
    return std::min<int64_t>(std::max<int64_t>(c, 0), dims[d] - 1);
  }
  int64_t cell_key(double x, double y, double z) const {
    return (coord(x, 0) * dims[1] + coord(y, 1)) * dims[2] + coord(z, 2);
  }
  template <class F> void visit(double x, double y, double z, F &&f) const {
    const int64_t c0 = coord(x, 0), c1 = coord(y, 1), c2 = coord(z, 2);
    for (int64_t a = std::max<int64_t>(0, c0 - 1); a <= std::min(dims[0] - 1, c0 + 1); ++a)
      for (int64_t b = std::max<int64_t>(0, c1 - 1); b <= std::min(dims[1] - 1, c1 + 1); ++b)
        for (int64_t c = std::max<int64_t>(0, c2 - 1); c <= std::min(dims[2] - 1, c2 + 1); ++c) {
          const int64_t k = (a * dims[1] + b) * dims[2] + c;
          auto it = std::lower_bound(key.begin(), key.end(), k);
          for (; it != key.end() && *it == k; ++it) f(idx[it - key.begin()]);
        }
  }
};

}  // namespace

// ------------------------------------------------------------ clock
hipEvent_t KernelClock::begin(hipStream_t s) {
  hipEvent_t e;
  if (pool.empty()) {
    PBMP_HIP(hipEventCreate(&e));
  } else {
    e = pool.back();
    pool.pop_back();
  }
  PBMP_HIP(hipEventRecord(e, s));
  return e;
}

void KernelClock::end(hipStream_t s, hipEvent_t a, int kind, double pairs) {
  hipEvent_t b;
  if (pool.empty()) {
    PBMP_HIP(hipEventCreate(&b));
  } else {
    b = pool.back();
    pool.pop_back();
  }
  PBMP_HIP(hipEventRecord(b, s));
  pending.push_back({a, b, kind});
  if (kind == P2P) {
    p2p_launches += 1;
    p2p_pairs += pairs;
  } else if (kind == M2P) {
    m2p_launches += 1;
    m2p_pairs += pairs;
  }
  if (pending.size() > 4096) resolve();
}

void KernelClock::resolve() {
  for (auto &p : pending) {
    PBMP_HIP(hipEventSynchronize(p.b));
    float ms = 0.f;
    PBMP_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    if (p.kind == P2P) p2p_ms += ms;
    else if (p.kind == M2P) m2p_ms += ms;
    else p2m_ms += ms;
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  pending.clear();
}

void KernelClock::reset() {
  resolve();
  p2p_ms = m2p_ms = p2m_ms = near_ms = matvec_ms = 0;
  p2p_launches = m2p_launches = matvec_calls = 0;
  p2p_pairs = m2p_pairs = 0;
}

KernelClock::~KernelClock() {
  for (auto &p : pending) {
    (void)hipEventSynchronize(p.b);
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

// ------------------------------------------------------------------ ctor
Runtime::Runtime(const pbmp_options &opt) : o(opt) {
  PBMP_REQUIRE(o.eps_in > 0 && o.eps_out > 0 && o.kappa >= 0, PBMP_EARG,
               "eps_in, eps_out must be > 0 and kappa >= 0");
  PBMP_REQUIRE(o.gauss_far == 1 || o.gauss_far == 3, PBMP_EARG,
               "gauss_far must be 1 or 3");
  PBMP_REQUIRE(o.near_eta >= 0, PBMP_EARG, "near_eta must be >= 0");
  PBMP_REQUIRE(o.mode >= 0 && o.mode <= 2, PBMP_EARG, "bad mode");
  PBMP_REQUIRE(o.theta > 0 && o.theta < 1, PBMP_EARG, "theta must be in (0,1)");
  PBMP_REQUIRE(o.order_P >= 1 && o.order_P <= 6, PBMP_EARG, "order_P in 1..6");
  PBMP_REQUIRE(o.leaf_panels >= 8, PBMP_EARG, "leaf_panels >= 8");
  PBMP_REQUIRE(o.gmres_restart >= 1 && o.gmres_restart <= 200, PBMP_EARG,
               "gmres_restart in 1..200");
  PBMP_REQUIRE(o.gmres_tol > 0 && o.gmres_maxit >= 1, PBMP_EARG,
               "gmres_tol > 0, gmres_maxit >= 1");
  PBMP_REQUIRE(o.scf_tol_debye > 0 && o.scf_maxit >= 1, PBMP_EARG,
               "scf_tol_debye > 0, scf_maxit >= 1");
  PBMP_REQUIRE(o.scf_omega > 0 && o.scf_omega < 2, PBMP_EARG, "scf_omega in (0,2)");
  PBMP_REQUIRE(o.thole_a >= 0, PBMP_EARG, "thole_a >= 0");
  PBMP_REQUIRE(o.precision == PBMP_FP64 || o.precision == PBMP_MIXED, PBMP_EARG,
               "bad precision");
  TriRule f = far_rule(o.gauss_far), nr = near_rule19();
  ru_.nf = f.n;
  ru_.nn = nr.n;
  for (int q = 0; q < f.n; ++q) {
    for (int d = 0; d < 3; ++d) ru_.fb[q][d] = f.b[q][d];
    ru_.fw[q] = f.w[q];
  }
  for (int q = 0; q < nr.n; ++q) {
    for (int d = 0; d < 3; ++d) ru_.nb[q][d] = nr.b[q][d];
    ru_.nw[q] = nr.w[q];
  }
  ru_.ngl = 16;
  gauss_legendre(16, ru_.glx, ru_.glw);
  // the first HIP calls come after the host-only set-up above: the static
  // scratch's device address is looked up now (once per device), so that
  // the entry point using it makes no runtime set-up call itself
  (void)static_scratch();
  if (o.hip_stream) {
    s_ = reinterpret_cast<hipStream_t>(o.hip_stream);
  } else {
    PBMP_HIP(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
    own_stream_ = true;
  }
}

void Runtime::set_options(const pbmp_options &n) {
  const double kap = outer_ ? kappa_ext_ : o.kappa;
  const double eout = outer_ ? eps_out_ext_ : o.eps_out;
  PBMP_REQUIRE(n.eps_in == o.eps_in && n.eps_out == eout && n.kappa == kap &&
                   n.gauss_far == o.gauss_far && n.near_eta == o.near_eta &&
                   n.mode == o.mode && n.theta == o.theta && n.order_P == o.order_P &&
                   n.leaf_panels == o.leaf_panels && n.thole_a == o.thole_a,
               PBMP_EARG, "only the solver settings and the precision can change on a context");
  PBMP_REQUIRE(n.precision == PBMP_FP64 || n.precision == PBMP_MIXED, PBMP_EARG,
               "precision must be PBMP_FP64 or PBMP_MIXED");
  PBMP_REQUIRE(n.precision == o.precision || !outer_, PBMP_EARG,
               "the precision of a context with a Stern layer is fixed");
  PBMP_REQUIRE(n.gmres_restart >= 1 && n.gmres_restart <= 200, PBMP_EARG,
               "gmres_restart in 1..200");
  PBMP_REQUIRE(n.gmres_tol > 0 && n.gmres_maxit >= 1, PBMP_EARG,
               "gmres_tol > 0, gmres_maxit >= 1");
  PBMP_REQUIRE(n.scf_tol_debye > 0 && n.scf_maxit >= 1, PBMP_EARG,
               "scf_tol_debye > 0, scf_maxit >= 1");
  PBMP_REQUIRE(n.scf_omega > 0 && n.scf_omega < 2, PBMP_EARG, "scf_omega in (0,2)");
  const bool restart_changed = n.gmres_restart != o.gmres_restart;
  const bool precision_changed = n.precision != o.precision;
  o.precision = n.precision;
  o.gmres_restart = n.gmres_restart;
  o.gmres_tol = n.gmres_tol;
  o.gmres_maxit = n.gmres_maxit;
  o.scf_tol_debye = n.scf_tol_debye;
  o.scf_omega = n.scf_omega;
  o.scf_maxit = n.scf_maxit;
  o.warm_start = n.warm_start;
  o.verbose = n.verbose;
  if (outer_) {
    outer_->o.gmres_restart = n.gmres_restart;
    outer_->o.gmres_tol = n.gmres_tol;
    outer_->o.gmres_maxit = n.gmres_maxit;
  }
  if (precision_changed && N_ > 0) {
    // the near corrections remove the far rule as the product of this
    // precision evaluates it; the solution and dipoles stay (a backward may
    // follow a solve at the other precision)
    near_values();
    alloc_work();
  } else if (restart_changed && N_ > 0) {
    alloc_work();
    if (outer_)
      partial_.reserve((size_t)(o.gmres_restart + 2) * ((sX_.n + 4095) / 4096 + 1));
  }
}

Runtime::~Runtime() {
  try {
    clock.resolve();
  } catch (...) {
  }
  if (s_) (void)hipStreamSynchronize(s_);
  for (hipEvent_t e : kev_) (void)hipEventDestroy(e);
  if (hpin_) (void)hipHostFree(hpin_);
  if (own_stream_ && s_) (void)hipStreamDestroy(s_);
}

void Runtime::sync() { PBMP_HIP(hipStreamSynchronize(s_)); }

// -------------------------------------------------------------- set_mesh
void Runtime::set_mesh(int64_t nv, const double *verts, int64_t nt,
                       const int32_t *tris, int where) {
  auto t0 = clk::now();
  ax_holds_x_ = gax_holds_x_ = false;
  adj_ok_ = false;
  PBMP_REQUIRE(nv >= 4 && nt >= 4 && nt < (1 << 28) && nv < (1 << 28), PBMP_EARG,
               "mesh sizes out of range");
  PBMP_REQUIRE(where == PBMP_HOST || where == PBMP_DEVICE, PBMP_EARG, "bad where");
  std::vector<double> hv = fetch(verts, 3 * nv, where, s_);
  std::vector<int32_t> ht = fetch(tris, 3 * nt, where, s_);
  PBMP_REQUIRE(finite_all(hv), PBMP_EARG, "non-finite vertex coordinate");
  const int N = (int)nt, Nv = (int)nv;
  // --- topology: every directed edge once, and its reverse once
  std::vector<uint64_t> edges;
  edges.reserve(3 * N);
  for (int j = 0; j < N; ++j) {
    const int a = ht[3 * j], b = ht[3 * j + 1], c = ht[3 * j + 2];
    PBMP_REQUIRE(a >= 0 && a < Nv && b >= 0 && b < Nv && c >= 0 && c < Nv,
                 PBMP_EMESH, "triangle vertex index out of range");
    PBMP_REQUIRE(a != b && b != c && a != c, PBMP_EMESH, "degenerate triangle");
    edges.push_back((uint64_t)a * Nv + b);
    edges.push_back((uint64_t)b * Nv + c);
    edges.push_back((uint64_t)c * Nv + a);
  }
  std::sort(edges.begin(), edges.end());
  for (size_t k = 1; k < edges.size(); ++k)
    PBMP_REQUIRE(edges[k] != edges[k - 1], PBMP_EMESH,
                 "mesh not 2-manifold or inconsistently oriented (repeated directed edge)");
  for (uint64_t e : edges) {
    const uint64_t a = e / Nv, b = e % Nv;
    PBMP_REQUIRE(std::binary_search(edges.begin(), edges.end(), b * Nv + a),
                 PBMP_EMESH, "mesh not closed (edge without its reverse)");
  }
  // --- enclosed volume
  double vol = 0.0;
  for (int j = 0; j < N; ++j) {
    const double *A = &hv[3 * ht[3 * j]], *B = &hv[3 * ht[3 * j + 1]],
                 *C = &hv[3 * ht[3 * j + 2]];
    vol += A[0] * (B[1] * C[2] - B[2] * C[1]) + A[1] * (B[2] * C[0] - B[0] * C[2]) +
           A[2] * (B[0] * C[1] - B[1] * C[0]);
  }
  PBMP_REQUIRE(vol > 0, PBMP_EMESH, "enclosed volume not positive (inward orientation)");
  // --- Morton order of the centroids (device radix sort)
  verts_.upload(hv.data(), hv.size(), s_);
  {
    Dbuf<int> tri_user;
    tri_user.upload(ht.data(), ht.size(), s_);
    d_perm_.alloc(N);
    keys_.alloc(N);
    morton_order_device(s_, N, verts_.p, tri_user.p, d_perm_.p, keys_.p);
  }
  perm_.resize(N);
  d_perm_.download(perm_.data(), N, s_);
  sync();
  h_tri_.resize(3 * (size_t)N);
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < 3; ++k) h_tri_[3 * i + k] = ht[3 * perm_[i] + k];
  N_ = N;
  Nv_ = Nv;
  warm_ok_ = false;
  h_verts_ = hv;
  solved_ = false;
  M_ = 0;
  tri_.upload(h_tri_.data(), h_tri_.size(), s_);
  geo_.alloc(7 * (size_t)N);
  src64_.alloc(16 * (size_t)N);
  src32_.alloc(16 * (size_t)N);
  tgt32_.alloc(3 * (size_t)N);
  launch_panel_geometry(s_, N, verts_.p, tri_.p, ru_, geo_.p, src64_.p,
                        src32_.p, tgt32_.p);
  h_geo_.resize(7 * (size_t)N);
  geo_.download(h_geo_.data(), h_geo_.size(), s_);
  sync();
  for (int j = 0; j < N; ++j)
    PBMP_REQUIRE(h_geo_[6 * (size_t)N + j] > 1e-12, PBMP_EMESH,
                 "panel with area <= 1e-12 A^2");
  // The three far nodes are interior: a node lies at least (smallest
  // altitude)/6 from its panel's boundary, hence from every other panel's
  // centroid, and a third of a median from its own.  When that exceeds 1e-4 A
  // plus the FP32 rounding of the coordinates, no FP32 pair distance can
  // fall below the cut-off and the product may skip the test.  The one-node
  // rule puts the node on its own centroid, so it always needs the test.
  {
    double min_alt = 1e300, max_abs = 0.0;
    for (int j = 0; j < N; ++j) {
      const int *t = &h_tri_[3 * (size_t)j];
      double len2 = 0.0;
      for (int e = 0; e < 3; ++e) {
        const double *a = &hv[3 * t[e]], *b = &hv[3 * t[(e + 1) % 3]];
        double l2 = 0.0;
        for (int d = 0; d < 3; ++d) {
          l2 += (a[d] - b[d]) * (a[d] - b[d]);
          max_abs = std::max(max_abs, std::fabs(a[d]));
        }
        len2 = std::max(len2, l2);
      }
      min_alt = std::min(min_alt, 2.0 * h_geo_[6 * (size_t)N + j] / std::sqrt(len2));
    }
    floor_r2_ = o.gauss_far == 1 || !(min_alt / 6.0 > 1e-4 + 1e-6 * max_abs);
  }
  build_near_lists();
  // --- tree
  tree_active_ = (o.mode == PBMP_MODE_TREECODE) ||
                 (o.mode == PBMP_MODE_AUTO && N > 20000);
  tree_.reset();
  if (tree_active_) {
    tree_.reset(new Tree());
    tree_->prm.theta = o.theta;
    tree_->prm.order = o.order_P;
    tree_->prm.leaf = o.leaf_panels;
    tree_->build_device(N, ru_.nf, keys_.p, geo_.p, src64_.p, s_);
  }
  alloc_work();
  sync();
  t_setup_ms_ = ms_since(t0);
  setup_reported_ = false;
}

void Runtime::build_near_lists() {
  const int N = N_;
  const double *g = h_geo_.data();
  double rmax = 0.0;
  for (int j = 0; j < N; ++j) rmax = std::max(rmax, o.near_eta * std::sqrt(g[6 * N + j]));
  Grid grid;
  grid.build(h_geo_, N, std::max(rmax, 1e-9));
  std::vector<int> row(N + 1, 0), col;
  col.reserve(16 * (size_t)N);
  std::vector<int> tmp;
  for (int i = 0; i < N; ++i) {
    const double x = g[i], y = g[N + i], z = g[2 * N + i];
    const double rad = o.near_eta * std::sqrt(g[6 * N + i]);
    tmp.clear();
    tmp.push_back(i);
    grid.visit(x, y, z, [&](int j) {
      if (j == i) return;
      const double dx = x - g[j], dy = y - g[N + j], dz = z - g[2 * N + j];
      const double dist = std::sqrt(dx * dx + dy * dy + dz * dz);
      if (dist < rad) tmp.push_back(j);
    });
    std::sort(tmp.begin() + 1, tmp.end());
    col.insert(col.end(), tmp.begin(), tmp.end());
    row[i + 1] = (int)col.size();
  }
  nrow_.upload(row.data(), row.size(), s_);
  ncol_.upload(col.data(), col.size(), s_);
  nnz_ = (int)col.size();
  nval_.alloc(4 * col.size());
  diag_.alloc(2 * (size_t)N);
  near_values();
  // transposed structure: for column j, the entry ids e with col[e] == j
  std::vector<int> trow(N + 1, 0), tent(col.size()), tcol(col.size());
  for (int c : col) trow[c + 1]++;
  for (int j = 0; j < N; ++j) trow[j + 1] += trow[j];
  std::vector<int> fill(trow.begin(), trow.end() - 1);
  for (int i = 0; i < N; ++i)
    for (int e = row[i]; e < row[i + 1]; ++e) {
      const int k = fill[col[e]]++;
      tent[k] = e;
      tcol[k] = i;
    }
  trow_.upload(trow.data(), trow.size(), s_);
  tcol_.upload(tcol.data(), tcol.size(), s_);
  tent_.upload(tent.data(), tent.size(), s_);
  sync();
}

// near/self correction values for the current precision (and, in mixed
// precision, against the FP64 far field for the refinement's products)
void Runtime::near_values() {
  const int N = N_;
  launch_near_values(s_, fp64(), N, nrow_.p, ncol_.p, verts_.p, tri_.p, geo_.p,
                     src64_.p, src32_.p, tgt32_.p, ru_, o.kappa, nval_.p, diag_.p);
  if (!fp64()) {
    nval64_.alloc(nval_.n);
    launch_near_values(s_, true, N, nrow_.p, ncol_.p, verts_.p, tri_.p, geo_.p, src64_.p,
                       src32_.p, tgt32_.p, ru_, o.kappa, nval64_.p, diag_.p);
  } else {
    nval64_.release();
  }
  sync();
}

void Runtime::alloc_work() {
  ax_holds_x_ = gax_holds_x_ = false;
  const int N = N_;
  const int n = 2 * N;
  const int m = o.gmres_restart;
  // direct-product chunking: enough blocks to fill the device
  const int tpt = fp64() ? 1 : 2;
  const int bx = (N + 256 * tpt - 1) / (256 * tpt);
  p2p_chunks_ = std::max(1, std::min((2048 + bx - 1) / bx, (N + 127) / 128));
  int slots = p2p_chunks_;
  if (tree_active_) slots = std::max({slots, tree_->max_slots, tree_->max_slots_T});
  part_.alloc((size_t)slots * 4 * N);
  V_.alloc((size_t)(m + 1) * n);
  w_.alloc(n);
  z_.alloc(n);
  ax_.alloc(n);
  b_.alloc(n);
  x_.alloc(n);
  ybuf_.alloc(m + 2);
  hbuf_.alloc(3 * (m + 2));
  partial_.alloc((size_t)(m + 2) * ((n + 4095) / 4096 + 1));
  tmp_.alloc(n);
  io_a_.alloc(n > 0 ? n : 1);
  io_b_.alloc(n > 0 ? n : 1);
}

// ------------------------------------------------------------- set_sites
void Runtime::set_sites(int64_t m, const double *xyz, const double *q,
                        const double *d, const double *Q9, const double *alpha,
                        const int32_t *group, int where) {
  PBMP_REQUIRE(N_ > 0, PBMP_ESTATE, "set_mesh must precede set_sites");
  PBMP_REQUIRE(m >= 1 && m < (1 << 24), PBMP_EARG, "site count out of range");
  PBMP_REQUIRE(where == PBMP_HOST || where == PBMP_DEVICE, PBMP_EARG, "bad where");
  const int M = (int)m;
  auto hx = fetch(xyz, 3 * (size_t)M, where, s_);
  auto hq = fetch(q, M, where, s_);
  auto hd = fetch(d, 3 * (size_t)M, where, s_);
  auto hQ = fetch(Q9, 9 * (size_t)M, where, s_);
  auto ha = fetch(alpha, M, where, s_);
  std::vector<int32_t> hg(M);
  if (group)
    hg = fetch(group, M, where, s_);
  else
    std::iota(hg.begin(), hg.end(), 0);
  PBMP_REQUIRE(finite_all(hx) && finite_all(hq) && finite_all(hd) &&
                   finite_all(hQ) && finite_all(ha),
               PBMP_EARG, "non-finite site input");
  for (int l = 0; l < M; ++l) {
    PBMP_REQUIRE(ha[l] >= 0, PBMP_EARG, "negative polarisability");
    const double *Q = &hQ[9 * (size_t)l];
    double nrm = 0.0;
    for (int k = 0; k < 9; ++k) nrm = std::max(nrm, std::fabs(Q[k]));
    const double tol = 1e-10 * std::max(nrm, 1e-300);
    PBMP_REQUIRE(std::fabs(Q[1] - Q[3]) <= tol && std::fabs(Q[2] - Q[6]) <= tol &&
                     std::fabs(Q[5] - Q[7]) <= tol,
                 PBMP_EARG, "quadrupole not symmetric");
    PBMP_REQUIRE(std::fabs(Q[0] + Q[4] + Q[8]) <= tol || nrm == 0.0, PBMP_EARG,
                 "quadrupole not traceless");
  }
  for (int l = 0; l < M; ++l)
    for (int k = l + 1; k < M; ++k) {
      const double dx = hx[3 * l] - hx[3 * k], dy = hx[3 * l + 1] - hx[3 * k + 1],
                   dz = hx[3 * l + 2] - hx[3 * k + 2];
      PBMP_REQUIRE(dx * dx + dy * dy + dz * dz > 0, PBMP_EARG, "coincident sites");
      if (M > 4096) break;  // pairwise check only for small inputs
    }
  if (M != M_) warm_ok_ = false;
  M_ = M;
  h_sxyz_ = hx;
  sxyz_.upload(hx.data(), hx.size(), s_);
  sq_.upload(hq.data(), hq.size(), s_);
  sd_.upload(hd.data(), hd.size(), s_);
  sQ_.upload(hQ.data(), hQ.size(), s_);
  salpha_.upload(ha.data(), ha.size(), s_);
  sgroup_.upload(hg.data(), hg.size(), s_);
  // inside test
  Dbuf<double> wind;
  wind.alloc(M);
  launch_winding(s_, N_, M, verts_.p, tri_.p, sxyz_.p, wind.p);
  std::vector<double> hw(M);
  wind.download(hw.data(), M, s_);
  sync();
  for (int l = 0; l < M; ++l)
    PBMP_REQUIRE(hw[l] > 0.5, PBMP_ESITE,
                 "site " + std::to_string(l) + " lies outside the surface");
  build_site_lists();
  mu_d_.alloc(3 * (size_t)M);
  mu_v_.alloc(3 * (size_t)M);
  Eperm_.alloc(3 * (size_t)M);
  Eind_.alloc(3 * (size_t)M);
  reac_.alloc(10 * (size_t)M);
  ind_.alloc(10 * (size_t)M);
  vac_perm_.alloc(10 * (size_t)M);
  vac_ind_.alloc(10 * (size_t)M);
  p_.alloc(3 * (size_t)M);
  f_.alloc(N_);
  dmu2_.alloc(1);
  e_.alloc(10);
  ro_chunks_ = readout_chunks(N_, M);
  rpart_.alloc((size_t)ro_chunks_ * M * 10);
  solved_ = false;
}

// panels j with |p_l - c_j| < eta sqrt(A_j) for the points p (AoS) as CSR
// (row [M+1], col sorted per row; col holds at least one entry)
void Runtime::point_lists(const std::vector<double> &pts, int M, std::vector<int> &row,
                          std::vector<int> &col) const {
  const int N = N_;
  const double *g = h_geo_.data();
  double rmax = 0.0;
  for (int j = 0; j < N; ++j) rmax = std::max(rmax, o.near_eta * std::sqrt(g[6 * N + j]));
  Grid grid;
  grid.build(h_geo_, N, std::max(rmax, 1e-9));
  row.assign(M + 1, 0);
  col.clear();
  std::vector<int> tmp;
  for (int l = 0; l < M; ++l) {
    const double x = pts[3 * l], y = pts[3 * l + 1], z = pts[3 * l + 2];
    tmp.clear();
    grid.visit(x, y, z, [&](int j) {
      const double dx = x - g[j], dy = y - g[N + j], dz = z - g[2 * N + j];
      const double dist = std::sqrt(dx * dx + dy * dy + dz * dz);
      if (dist < o.near_eta * std::sqrt(g[6 * N + j])) tmp.push_back(j);
    });
    std::sort(tmp.begin(), tmp.end());
    col.insert(col.end(), tmp.begin(), tmp.end());
    row[l + 1] = (int)col.size();
  }
}

void Runtime::build_site_lists() {
  const int N = N_, M = M_;
  std::vector<int> row, col;
  point_lists(h_sxyz_, M, row, col);
  // per panel: the sites for which it is near (transposed lists)
  std::vector<int> trow(N + 1, 0), tcol(std::max<size_t>(1, col.size()), 0);
  for (int l = 0; l < M; ++l)
    for (int e = row[l]; e < row[l + 1]; ++e) trow[col[e] + 1]++;
  for (int j = 0; j < N; ++j) trow[j + 1] += trow[j];
  std::vector<int> fill(trow.begin(), trow.end() - 1);
  for (int l = 0; l < M; ++l)
    for (int e = row[l]; e < row[l + 1]; ++e) tcol[fill[col[e]]++] = l;
  if (col.empty()) col.push_back(0);  // keep a valid allocation
  srow_.upload(row.data(), row.size(), s_);
  scol_.upload(col.data(), col.size(), s_);
  tsrow_.upload(trow.data(), trow.size(), s_);
  tscol_.upload(tcol.data(), tcol.size(), s_);
  sync();
}

// -------------------------------------------------------------- operator
void Runtime::apply(const double *x, double *y, bool f64, bool packed) {
  const int N = N_;
  const bool use64 = f64 || fp64();
  const double *val = (use64 && !fp64()) ? nval64_.p : nval_.p;
  // refinement products are FP64 by request: kept out of the kernel timers
  const bool timed = clock.on;
  if (f64 && !fp64()) clock.on = false;
  if (!packed) launch_pack_strengths(s_, N, ru_.nf, geo_.p, x, src64_.p, src32_.p);
  if (use_tree()) {
    tree_apply(*tree_, s_, use64, ru_.nf, N, geo_.p, src64_.p, src32_.p,
               tgt32_.p, o.kappa, part_.p, clock, floor_r2_);
    launch_finish_slots(s_, N, tree_->d_tslots.p, part_.p, nrow_.p, ncol_.p,
                        val, x, o.eps_in / o.eps_out, y);
  } else {
    hipEvent_t e0 = clock.on ? clock.begin(s_) : nullptr;
    launch_p2p_direct(s_, use64, ru_.nf, N, N, src64_.p, src32_.p, geo_.p,
                      tgt32_.p, o.kappa, p2p_chunks_, part_.p, floor_r2_);
    if (clock.on) clock.end(s_, e0, KernelClock::P2P, (double)N * N * ru_.nf);
    launch_finish(s_, N, p2p_chunks_, part_.p, nrow_.p, ncol_.p, val, x,
                  o.eps_in / o.eps_out, y);
  }
  clock.on = timed;
  ++matvecs_;
}

// ----------------------------------------------------------------- GMRES
// Right-preconditioned restarted GMRES with classical Gram-Schmidt applied
// twice, the true residual recomputed at every restart.  The Arnoldi steps
// run on the device; each step's Hessenberg column is copied to pinned host
// memory and rotated there (Givens).  The host launches the next step
// before it has read the current one's column whenever the residual
// estimate cannot reach the tolerance within the current step, so the
// device never waits for the host: with r the last known residual and rho
// the smallest of the last three reduction ratios, the next step is
// launched early when r rho exceeds the target.  A step launched early past
// convergence only extends the Krylov basis; the update uses the converged
// columns.
void Runtime::krylov_reserve(int n) {
  const int m = o.gmres_restart;
  partial_.reserve((size_t)(m + 2) * ((n + 4095) / 4096 + 1));
  hbuf_.reserve(3 * (size_t)(m + 2));
  ybuf_.reserve((size_t)(m + 2));
  const size_t need = (size_t)m * 3 * (m + 2);
  if (hpin_n_ < need) {
    if (hpin_) PBMP_HIP(hipHostFree(hpin_));
    hpin_ = nullptr;
    hpin_n_ = 0;
    PBMP_HIP(hipHostMalloc((void **)&hpin_, need * sizeof(double), hipHostMallocDefault));
    hpin_n_ = need;
  }
  while ((int)kev_.size() < m) {
    hipEvent_t e;
    PBMP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    kev_.push_back(e);
  }
}

int Runtime::gmres_core(int n, const KOp &op, const KPrec &prec, const KUpdate &update,
                        const double *b, double *x, double *V, double *w, double *z,
                        double *ax, int *iters, bool *ax_valid, const KPrecOp &precop) {
  // ax_valid (may be null): in, ax already holds op(x) for this x (the last
  // residual product of the previous solve, x unchanged since), so the first
  // residual needs no product; out, whether ax holds op(x) on return
  bool have_ax = ax_valid && *ax_valid;
  if (ax_valid) *ax_valid = false;
  const int m = o.gmres_restart;
  const size_t ld = n;
  const size_t stride = 3 * (size_t)(m + 2);
  krylov_reserve(n);
  auto dot_host = [&](const double *a, const double *bb) {
    launch_mdot(s_, n, 1, a, ld, bb, partial_.p, hbuf_.p);
    double h;
    PBMP_HIP(hipMemcpyAsync(&h, hbuf_.p, sizeof(double), hipMemcpyDeviceToHost, s_));
    sync();
    return h;
  };
  const double bnorm = std::sqrt(dot_host(b, b));
  *iters = 0;
  if (bnorm == 0.0) {
    launch_scale(s_, n, 0.0, x, x);
    last_relres_ = 0.0;
    return 0;
  }
  // Mixed precision: restart residuals come from the FP32-far-field product
  // while they keep falling; once one reaches that product's accuracy (a
  // relative residual of kFloor32) or a cycle stalls, they are recomputed
  // with the FP64 product, which turns the restarts into iterative
  // refinement with FP64 residuals.  Before that, a cycle aims no lower
  // than kFloor32: Arnoldi steps beyond it would only solve the FP32
  // system more exactly.
  constexpr double kFloor32 = 1e-6;
  bool refine = false;
  double prev = 0.0;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  double ratio[3] = {0.1, 0.1, 0.1};
  int it = 0;
  while (true) {
    if (!have_ax) op(x, ax, refine);
    have_ax = false;
    launch_xmy(s_, n, b, ax, w);
    double beta = std::sqrt(dot_host(w, w));
    if (!refine && !fp64() && beta / bnorm > o.gmres_tol &&
        ((it > 0 && beta / bnorm > 0.5 * prev) || beta / bnorm <= kFloor32)) {
      refine = true;
      op(x, ax, true);
      launch_xmy(s_, n, b, ax, w);
      beta = std::sqrt(dot_host(w, w));
    }
    last_relres_ = beta / bnorm;
    prev = last_relres_;
    if (last_relres_ <= o.gmres_tol || it >= o.gmres_maxit) {
      if (ax_valid) *ax_valid = true;
      return last_relres_ <= o.gmres_tol ? 0 : PBMP_WGMRES;
    }
    launch_scale(s_, n, 1.0 / beta, w, V);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    // a refinement cycle (FP32 Arnoldi on an FP64 residual) gains at most
    // about kFloor32 per restart, so it aims no lower than that either
    const double target =
        fp64() ? 0.5 * bnorm * o.gmres_tol
        : refine ? std::max(0.5 * bnorm * o.gmres_tol, kFloor32 * beta)
                 : 0.5 * bnorm * std::max(o.gmres_tol, kFloor32);
    const int kmax = std::min(m, o.gmres_maxit - it);
    auto enqueue = [&](int k) {
      if (precop) {
        precop(V + (size_t)k * ld, z, w);
      } else {
        prec(V + (size_t)k * ld, z);
        op(z, w, false);
      }
      // CGS2: h1 = V^T w, w -= V h1, h2 = V^T w, w -= V h2, |w|^2; the
      // totals land in hbuf (h1, h2, |w|^2) for the host
      int nb = launch_mdot_partial(s_, n, k + 1, V, ld, w, partial_.p);
      launch_gemv_sub_p(s_, n, k + 1, V, ld, nb, partial_.p, hbuf_.p, w);
      nb = launch_mdot_partial(s_, n, k + 1, V, ld, w, partial_.p);
      launch_gemv_sub_p(s_, n, k + 1, V, ld, nb, partial_.p, hbuf_.p + (m + 2), w);
      nb = launch_mdot_partial(s_, n, 1, w, ld, w, partial_.p);
      launch_scale_inv_sqrt_p(s_, n, nb, partial_.p, hbuf_.p + 2 * (m + 2), w,
                              V + (size_t)(k + 1) * ld);
      PBMP_HIP(hipMemcpyAsync(hpin_ + k * stride, hbuf_.p, sizeof(double) * stride,
                              hipMemcpyDeviceToHost, s_));
      PBMP_HIP(hipEventRecord(kev_[k], s_));
      ++gmres_iters_;
    };
    enqueue(0);
    int enq = 1, done = 0;
    double last = beta;
    while (true) {
      const double rho = std::min({ratio[0], ratio[1], ratio[2], 1.0});
      if (enq == done + 1 && enq < kmax && last * rho > target) enqueue(enq++);
      PBMP_HIP(hipEventSynchronize(kev_[done]));
      const double *hh = hpin_ + done * stride;
      const int k = done;
      for (int i = 0; i <= k; ++i) H[(size_t)i * m + k] = hh[i] + hh[m + 2 + i];
      const double hn = std::sqrt(hh[2 * (m + 2)]);
      H[(size_t)(k + 1) * m + k] = hn;
      for (int i = 0; i < k; ++i) {
        const double a = H[(size_t)i * m + k], bb = H[(size_t)(i + 1) * m + k];
        H[(size_t)i * m + k] = cs[i] * a + sn[i] * bb;
        H[(size_t)(i + 1) * m + k] = -sn[i] * a + cs[i] * bb;
      }
      const double a = H[(size_t)k * m + k], bb = H[(size_t)(k + 1) * m + k];
      const double den = std::hypot(a, bb);
      cs[k] = den > 0 ? a / den : 1.0;
      sn[k] = den > 0 ? bb / den : 0.0;
      H[(size_t)k * m + k] = den;
      H[(size_t)(k + 1) * m + k] = 0.0;
      g[k + 1] = -sn[k] * g[k];
      g[k] = cs[k] * g[k];
      ++it;
      done = k + 1;
      const double res = std::fabs(g[k + 1]);
      if (last > 0.0) {
        ratio[2] = ratio[1];
        ratio[1] = ratio[0];
        ratio[0] = res / last;
      }
      last = res;
      if (res <= target || hn == 0.0 || done >= kmax) break;
      if (enq == done) enqueue(enq++);
    }
    const int k_done = done;
    for (int i = k_done - 1; i >= 0; --i) {
      double sacc = g[i];
      for (int j = i + 1; j < k_done; ++j) sacc -= H[(size_t)i * m + j] * y[j];
      y[i] = sacc / H[(size_t)i * m + i];
    }
    update(k_done, y.data());
    *iters = it;
  }
}

int Runtime::gmres(const double *b, double *x, bool transpose, int *iters) {
  const int N = N_, n = 2 * N;
  const size_t ld = n;
  KOp op = [&](const double *in, double *out, bool f64) {
    if (transpose) apply_transpose(in, out, f64);
    else apply(in, out, f64);
  };
  KPrec prec = [&](const double *u, double *zz) {
    if (transpose) precond_T(u, zz);
    else launch_precond(s_, N, diag_.p, o.eps_in / o.eps_out, u, zz);
  };
  KUpdate update = [&](int k_done, const double *y) {
    if (transpose) {
      // x += M^{-T} (V y): ax = 0 - V (-y), then the preconditioner
      std::vector<double> ny(y, y + k_done);
      for (double &v : ny) v = -v;
      PBMP_HIP(hipMemcpyAsync(ybuf_.p, ny.data(), sizeof(double) * k_done,
                              hipMemcpyHostToDevice, s_));
      launch_scale(s_, n, 0.0, ax_.p, ax_.p);
      launch_gemv_sub(s_, n, k_done, V_.p, ld, ybuf_.p, ax_.p);
      precond_T(ax_.p, z_.p);
      launch_axpy(s_, n, 1.0, z_.p, x);
      sync();
    } else {
      PBMP_HIP(hipMemcpyAsync(ybuf_.p, y, sizeof(double) * k_done, hipMemcpyHostToDevice,
                              s_));
      launch_update_solution(s_, N, k_done, V_.p, ld, ybuf_.p, diag_.p,
                             o.eps_in / o.eps_out, x);
    }
  };
  // the forward solve of the SCF loop reuses A x_ from the previous solve
  bool *valid = (!transpose && x == x_.p) ? &ax_holds_x_ : nullptr;
  if (!valid) ax_holds_x_ = false;  // ax_ is overwritten
  // forward Arnoldi steps: preconditioner and strength packing in one launch
  KPrecOp precop;
  if (!transpose)
    precop = [&](const double *v, double *zz, double *ww) {
      launch_precond_pack(s_, N, ru_.nf, diag_.p, o.eps_in / o.eps_out, geo_.p, v, zz,
                          src64_.p, src32_.p);
      apply(zz, ww, false, true);
    };
  return gmres_core(n, op, prec, update, b, x, V_.p, w_.p, z_.p, ax_.p, iters, valid, precop);
}

// GMRES for a general operator of size n (right preconditioning, CGS2,
// FP64 refinement as in gmres).  x holds the initial guess.
int Runtime::gmres_generic(int n, const KOp &op, const KPrec &prec, const double *b, double *x,
                           int *iters, bool *ax_valid) {
  const int m = o.gmres_restart;
  const size_t ld = n;
  gV_.reserve((size_t)(m + 1) * n);
  gw_.reserve(n);
  gz_.reserve(n);
  gax_.reserve(n);
  KUpdate update = [&](int k_done, const double *y) {
    // x += M^{-1} (V y)
    std::vector<double> ny(y, y + k_done);
    for (double &v : ny) v = -v;
    PBMP_HIP(hipMemcpyAsync(ybuf_.p, ny.data(), sizeof(double) * k_done, hipMemcpyHostToDevice,
                            s_));
    launch_scale(s_, n, 0.0, gax_.p, gax_.p);
    launch_gemv_sub(s_, n, k_done, gV_.p, ld, ybuf_.p, gax_.p);
    prec(gax_.p, gz_.p);
    launch_axpy(s_, n, 1.0, gz_.p, x);
    sync();
  };
  return gmres_core(n, op, prec, update, b, x, gV_.p, gw_.p, gz_.p, gax_.p, iters, ax_valid,
                    KPrecOp());
}

// ------------------------------------------------------------- readout
void Runtime::readout(const double *x, bool full, double *out) {
  launch_pack_strengths(s_, N_, ru_.nf, geo_.p, x, src64_.p, src32_.p);
  launch_readout(s_, fp64(), full, N_, M_, src64_.p, src32_.p, geo_.p, verts_.p,
                 tri_.p, ru_, x, sxyz_.p, srow_.p, scol_.p, ro_chunks_, rpart_.p,
                 out);
}

// ----------------------------------------------------------------- SCF
int Runtime::scf(bool solvent, double *mu, int *gm_warn) {
  const int M = M_, N = N_;
  const auto t_start = clk::now();
  const double dbye = debye_per_e_ang();
  // warm start: keep the previous solve's dipoles and surface solution
  const bool warm = o.warm_start && warm_ok_;
  if (!warm) PBMP_HIP(hipMemsetAsync(mu, 0, sizeof(double) * 3 * M, s_));
  launch_perm_field(s_, M, sxyz_.p, sq_.p, sd_.p, sQ_.p, sgroup_.p, o.eps_in, Eperm_.p);
  if (solvent) {
    PBMP_HIP(hipMemsetAsync(b_.p, 0, sizeof(double) * 2 * N, s_));
    if (!warm) {
      PBMP_HIP(hipMemsetAsync(x_.p, 0, sizeof(double) * 2 * N, s_));
      if (outer_) PBMP_HIP(hipMemsetAsync(sX_.p, 0, sizeof(double) * sX_.n, s_));
      ax_holds_x_ = gax_holds_x_ = false;
    }
  }
  for (int it = 1; it <= o.scf_maxit; ++it) {
    int gi = 0;
    if (solvent) {
      launch_scale(s_, 3 * M, 1.0, sd_.p, p_.p);
      launch_axpy(s_, 3 * M, 1.0, mu, p_.p);
      launch_rhs(s_, fp64(), N, M, geo_.p, sxyz_.p, sq_.p, p_.p, sQ_.p, o.eps_in, b_.p);
      auto tm = clk::now();
      const int rc = outer_ ? gmres_stern(b_.p, x_.p, &gi) : gmres(b_.p, x_.p, false, &gi);
      t_matvec_ms_ += ms_since(tm);
      if (rc > 0) *gm_warn = rc;
      readout(x_.p, false, reac_.p);
    }
    launch_induced(s_, false, M, sxyz_.p, mu, salpha_.p, o.thole_a, o.eps_in, Eind_.p);
    launch_scf_update(s_, M, salpha_.p, Eperm_.p, Eind_.p, solvent ? reac_.p : nullptr,
                      4, o.scf_omega, mu, dmu2_.p);
    double d2;
    PBMP_HIP(hipMemcpyAsync(&d2, dmu2_.p, sizeof(double), hipMemcpyDeviceToHost, s_));
    sync();
    const double rms = std::sqrt(d2 / M) * dbye;
    if (o.verbose)
      std::fprintf(stderr, "pbmp solve: %s iteration %d gmres %d rms change %.3e D %.1f s\n",
                   solvent ? "dissolved" : "vacuum", it, gi, rms, 1e-3 * ms_since(t_start));
    if (!std::isfinite(rms)) throw Error(PBMP_WSCF, "induced dipoles diverged");
    if (rms < o.scf_tol_debye) return it;
  }
  return -o.scf_maxit;
}

int Runtime::solve(pbmp_result *r) {
  PBMP_REQUIRE(N_ > 0 && M_ > 0, PBMP_ESTATE, "set_mesh and set_sites must precede solve");
  PBMP_REQUIRE(r != nullptr, PBMP_EARG, "null result");
  auto t0 = clk::now();
  gmres_iters_ = 0;
  matvecs_ = 0;
  t_matvec_ms_ = 0.0;
  int warn = 0, gm_warn = 0;
  int it_v = scf(false, mu_v_.p, &gm_warn);
  int it_d = scf(true, mu_d_.p, &gm_warn);
  if (it_v < 0 || it_d < 0) warn = PBMP_WSCF;
  if (gm_warn && !warn) warn = gm_warn;
  // energy (eq. energy_multipole_polarizable with d in place of p; the
  // permanent-permanent terms cancel between the two states)
  readout(x_.p, true, reac_.p);
  launch_scale(s_, 3 * M_, 1.0, mu_d_.p, p_.p);
  launch_axpy(s_, 3 * M_, -1.0, mu_v_.p, p_.p);
  launch_induced(s_, true, M_, sxyz_.p, p_.p, salpha_.p, o.thole_a, o.eps_in, ind_.p);
  launch_energy(s_, M_, sq_.p, sd_.p, sQ_.p, reac_.p, ind_.p, e_.p);
  // vacuum Coulomb energy (the same energy form with phi = potential of
  // the other sites' permanent multipoles and vacuum induced dipoles)
  launch_perm_potential(s_, M_, sxyz_.p, sq_.p, sd_.p, sQ_.p, o.eps_in, vac_perm_.p);
  launch_induced(s_, true, M_, sxyz_.p, mu_v_.p, salpha_.p, o.thole_a, o.eps_in, vac_ind_.p);
  launch_energy(s_, M_, sq_.p, sd_.p, sQ_.p, vac_perm_.p, vac_ind_.p, e_.p + 2);
  launch_total_dipole(s_, M_, sxyz_.p, sq_.p, sd_.p, mu_v_.p, mu_d_.p, e_.p + 4);
  double e[10];
  PBMP_HIP(hipMemcpyAsync(e, e_.p, sizeof(e), hipMemcpyDeviceToHost, s_));
  sync();
  const double C = coulomb_kcal();
  r->dG_solv_kcal = C * e[0];
  r->dG_pol_kcal = C * e[1];
  r->dG_kcal = C * (e[0] + e[1]);
  r->G_vac_kcal = C * (e[2] + e[3]);
  last_dG_ = r->dG_kcal;
  last_Gvac_ = r->G_vac_kcal;
  for (int c = 0; c < 3; ++c) {
    r->dipole_vac_debye[c] = debye_per_e_ang() * e[4 + c];
    r->dipole_diss_debye[c] = debye_per_e_ang() * e[7 + c];
  }
  warm_ok_ = true;
  r->scf_iters = std::abs(it_d);
  r->scf_iters_vac = std::abs(it_v);
  r->gmres_iters_total = gmres_iters_;
  r->matvecs = matvecs_;
  r->final_relres = last_relres_;
  r->t_matvec_ms = t_matvec_ms_;
  r->t_setup_ms = setup_reported_ ? 0.0 : t_setup_ms_;
  setup_reported_ = true;
  // outputs in user order / units
  const int w = r->where;
  PBMP_REQUIRE(w == PBMP_HOST || w == PBMP_DEVICE, PBMP_EARG, "bad result.where");
  if (r->phi || r->dphidn) {
    // physical: 4 pi times the integral-equation normalisation
    launch_permute(s_, N_, 2, d_perm_.p, x_.p, io_a_.p, false);
    launch_scale(s_, 2 * N_, 4.0 * M_PI, io_a_.p, io_a_.p);
    auto put = [&](double *dst, const double *src) {
      if (!dst) return;
      PBMP_HIP(hipMemcpyAsync(dst, src, sizeof(double) * N_,
                              w == PBMP_DEVICE ? hipMemcpyDeviceToDevice
                                               : hipMemcpyDeviceToHost, s_));
    };
    put(r->phi, io_a_.p);
    put(r->dphidn, io_a_.p + N_);
  }
  auto put3 = [&](double *dst, const double *src) {
    if (!dst) return;
    PBMP_HIP(hipMemcpyAsync(dst, src, sizeof(double) * 3 * M_,
                            w == PBMP_DEVICE ? hipMemcpyDeviceToDevice
                                             : hipMemcpyDeviceToHost, s_));
  };
  put3(r->mu_diss, mu_d_.p);
  put3(r->mu_vac, mu_v_.p);
  sync();
  solved_ = true;
  r->t_solve_ms = ms_since(t0);
  return warn;
}

// ---------------------------------------------------- user-order helpers
void Runtime::to_internal(const double *user, double *dev, int blocks, int where) {
  const size_t n = (size_t)N_ * blocks;
  PBMP_REQUIRE(user != nullptr, PBMP_EARG, "null input");
  PBMP_HIP(hipMemcpyAsync(tmp_.p, user, sizeof(double) * n,
                          where == PBMP_DEVICE ? hipMemcpyDeviceToDevice
                                               : hipMemcpyHostToDevice, s_));
  launch_permute(s_, N_, blocks, d_perm_.p, tmp_.p, dev, true);
}

void Runtime::to_user(const double *dev, double *user, int blocks, int where) {
  const size_t n = (size_t)N_ * blocks;
  PBMP_REQUIRE(user != nullptr, PBMP_EARG, "null output");
  launch_permute(s_, N_, blocks, d_perm_.p, dev, tmp_.p, false);
  PBMP_HIP(hipMemcpyAsync(user, tmp_.p, sizeof(double) * n,
                          where == PBMP_DEVICE ? hipMemcpyDeviceToDevice
                                               : hipMemcpyDeviceToHost, s_));
  sync();
}

void Runtime::matvec_user(const double *x, double *y, int transpose, int where) {
  PBMP_REQUIRE(N_ > 0, PBMP_ESTATE, "no mesh");
  PBMP_REQUIRE(where == PBMP_HOST || where == PBMP_DEVICE, PBMP_EARG, "bad where");
  if (outer_) {
    PBMP_REQUIRE(!transpose, PBMP_ESTATE, "no transposed product with a Stern layer");
    stern_matvec_user(x, y, where);
    return;
  }
  to_internal(x, io_a_.p, 2, where);
  auto t0 = clk::now();
  if (transpose) apply_transpose(io_a_.p, io_b_.p);
  else apply(io_a_.p, io_b_.p);
  if (clock.on) {
    sync();
    clock.matvec_ms += ms_since(t0);
    clock.matvec_calls += 1;
  }
  to_user(io_b_.p, y, 2, where);
}

void Runtime::rhs_user(const double *p, double *f, int where) {
  PBMP_REQUIRE(N_ > 0 && M_ > 0, PBMP_ESTATE, "no mesh or sites");
  PBMP_REQUIRE(p != nullptr && f != nullptr, PBMP_EARG, "null pointer");
  PBMP_HIP(hipMemcpyAsync(p_.p, p, sizeof(double) * 3 * M_,
                          where == PBMP_DEVICE ? hipMemcpyDeviceToDevice
                                               : hipMemcpyHostToDevice, s_));
  launch_rhs(s_, fp64(), N_, M_, geo_.p, sxyz_.p, sq_.p, p_.p, sQ_.p, o.eps_in, io_b_.p);
  to_user(io_b_.p, f, 1, where);
}

void Runtime::site_fields_user(const double *x, double *out, int where) {
  PBMP_REQUIRE(N_ > 0 && M_ > 0, PBMP_ESTATE, "no mesh or sites");
  PBMP_REQUIRE(out != nullptr, PBMP_EARG, "null output");
  to_internal(x, io_a_.p, 2, where);
  readout(io_a_.p, true, reac_.p);
  PBMP_HIP(hipMemcpyAsync(out, reac_.p, sizeof(double) * 10 * M_,
                          where == PBMP_DEVICE ? hipMemcpyDeviceToDevice
                                               : hipMemcpyDeviceToHost, s_));
  sync();
}

}  // namespace pbmp
