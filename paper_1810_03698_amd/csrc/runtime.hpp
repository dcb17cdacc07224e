// Context of the pbmp library: device-resident mesh, site and solver state.
#pragma once

#include <chrono>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "tree.hpp"

struct pbmp_ctx;

namespace pbmp {

// Accumulated device time per kernel class, when enabled.  Each timed
// launch is bracketed by two HIP events on the launch stream; the events are
// only resolved (synchronised and summed) when the totals are read, so the
// accounting does not serialise the stream.
struct KernelClock {
  enum Kind { P2P = 0, M2P = 1, P2M = 2 };
  bool on = false;
  double p2p_ms = 0, m2p_ms = 0, p2m_ms = 0, near_ms = 0, matvec_ms = 0;
  long p2p_launches = 0, m2p_launches = 0, matvec_calls = 0;
  double p2p_pairs = 0, m2p_pairs = 0;  // executed interactions
  struct Pending {
    hipEvent_t a, b;
    int kind;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t begin(hipStream_t s);
  void end(hipStream_t s, hipEvent_t a, int kind, double pairs);
  void resolve();
  void reset();
  ~KernelClock();
};

class Runtime {
 public:
  explicit Runtime(const pbmp_options &o);
  ~Runtime();

  void set_mesh(int64_t nv, const double *verts, int64_t nt, const int32_t *tris,
                int where);
  void set_sites(int64_t m, const double *xyz, const double *q, const double *d,
                 const double *Q9, const double *alpha, const int32_t *group,
                 int where);
  int solve(pbmp_result *r);
  void matvec_user(const double *x, double *y, int transpose, int where);
  void rhs_user(const double *p, double *f, int where);
  void site_fields_user(const double *x, double *out, int where);
  // site_fields_user with device pointers and its work memory in the static
  // scratch (k_static.hip): no device allocation
  void site_fields_noalloc(const double *x, double *out);
  void tree_export(int64_t counts[4], int32_t *perm, int32_t *box_range, int32_t *box_level,
                   double *box_centre, double *box_radius, int32_t *leaf_box,
                   int32_t *m2p_ptr, int32_t *m2p_box, int32_t *p2p_ptr,
                   int32_t *p2p_box) const;
  // solver settings between solves (discretisation fields must not change)
  void set_options(const pbmp_options &n);
  // ion-exclusion layer: outer surface G2 and its permittivity (nt = 0 removes it)
  void set_stern(int64_t nv, const double *verts, int64_t nt, const int32_t *tris,
                 double eps_stern, int where);
  bool has_stern() const { return (bool)outer_; }
  int backward(double dGbar, double *g_xyz, double *g_q, double *g_d,
               double *g_Q, double *g_verts, int where);
  // the last solve's solvation energy and vacuum Coulomb energy (binding.cpp)
  void binding_terms(double *dG, double *G_vac) const;
  // d dG / dt for a rigid translation t of the sites [first_ligand, m) and
  // of the vertices those sites own (binding.cpp)
  int ligand_translation_gradient(int64_t first_ligand, const double *radii, int where,
                                  double g_t[3], int64_t *n_ligand_vertices);

  std::string err;
  KernelClock clock;
  pbmp_options o;

 private:
  hipStream_t s_ = nullptr;
  bool own_stream_ = false;
  RuleArgs ru_{};
  bool fp64() const { return o.precision == PBMP_FP64; }
  bool use_tree() const { return tree_active_; }

  // ---- mesh (internal panel order) ----
  int N_ = 0, Nv_ = 0;
  std::vector<int> perm_;  // internal -> user panel index
  Dbuf<int> d_perm_;
  Dbuf<uint64_t> keys_;  // Morton keys in internal order
  Dbuf<double> verts_;
  Dbuf<int> tri_;
  Dbuf<double> geo_, src64_;
  Dbuf<float> src32_, tgt32_;
  std::vector<double> h_geo_;
  std::vector<double> h_verts_;
  std::vector<int> h_tri_;  // internal order
  Dbuf<int> nrow_, ncol_;
  int nnz_ = 0;
  Dbuf<double> nval_, nval64_, diag_;  // nval64_: FP64-far-field corrections (mixed mode)
  Dbuf<int> trow_, tcol_;  // transposed near structure (entry ids)
  Dbuf<int> tent_;
  bool tree_active_ = false;
  bool floor_r2_ = true;  // FP32 distance cut-off needed (one-node rule, tiny panels)
  std::unique_ptr<Tree> tree_;

  // ---- sites ----
  int M_ = 0;
  Dbuf<double> sxyz_, sq_, sd_, sQ_, salpha_;
  Dbuf<int> sgroup_, srow_, scol_, tsrow_, tscol_;
  std::vector<double> h_sxyz_;

  // ---- work ----
  Dbuf<double> part_, rpart_;
  int p2p_chunks_ = 1, ro_chunks_ = 1;
  Dbuf<double> V_, w_, z_, ax_, b_, x_, hbuf_, partial_, ybuf_, tmp_;
  Dbuf<double> mu_d_, mu_v_, Eperm_, Eind_, reac_, ind_, p_, f_, dmu2_, e_;
  Dbuf<double> io_a_, io_b_;  // permutation staging
  Dbuf<double> vac_perm_, vac_ind_;  // vacuum-state potential data [10M]
  bool solved_ = false;
  double last_dG_ = 0.0, last_Gvac_ = 0.0;  // of the last solve
  bool warm_ok_ = false;  // x_, mu_d_, mu_v_ hold a previous solve of this mesh and site count
  int gmres_iters_ = 0, matvecs_ = 0;
  double last_relres_ = 0.0;
  double t_matvec_ms_ = 0.0;
  double t_setup_ms_ = 0.0;
  bool setup_reported_ = false;

  void sync();
  void build_near_lists();
  void near_values();
  void build_site_lists();
  void alloc_work();
  // y = A x (internal order, device)
  // y = A x (transpose: A^T x); f64 forces the FP64 far field in mixed mode
  // packed: the strengths of x are already in the source records
  void apply(const double *x, double *y, bool f64 = false, bool packed = false);
  void apply_transpose(const double *x, double *y, bool f64 = false);
  void precond_T(const double *u, double *z);
  // GMRES on A x = b (device, internal order), x holds the initial guess.
  int gmres(const double *b, double *x, bool transpose, int *iters);
  // readout at the sites for surface solution x (internal): out [M*nout]
  void readout(const double *x, bool full, double *out);
  // induced-dipole loop; solvent=false: vacuum.  Returns iterations (<0:
  // not converged).
  int scf(bool solvent, double *mu, int *gm_warn);
  void to_internal(const double *user, double *dev, int blocks, int where);
  void to_user(const double *dev, double *user, int blocks, int where);
  // ---- Stern layer ----
  std::unique_ptr<Runtime> outer_;  // G2 with eps_in = eps_stern, its own kappa
  double kappa_ext_ = 0.0, eps_out_ext_ = 0.0, eps_stern_ = 0.0;
  int Mp_ = 0, p_chunks_ = 1;  // probe points: layer potentials of this surface there
  Dbuf<double> pxyz_, ppart_, pout_;
  Dbuf<int> prow_, pcol_;
  Dbuf<double> sX_, sB_, sY_, sT_;       // [phi1, q1, phi2, q2] work
  Dbuf<double> gV_, gw_, gz_, gax_;      // general GMRES work
  void point_lists(const std::vector<double> &pts, int M, std::vector<int> &row,
                   std::vector<int> &col) const;
  void set_probe(int M, const std::vector<double> &pts);
  void probe(const double *x, bool f64, double *out4);
  void apply_stern(const double *X, double *Y, bool f64);
  void precond_stern(const double *v, double *z);
  int gmres_stern(const double *b, double *x, int *iters);
  void stern_matvec_user(const double *x, double *y, int where);
  using KOp = std::function<void(const double *, double *, bool)>;  // y = A x (f64 flag)
  using KPrec = std::function<void(const double *, double *)>;      // z = M^{-1} v
  using KUpdate = std::function<void(int, const double *)>;         // x += M^{-1} V y
  using KPrecOp = std::function<void(const double *, double *, double *)>;  // z = M^{-1} v, w = A z
  int gmres_generic(int n, const KOp &op, const KPrec &prec, const double *b, double *x,
                    int *iters, bool *ax_valid = nullptr);
  int gmres_core(int n, const KOp &op, const KPrec &prec, const KUpdate &update,
                 const double *b, double *x, double *V, double *w, double *z, double *ax,
                 int *iters, bool *ax_valid, const KPrecOp &precop);
  // ax_ = A x_ (gax_ = A sX_ for the layer system): the residual product of
  // the last solve, valid while neither x nor the operator changed
  bool ax_holds_x_ = false, gax_holds_x_ = false;
  // adjoint multipliers of the last backward (vacuum and dissolved dipole
  // loops, surface) for warm-started backward calls
  Dbuf<double> adj_lv_, adj_ld_, adj_lx_;
  bool adj_ok_ = false;
  double adj_bar_ = 0.0;
  int adj_M_ = 0;
  void krylov_reserve(int n);
  double *hpin_ = nullptr;           // pinned Hessenberg columns [m][3(m+2)]
  size_t hpin_n_ = 0;
  std::vector<hipEvent_t> kev_;      // one per Arnoldi step of a cycle
  friend struct Backward;
};

// Physical constants (CODATA 2018; e, N_A exact)
double coulomb_kcal();      // e^2 N_A / (4 pi eps0 1 A) in kcal/mol
double debye_per_e_ang();   // 1 e*A in Debye

}  // namespace pbmp

struct pbmp_ctx {
  std::unique_ptr<pbmp::Runtime> rt;
  std::string err;
};
