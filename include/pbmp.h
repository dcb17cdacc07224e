/*
 * pbmp -- boundary-integral Poisson-Boltzmann solver with polarisable point
 * multipoles, on one AMD Instinct MI355X (gfx950).
 *
 * The method (Cooper, "A boundary-integral approach for the Poisson-Boltzmann
 * equation with polarizable force fields"):
 *   - molecule = closed triangulated surface Gamma (normal pointing out of the
 *     molecule), dielectric eps_in inside, eps_out and inverse Debye length
 *     kappa outside (eq. pde);
 *   - surface unknowns phi and dphi/dn, piecewise constant on flat panels,
 *     collocated at panel centroids, from the Yoon-Lenhoff system
 *     (eq. integral_eq) solved by GMRES, whose matrix-vector product is an
 *     N-body sum over far-field Gauss nodes, optionally accelerated by a
 *     Cartesian-Taylor treecode (section "The treecode algorithm");
 *   - point multipoles q, d, Q (Buckingham, traceless) with isotropic
 *     polarisability alpha enter through the right-hand side
 *     (eq. rhs_multipole); induced dipoles mu = alpha E are found by the
 *     relaxed self-consistent loop (section "Self-consistent induced field");
 *   - solvation energy from eq. energy_multipole_polarizable.
 *
 * Conventions for every call:
 *   - Units: Angstrom, elementary charge e, kcal/mol.  phi in e/A (physical,
 *     i.e. 4*pi times the integral-equation normalisation G = 1/(4 pi r)),
 *     dphi/dn in e/A^2, dipoles in e*A, quadrupoles in e*A^2, alpha in A^3.
 *   - `where` selects the address space of every caller pointer passed to
 *     that call: PBMP_HOST (pageable or pinned host memory) or PBMP_DEVICE
 *     (device memory of the current HIP device).  The library copies inputs
 *     and writes outputs; the caller keeps ownership of its buffers.
 *   - Return value 0 = success.  Negative = error, outputs undefined:
 *       PBMP_EARG  -1 bad argument or option out of range
 *       PBMP_EMESH -2 mesh not closed / not 2-manifold / inconsistently
 *                     oriented / inward / degenerate panel (area <= 1e-12 A^2)
 *       PBMP_ESITE -3 a site lies outside the surface (winding number < 0.5)
 *       PBMP_EHIP  -4 HIP runtime error
 *       PBMP_ENOMEM -5 device allocation failed
 *       PBMP_ESTATE -6 call out of order (e.g. solve before set_mesh)
 *     Positive = warning, outputs filled from the best iterate:
 *       PBMP_WGMRES +1 GMRES not converged, PBMP_WSCF +2 SCF not converged.
 *     pbmp_last_error() returns a message for the last failing call.
 *   - A context is not thread safe; use one per host thread.  All device
 *     work is issued on the context's stream (options.hip_stream, or a
 *     stream the library creates when that is NULL); calls return after
 *     their results are complete.
 */
#ifndef PBMP_H
#define PBMP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PBMP_HOST 0
#define PBMP_DEVICE 1

#define PBMP_OK 0
#define PBMP_EARG (-1)
#define PBMP_EMESH (-2)
#define PBMP_ESITE (-3)
#define PBMP_EHIP (-4)
#define PBMP_ENOMEM (-5)
#define PBMP_ESTATE (-6)
#define PBMP_WGMRES 1
#define PBMP_WSCF 2

#define PBMP_MODE_DIRECT 0
#define PBMP_MODE_TREECODE 1
#define PBMP_MODE_AUTO 2 /* treecode above 20000 panels */

#define PBMP_FP64 0
#define PBMP_MIXED 1 /* FP32 far field (P2P, M2P, far readout, RHS pair
                        terms) with FP64 accumulation; FP64 near/self
                        integrals, Krylov vectors, SCF and energy.  GMRES
                        tolerances below 1e-6 are met by iterative
                        refinement: restart residuals from the FP64
                        operator, Arnoldi steps on the FP32 one */

typedef struct pbmp_options {
  double eps_in;        /* solute dielectric constant (eq. pde), > 0        */
  double eps_out;       /* solvent dielectric constant, > 0                 */
  double kappa;         /* inverse Debye length [1/A], >= 0                 */
  int gauss_far;        /* far-field nodes per panel: 1 or 3                */
  double near_eta;      /* near-singular iff |c_i - c_j| < eta sqrt(A_i)    */
  int mode;             /* PBMP_MODE_*                                      */
  double theta;         /* treecode MAC: R_box < theta * distance, (0, 1)   */
  int order_P;          /* Taylor order of the treecode, 1..6               */
  int leaf_panels;      /* max panels per tree leaf, >= 8                   */
  int gmres_restart;    /* Krylov dimension before restart, 1..200          */
  double gmres_tol;     /* stop when |b - A x| <= tol |b|                   */
  int gmres_maxit;      /* max GMRES iterations per solve                   */
  double scf_tol_debye; /* stop when RMS |mu_new - mu| (Debye) < tol        */
  double scf_omega;     /* relaxation mu <- (1-w) mu + w alpha E, (0, 2)    */
  int scf_maxit;        /* max induced-dipole iterations per state          */
  double thole_a;       /* Thole damping parameter, >= 0                    */
  int precision;        /* PBMP_FP64 or PBMP_MIXED                          */
  void *hip_stream;     /* hipStream_t to run on, or NULL                   */
  int warm_start;       /* nonzero: a solve starts GMRES and both induced-
                           dipole loops from the previous solve's surface
                           solution and dipoles (same mesh and site count;
                           sites may have moved), e.g. for nearby geometries
                           in finite differences or dynamics, and a backward
                           starts its transposed loops from the previous
                           backward's multipliers; 0: from zero */
  int verbose;          /* nonzero: one line on stderr per induced-dipole
                           iteration of a solve or backward (state,
                           iteration, GMRES steps, change, seconds since the
                           call began), as progress for long solves       */
} pbmp_options;

typedef struct pbmp_ctx pbmp_ctx;

typedef struct pbmp_result {
  /* caller-allocated outputs in the address space `where`; any may be NULL */
  int where;
  double *phi;     /* [nt] surface potential (inside trace), e/A           */
  double *dphidn;  /* [nt] normal derivative, e/A^2                        */
  double *mu_diss; /* [3m] induced dipoles, dissolved state, e*A           */
  double *mu_vac;  /* [3m] induced dipoles, vacuum state, e*A              */
  /* written by the library */
  double dG_kcal;          /* solvation energy, kcal/mol                   */
  double dG_solv_kcal;     /* reaction-potential part of dG               */
  double dG_pol_kcal;      /* induced-dipole Coulomb part of dG            */
  int scf_iters;           /* dissolved-state SCF iterations               */
  int scf_iters_vac;       /* vacuum-state SCF iterations                  */
  int gmres_iters_total;   /* Arnoldi steps over all solves                */
  int matvecs;             /* operator applications over all solves        */
  double final_relres;     /* true relative residual of the last solve     */
  double t_setup_ms;       /* mesh/site preparation (first solve only)     */
  double t_solve_ms;       /* wall time of pbmp_solve                      */
  double t_matvec_ms;      /* time spent in operator applications          */
  double G_vac_kcal;       /* Coulomb energy of the vacuum state: half the
                              sum over sites of q phi + d.grad phi +
                              (1/6) Q:grad grad phi, phi from the other
                              sites' permanent multipoles (unmasked) and
                              vacuum induced dipoles (eq. energy_multipole_
                              polarizable); G_AB - G_A - G_B of three solves
                              is the vacuum binding energy (eq. bind_vac)  */
  double dipole_vac_debye[3];  /* total dipole of the molecule, vacuum state:
                                  sum of q (r - o) + d + mu_vac over sites,
                                  o = mean site position, Debye (the
                                  diagnostic of Table "dipole")           */
  double dipole_diss_debye[3]; /* the same with mu_diss (dissolved state)  */
} pbmp_result;

/* Fill `o` with defaults: eps 1/80, kappa 0.125, 3 far nodes, eta 2,
 * AUTO mode, theta 0.5, P 4, leaf 300, GMRES(50) tol 1e-6 maxit 1000,
 * SCF tol 1e-6 D, omega 0.7, maxit 200, Thole a 0.39, MIXED, NULL stream,
 * no warm start, not verbose. */
void pbmp_default_options(pbmp_options *o);

/* Create a context on the current HIP device for one dielectric problem of
 * the method (section "The boundary integral formulation", eq. pde: eps_in
 * inside the surface, eps_out and kappa outside) and its discretisation
 * (section "The boundary element method": far and near rules; section
 * "The treecode algorithm": theta, order, leaf size; GMRES and the
 * self-consistent loop of section "Self-consistent induced field").
 * Validates the options (PBMP_EARG on a value out of range, before any
 * device call).  *out receives the context. */
int pbmp_create(const pbmp_options *o, pbmp_ctx **out);

/* Change the solver settings of an existing context between solves (the
 * GMRES and self-consistent-loop settings of sections "The boundary element
 * method" and "Self-consistent induced field", and the precision):
 * gmres_restart, gmres_tol, gmres_maxit, scf_tol_debye, scf_omega,
 * scf_maxit, warm_start, verbose and precision are taken from *o (range-checked as
 * in pbmp_create); every other field must equal the context's (PBMP_EARG
 * otherwise: the discretisation is fixed at creation).  A precision change
 * keeps the last solution, so a backward may run at another precision than
 * the solve it differentiates (e.g. an FP64 state with mixed-precision
 * adjoint solves, whose FP64 refinement keeps them at the GMRES tolerance);
 * not available with a Stern layer (PBMP_EARG). */
int pbmp_set_options(pbmp_ctx *c, const pbmp_options *o);

/* Set the surface mesh: nv vertices [nv*3] (x,y,z per vertex, row-major),
 * nt triangles [nt*3] of vertex indices, counter-clockwise seen from the
 * solvent (section "The boundary integral formulation": n points out of the
 * molecule).  The library copies both arrays, checks that the mesh is
 * closed, 2-manifold, consistently oriented with positive enclosed volume
 * and that every panel area exceeds 1e-12 A^2 (PBMP_EMESH otherwise), and
 * prepares panel geometry, near-singular lists and the tree.  Invalidates
 * previously set sites' surface data and any previous solution. */
int pbmp_set_mesh(pbmp_ctx *c, int64_t nv, const double *verts, int64_t nt,
                  const int32_t *tris, int where);

/* Set m point-multipole sites (section "The implicit-solvent model with
 * polarizable point multipoles"): positions xyz [3m], charges q [m],
 * permanent dipoles d [3m], quadrupoles Q9 [9m] (full row-major 3x3 per
 * site, Buckingham convention of eq. pot_multipole: symmetric and traceless
 * to 1e-10 |Q|, else PBMP_EARG), polarisabilities alpha [m] (>= 0) and
 * polarisation groups group [m] (NULL: every site its own group; permanent
 * fields between sites of one group are excluded from the polarising field).
 * Requires a mesh; every site must lie inside it (PBMP_ESITE). */
int pbmp_set_sites(pbmp_ctx *c, int64_t m, const double *xyz, const double *q,
                   const double *d, const double *Q9, const double *alpha,
                   const int32_t *group, int where);

/* Solve the vacuum and dissolved induced-dipole loops and the solvation
 * energy (eq. energy_general, evaluated with eq.
 * energy_multipole_polarizable).  Writes the outputs named in r. */
int pbmp_solve(pbmp_ctx *c, pbmp_result *r);

/* One application of the boundary-integral operator (eq. integral_eq):
 * y = A x with x = [phi; dphi] in integral-equation normalisation
 * ([2nt], panel order of pbmp_set_mesh), y [2nt].  transpose != 0 applies
 * A^T: in direct mode the transposed entries, in treecode mode the exact
 * transpose of the treecode product (the same lists and expansions).
 * Uses the context's mode and precision. */
int pbmp_matvec(pbmp_ctx *c, const double *x, double *y, int transpose,
                int where);

/* Right-hand side of eq. integral_eq for total dipoles p_total [3m]
 * (p = d + mu): f [nt] = multipole potential at the centroids / (4 pi
 * eps_in) (eq. rhs_multipole), integral-equation normalisation. */
int pbmp_rhs(pbmp_ctx *c, const double *p_total, double *f, int where);

/* Reaction potential data at the sites for a surface solution x [2nt]
 * (eq. pot_solvent, eq. Efield_solv, eq. ddphi): out [10m] per site
 * phi, dphi/dx, dphi/dy, dphi/dz, xx, xy, xz, yy, yz, zz, physical units. */
int pbmp_site_fields(pbmp_ctx *c, const double *x, double *out, int where);

/* pbmp_site_fields for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same values, with no device allocation, no free and no
 * allocating library call.  x [2nt] and out [10m] are device pointers (the
 * caller's panel and site order, as pbmp_site_fields).  The work memory (x in
 * the internal panel order and the readout's per-chunk partial sums,
 * 8 (2 nt + 10 m nchunk) bytes) lives in one static device buffer of 32 MiB
 * per GPU that the library holds until the process ends; its address is
 * looked up when a context is created.  PBMP_EARG when 8 (2 nt + 10 m) bytes
 * exceed 32 MiB (fewer partial-sum chunks are used when the full count does
 * not fit); PBMP_ESTATE without mesh and sites or with a Stern layer.  Every
 * call on one GPU uses the same buffer, which keeps the last call's
 * contents (every value a call reads it writes first): calls that overlap
 * on one GPU, from any contexts or threads, race. */
int pbmp_site_fields_noalloc(pbmp_ctx *c, const double *x, double *out);

/* Gradient of dG_bar * dG (eq. energy_multipole_polarizable, through the
 * adjoint of eq. integral_eq and of the self-consistent loop) with respect
 * to site positions g_xyz [3m],
 * charges g_q [m], dipoles g_d [3m], quadrupole entries g_Q9 [9m] (the nine
 * entries taken as independent, as they enter eq. rhs_multipole and eq.
 * energy_multipole_polarizable) and vertex positions g_verts [3nv], by the
 * adjoint of the converged solve: relaxed transposed induced-dipole loops,
 * GMRES on the transposed operator, and the explicit derivatives of every
 * pair term (operator entries including near-singular and singular panels,
 * right-hand side, readout, Coulomb and Thole interactions).  Near/far
 * decisions and lists are held fixed.  The transposed solves use the
 * context's GMRES tolerance and the transposed loops stop at a relative
 * change of a tenth of it (clamped to [1e-11, 1e-7]); pbmp_set_options may
 * loosen it for the backward after a tight forward solve.  Needs a successful pbmp_solve with
 * unchanged inputs (PBMP_ESTATE otherwise).  Any output may be NULL
 * (skipped).  In treecode mode the transposed solves use the exact
 * transpose of the treecode product, so site gradients are those of the
 * treecode energy, and the far-field operator entries are differentiated
 * with the same lists and expansions (direct pairs; expansions
 * differentiated in the target; local expansions differentiated in the
 * source nodes), so vertex gradients are those of the treecode energy with
 * the expansion centres held fixed, at the cost of a few products.
 * Returns +1/+2 when an adjoint solve did not converge. */
int pbmp_backward(pbmp_ctx *c, double dG_bar, double *g_xyz, double *g_q,
                  double *g_d, double *g_Q9, double *g_verts, int where);

/* Device-time accounting of the operator kernels, measured with HIP events
 * on the context's stream around each launch (adds one event
 * synchronisation per launch while enabled).  mode 1: reset and enable,
 * 0: disable, -1: leave as is.  *out receives the totals since the last
 * reset: milliseconds in the far-field P2P, M2P and P2M kernels and in
 * whole pbmp_matvec calls, launch counts, and the interactions executed
 * (P2P: target x far-field node pairs; M2P: target x box pairs). */
typedef struct pbmp_kstats {
  double p2p_ms, m2p_ms, p2m_ms, matvec_ms;
  int64_t p2p_launches, m2p_launches, matvec_calls;
  double p2p_pairs, m2p_pairs;
} pbmp_kstats;
int pbmp_kernel_stats(pbmp_ctx *c, int mode, pbmp_kstats *out);

/* Ion-exclusion (Stern) layer (section "Spherical cavity": the verification
 * case surrounds the cavity by a 1 A layer): an outer closed surface
 * enclosing the mesh of pbmp_set_mesh, same layout and checks as there.
 * Regions: inside the mesh eps_in (the sites), between the two surfaces
 * eps_stern without ions, outside the outer surface eps_out and kappa.  The
 * solve then works on both surfaces' densities (the one-surface system of
 * each surface coupled by the layer potentials of the other at its
 * collocation points; the reaction field comes from the inner surface);
 * pbmp_matvec applies that coupled operator to [phi1, dphi1, phi2, dphi2]
 * ([2 nt1 + 2 nt2], caller's panel order within each surface).  Call after
 * pbmp_set_mesh; nt = 0 removes the layer.  Direct mode only (PBMP_EARG in
 * treecode mode); pbmp_backward and transposed products are not available
 * with a layer (PBMP_ESTATE).  PBMP_EMESH when the outer surface does not
 * enclose the inner one. */
int pbmp_set_stern(pbmp_ctx *c, int64_t nv, const double *verts, int64_t nt,
                   const int32_t *tris, double eps_stern, int where);

/* The octree and interaction lists that pbmp_set_mesh built in treecode
 * mode (section "The treecode algorithm"; panels binned by centroid on a
 * 2^21 grid over the bounding cube, a cell split while it holds more than
 * leaf_panels panels; lists per target leaf under the acceptance test
 * R_B < theta (|c_B - c_T| - R_T)), for inspection and tests.
 * counts[0..3] receive nbox, nleaf, the total number of M2P list entries
 * and of P2P list entries.  Every array may be NULL (skipped); non-NULL
 * arrays are host memory of at least
 *   perm[N]            internal panel order -> user panel index
 *   box_range[2 nbox]  internal panel range [start, end) of each box
 *   box_level[nbox]    depth (root 0)
 *   box_centre[3 nbox] expansion centre (midpoint of the far nodes' bounding box)
 *   box_radius[2 nbox] R_B (far nodes) and R_T (centroids) about the centre
 *   leaf_box[nleaf]    box id of each target leaf
 *   m2p_ptr[nleaf+1], m2p_box[n_m2p]   accepted boxes of target leaf k
 *   p2p_ptr[nleaf+1], p2p_box[n_p2p]   leaves summed directly for leaf k
 * Returns PBMP_ESTATE when no tree was built (direct mode, or no mesh). */
int pbmp_tree_export(pbmp_ctx *c, int64_t counts[4], int32_t *perm, int32_t *box_range,
                     int32_t *box_level, double *box_centre, double *box_radius,
                     int32_t *leaf_box, int32_t *m2p_ptr, int32_t *m2p_box,
                     int32_t *p2p_ptr, int32_t *p2p_box);

/* Binding energies of a complex AB from three contexts solved with the
 * same options: AB (the complex: receptor sites first, then the ligand's),
 * the receptor A and the ligand B alone (section "Calculation of the
 * binding energy").  out[0] = dG_solv(AB) - dG_solv(A) - dG_solv(B)
 * (eq. rel_bind_energy); out[1] = G_AB - G_A - G_B with G the vacuum-state
 * Coulomb energy of each solve (eq. bind_vac); out[2] = out[0] + out[1]
 * (eq. bind_energy); kcal/mol, host memory.  PBMP_ESTATE unless each
 * context holds a completed solve; errors are reported on `complex`. */
int pbmp_binding_energies(pbmp_ctx *complex, pbmp_ctx *receptor, pbmp_ctx *ligand,
                          double out[3]);

/* Gradient of the relative binding energy with respect to a rigid
 * translation t of the ligand, from the solved complex: sites
 * [first_ligand_site, m) of the complex are the ligand's; a vertex of the
 * complex surface belongs to the ligand when the site minimising
 * |v - r_a| - R_a (radii [m], the sites' atomic radii, in `where` memory)
 * is a ligand site; the ligand's own surface moves as a whole and the
 * receptor does not move, so only the complex contributes:
 *   g_t = sum over ligand sites of d dG_AB/dr + sum over ligand vertices of d dG_AB/dv,
 * through a backward of the complex (pbmp_backward with dG_bar = 1; its
 * tolerances and warnings).  g_t [3] (kcal/mol/A) and n_ligand_vertices
 * (nullable) are host memory. */
int pbmp_ligand_translation_gradient(pbmp_ctx *complex, int64_t first_ligand_site,
                                     const double *radii, double g_t[3],
                                     int64_t *n_ligand_vertices, int where);

/* Message for the last failing call on c (never NULL). */
const char *pbmp_last_error(const pbmp_ctx *c);

/* Release all device memory and the stream the library created. */
void pbmp_destroy(pbmp_ctx *c);

#ifdef __cplusplus
}
#endif
#endif /* PBMP_H */
