// Launchers of the pbmp device kernels (gfx950).  Every launcher enqueues on
// the given stream and returns immediately.  Arrays are in the library's
// internal panel order.
#pragma once

#include "common.hpp"

namespace pbmp {

// Panel geometry, FP64 SoA layout of `geo` [7N]: cx, cy, cz, nx, ny, nz, A.
// src64 [16N] and src32 [16N]: per panel the far-field nodes y0, y1, y2
// (unused ones zero), the normal, the plane offset n.y, then two strengths
// (written per product) and one pad.  tgt32 [3N]: centroids in FP32 (SoA).
void launch_panel_geometry(hipStream_t s, int N, const double *verts,
                           const int *tri, const RuleArgs &ru, double *geo,
                           double *src64, float *src32, float *tgt32);

// Near-singular / singular correction for the CSR entries (row i, col j):
// val[4e..4e+3] = (V_L, K_L, V_Y, K_Y)(exact or 19-node) - (far rule), in the
// integral-equation normalisation; diag [2N] gets V_L,ii and V_Y,ii.
// The far-rule value subtracted is computed exactly as the far-field product
// of the chosen precision computes it (fp64 or FP32 from src32/tgt32).
void launch_near_values(hipStream_t s, bool fp64, int N, const int *rowptr,
                        const int *col, const double *verts, const int *tri,
                        const double *geo, const double *src64,
                        const float *src32, const float *tgt32,
                        const RuleArgs &ru, double kappa, double *val,
                        double *diag);

// Winding number of each point with respect to the surface: [M].
void launch_winding(hipStream_t s, int N, int M, const double *verts,
                    const int *tri, const double *pts, double *wind);

// Strengths of the product: s_V = w_q A phi'/(4 pi), s_K = w_q A phi/(4 pi)
// written into slots 13, 14 of src64 and src32.  x = [phi; dphi] [2N].
void launch_pack_strengths(hipStream_t s, int N, int nf, const double *geo,
                           const double *x, double *src64, float *src32);

// Direct far-field sums over all panels of the source range, per target:
// part[(chunk*4 + k)*Nt + i], k = V_L, K_L, V_Y, K_Y.
// floor_r2: FP32 pairs closer than 1e-4 A add nothing (needed only for the
// one-node rule, or panels small enough for a node and a centroid to
// coincide in FP32).
void launch_p2p_direct(hipStream_t s, bool fp64, int nf, int N, int Nt,
                       const double *src64, const float *src32,
                       const double *geo, const float *tgt32, double kappa,
                       int nchunk, double *part, bool floor_r2 = true);

// y = A x from the far partials (summed over nchunk chunks in order), the
// near/self CSR correction and the identity terms (eq. integral_eq).
void launch_finish(hipStream_t s, int N, int nchunk, const double *part,
                   const int *rowptr, const int *col, const double *val,
                   const double *x, double eps_ratio, double *y);

// z -> A^T z (direct): transposed far sums and the transposed near/self
// correction (trow/tcol/tent: for column j the rows i and entry ids).
void launch_transpose(hipStream_t s, bool fp64, int nf, int N,
                      const double *src64, const float *src32,
                      const double *geo, const float *tgt32, const double *z,
                      double kappa, int nchunk, double *part,
                      const int *trow, const int *tcol, const int *tent,
                      const double *val, double eps_ratio, double *y);

// Right-hand side f[N] (eq. rhs_multipole) from sites (xyz[3M], q[M],
// p[3M], Q9[9M]); fp64 selects FP64 pair terms, else FP32 pair terms with
// FP64 accumulation.
void launch_rhs(hipStream_t s, bool fp64, int N, int M, const double *geo,
                const double *xyz, const double *q, const double *p,
                const double *Q9, double eps_in, double *f);

// Reaction-potential readout at M sites (eq. pot_solvent and its first and
// second derivatives): out[10M] (full) or first 4 entries only (full=0),
// integral-equation normalisation.  Far rule over all panels, then the
// near-singular correction over the site's near panels (srow/scol).
void launch_readout(hipStream_t s, bool fp64, bool full, int N, int M,
                    const double *src64, const float *src32, const double *geo,
                    const double *verts, const int *tri, const RuleArgs &ru,
                    const double *x, const double *xyz, const int *srow,
                    const int *scol, int nchunk, double *part, double *out);
// Source chunks of the far readout for N panels and M sites (enough blocks
// of 64 sites x one chunk to fill the device); part holds nchunk * M * 10.
int readout_chunks(int N, int M);
// static device scratch of the entry point that allocates nothing: its size
// and its address on the current device (looked up once per device)
size_t static_scratch_bytes();
double *static_scratch();

// Coulomb field of the permanent multipoles at the sites, excluding pairs of
// the same polarisation group: Eperm[3M] = -grad phi_perm / eps_in.
void launch_perm_field(hipStream_t s, int M, const double *xyz,
                       const double *q, const double *d, const double *Q9,
                       const int *group, double eps_in, double *E);

// Thole-damped induced-dipole data at the sites from dipoles mu (all other
// sites): full=0 -> field E[3M] = -grad phi / eps_in; full=1 -> out[10M]
// = (phi, grad, hessian upper) / eps_in.
void launch_induced(hipStream_t s, bool full, int M, const double *xyz,
                    const double *mu, const double *alpha, double thole_a,
                    double eps_in, double *out);

// mu <- (1-w) mu + w alpha (Eperm + Eind - 4 pi grad phi_solv) ; sums
// |dmu|^2 into *dmu2 (single block, fixed order).  solv may be NULL.
void launch_scf_update(hipStream_t s, int M, const double *alpha,
                       const double *Eperm, const double *Eind,
                       const double *solv10, int solv_stride, double omega,
                       double *mu, double *dmu2);

// e[0] = 1/2 sum D_l (4 pi reac_l), e[1] = 1/2 sum D_l ind_l  with D_l =
// q + d.grad + (1/6) Q:grad grad (single block, fixed order).
// potential data [M,10] of the other sites' permanent multipoles (unmasked)
void launch_perm_potential(hipStream_t s, int M, const double *xyz, const double *q,
                           const double *d, const double *Q, double eps_in, double *out);
// Total molecular dipoles out[0..2] (vacuum) and out[3..5] (dissolved), e*A,
// about the mean site position (one block).
void launch_total_dipole(hipStream_t s, int M, const double *xyz, const double *q,
                         const double *d, const double *mu_v, const double *mu_d,
                         double *out);
void launch_energy(hipStream_t s, int M, const double *q, const double *d,
                   const double *Q9, const double *reac10, const double *ind10,
                   double *e);

// ----- Krylov helpers (FP64) -----
// h[k] = sum_i V[k*ld + i] w[i], k < nv (two-pass, deterministic)
void launch_mdot(hipStream_t s, int n, int nv, const double *V, size_t ld,
                 const double *w, double *partial, double *h);
// w -= sum_k V[k*ld + i] h[k]
void launch_gemv_sub(hipStream_t s, int n, int nv, const double *V, size_t ld,
                     const double *h, double *w);
// Arnoldi-step forms without the final reduction launch: the block sums of
// launch_mdot_partial (returns their count per vector) are added by every
// block of the consumer in a fixed order; block 0 stores the totals to hout.
// gemv_sub_p: w -= V h (nv <= 256); scale_inv_sqrt_p: v = w / |w| (zero
// stays zero).
int launch_mdot_partial(hipStream_t s, int n, int nv, const double *V, size_t ld,
                        const double *w, double *partial);
void launch_gemv_sub_p(hipStream_t s, int n, int nv, const double *V, size_t ld, int nblk,
                       const double *partial, double *hout, double *w);
void launch_scale_inv_sqrt_p(hipStream_t s, int n, int nblk, const double *partial,
                             double *hout, const double *w, double *v);
// v = w * (1/ *nrm) with nrm = sqrt(*nrm2); zero when *nrm2 is zero
void launch_scale_inv_sqrt(hipStream_t s, int n, const double *w,
                           const double *nrm2, double *v);
void launch_axpy(hipStream_t s, int n, double a, const double *x, double *y);
void launch_xmy(hipStream_t s, int n, const double *b, const double *ax,
                double *r);  // r = b - ax
// z = M^{-1} u with M the 2x2 panel blocks [[1/2, -VLii],[1/2, e VYii]]
void launch_precond(hipStream_t s, int N, const double *diag, double eps_ratio,
                    const double *u, double *z);
// x += M^{-1} (V y) with nv basis vectors
// z = M^{-1} u with the far-field strengths of z packed into src64/src32
// (launch_precond followed by launch_pack_strengths, one launch)
void launch_precond_pack(hipStream_t s, int N, int nf, const double *diag, double eps_ratio,
                         const double *geo, const double *u, double *z, double *src64,
                         float *src32);
void launch_update_solution(hipStream_t s, int N, int nv, const double *V,
                            size_t ld, const double *y, const double *diag,
                            double eps_ratio, double *x);
// gather/scatter with a permutation: out[i] = in[perm[i]] (gather) or
// out[perm[i]] = in[i] (scatter), for `blocks` consecutive blocks of n.
void launch_permute(hipStream_t s, int n, int blocks, const int *perm,
                    const double *in, double *out, bool gather);
void launch_scale(hipStream_t s, int n, double a, const double *x, double *y);

class Tree;
struct KernelClock;
// Treecode far field: P2M/M2M moments, P2P over near leaves and M2P over
// accepted boxes, into part[slot][4][N].
void tree_apply(Tree &t, hipStream_t s, bool fp64, int nf, int N,
                const double *geo, const double *src64, const float *src32,
                const float *tgt32, double kappa, double *part, KernelClock &clk,
                bool floor_r2);
// finish with a per-target number of partial slots
// A^T z with the treecode (transposed P2P, M2P^T + L2L + L2P, transposed
// near/self correction)
void tree_apply_transpose(Tree &t, hipStream_t s, bool fp64, int nf, int N, const double *geo,
                          const double *src64, const float *src32, const float *tgt32,
                          const double *z, double kappa, double *part, const int *trow,
                          const int *tcol, const int *tent, const double *val, double eps_ratio,
                          double *y);
// Far-field part of the mesh adjoint with the treecode: d/d(collocation
// points) gc [3N] and d/d(far nodes, normals, areas) gy [9N], gn [3N],
// gA [N] of lambda . A x (assigned, not accumulated); part: the product's
// forward slots [max_slots][4][N], partT: [max_slots_T][13][N]
void tree_mesh_adjoint_far(Tree &t, hipStream_t s, int nf, int N, const double *geo,
                           const double *src64, const double *lam, double kappa,
                           double eps_ratio, double *part, double *partT, double *gc,
                           double *gy, double *gn, double *gA);
void launch_finish_slots(hipStream_t s, int N, const int *tslots,
                         const double *part, const int *rowptr, const int *col,
                         const double *val, const double *x, double eps_ratio,
                         double *y);

}  // namespace pbmp
