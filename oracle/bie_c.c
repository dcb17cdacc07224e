/*
 * FP64 CPU oracle: boundary-integral operator entries, matrix-free products
 * and site readout (TEST INFRASTRUCTURE ONLY -- never linked into the
 * product library).  Plain loops, OpenMP over targets, no blocking.
 *
 * Operators (eq. layers, eq. free-space), with R = x - y, r = |R|:
 *   V_L = int G_L dy,          G_L  = 1/(4 pi r)
 *   K_L = int dG_L/dn_y dy,    dG_L/dn_y = n_y . R / (4 pi r^3)
 *   V_Y = int G_Y dy,          G_Y  = exp(-kappa r)/(4 pi r)
 *   K_Y = int dG_Y/dn_y dy,    dG_Y/dn_y = n_y . R (1 + kappa r) exp(-kappa r)/(4 pi r^3)
 * over flat panels with piecewise-constant densities and centroid
 * collocation (Algorithmic details, "boundary element method"):
 *   j == i:                      singular: V exact / semi-analytic, K = 0
 *   |c_i - c_j| < eta sqrt(A_i): near-singular: 19-node rule
 *   otherwise:                   far: low-order rule
 *
 * Singular panel (polar decomposition about the collocation point c into
 * the three sub-triangles (c, v_a, v_b); h = distance from c to edge ab,
 * s_a, s_b = signed offsets of v_a, v_b from the foot of the perpendicular):
 *   V_L = 1/(4 pi) sum_e h [asinh(s_b/h) - asinh(s_a/h)]
 *   V_Y = V_L + 1/(4 pi) sum_e int_{th_a}^{th_b} [(1-exp(-kappa rho))/kappa - rho] dth,
 *         rho = h / cos(th); the remainder is integrated with Gauss-Legendre
 *         nodes placed along each edge, in the variable u = asinh(s/h) of the
 *         edge coordinate s = h tan(th) (rho = h cosh u, dth = du / cosh u),
 *         in which the integrand is smooth.
 */
#include <math.h>
#include <stddef.h>

#define FOUR_PI (4.0 * 3.14159265358979323846)

typedef struct {
    int N;
    const double *verts;   /* [Nv*3] */
    const int *tris;       /* [N*3]  */
    const double *cen;     /* [N*3]  */
    const double *nrm;     /* [N*3]  */
    const double *area;    /* [N]    */
    int nf; const double *fb; const double *fw;   /* far rule   */
    int nn; const double *nb; const double *nw;   /* near rule  */
    int ngl; const double *glx; const double *glw; /* edge rule on [-1,1] */
    double kappa, eta;
} orc_mesh;

static void vert(const orc_mesh *m, int j, int k, double *v)
{
    const double *p = m->verts + 3 * (size_t)m->tris[3 * (size_t)j + k];
    v[0] = p[0]; v[1] = p[1]; v[2] = p[2];
}

/* Singular V_L and V_Y of panel j seen from point c (c in the panel). */
static void self_integrals(const orc_mesh *m, int j, const double *c,
                           double *VL, double *VY)
{
    double v[3][3];
    for (int k = 0; k < 3; ++k) vert(m, j, k, v[k]);
    double sl = 0.0, sy = 0.0;
    for (int e = 0; e < 3; ++e) {
        const double *a = v[e], *b = v[(e + 1) % 3];
        double t[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double L = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
        t[0] /= L; t[1] /= L; t[2] /= L;
        double ca[3] = {a[0] - c[0], a[1] - c[1], a[2] - c[2]};
        double sa = ca[0] * t[0] + ca[1] * t[1] + ca[2] * t[2];
        double sb = sa + L;
        double p[3] = {ca[0] - sa * t[0], ca[1] - sa * t[1], ca[2] - sa * t[2]};
        double h = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        sl += h * (asinh(sb / h) - asinh(sa / h));
        if (m->kappa > 0.0) {
            /* remainder along the edge in u = asinh(s/h): rho = h cosh(u),
             * dth = du / cosh(u); the integrand is smooth in u */
            double ua = asinh(sa / h), ub = asinh(sb / h);
            double half = 0.5 * (ub - ua), mid = 0.5 * (ub + ua);
            for (int g = 0; g < m->ngl; ++g) {
                double u = mid + half * m->glx[g];
                double ch = cosh(u);
                double rho = h * ch;
                double f = -expm1(-m->kappa * rho) / m->kappa - rho;
                sy += half * m->glw[g] * f / ch;
            }
        }
    }
    *VL = sl / FOUR_PI;
    *VY = (sl + sy) / FOUR_PI;
}

/* Entries (V_L, K_L, V_Y, K_Y) of target point x against panel j with a
 * given rule. */
static void rule_entries(const orc_mesh *m, int j, const double *x, int nq,
                         const double *bary, const double *w, double *out)
{
    double v[3][3];
    for (int k = 0; k < 3; ++k) vert(m, j, k, v[k]);
    const double *n = m->nrm + 3 * (size_t)j;
    double A = m->area[j];
    double vl = 0, kl = 0, vy = 0, ky = 0;
    for (int q = 0; q < nq; ++q) {
        double y[3];
        for (int d = 0; d < 3; ++d)
            y[d] = bary[3 * q] * v[0][d] + bary[3 * q + 1] * v[1][d] + bary[3 * q + 2] * v[2][d];
        double R[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
        double r = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
        double nR = n[0] * R[0] + n[1] * R[1] + n[2] * R[2];
        double e = exp(-m->kappa * r);
        double wa = w[q] * A;
        vl += wa / (FOUR_PI * r);
        kl += wa * nR / (FOUR_PI * r * r * r);
        vy += wa * e / (FOUR_PI * r);
        ky += wa * nR * (1.0 + m->kappa * r) * e / (FOUR_PI * r * r * r);
    }
    out[0] = vl; out[1] = kl; out[2] = vy; out[3] = ky;
}

/* Matrix entry (i, j) of the four operators (collocation at centroid c_i). */
static void entry(const orc_mesh *m, int i, int j, double *out)
{
    const double *ci = m->cen + 3 * (size_t)i;
    if (i == j) {
        double vl, vy;
        self_integrals(m, j, ci, &vl, &vy);
        out[0] = vl; out[1] = 0.0; out[2] = vy; out[3] = 0.0;
        return;
    }
    const double *cj = m->cen + 3 * (size_t)j;
    double d[3] = {ci[0] - cj[0], ci[1] - cj[1], ci[2] - cj[2]};
    double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (dist < m->eta * sqrt(m->area[i]))
        rule_entries(m, j, ci, m->nn, m->nb, m->nw, out);
    else
        rule_entries(m, j, ci, m->nf, m->fb, m->fw, out);
}

/* Dense rows [i0, i1) of V_L, K_L, V_Y, K_Y, each written row-major into
 * an array of (i1-i0) x N. */
void orc_entries(const orc_mesh *m, int i0, int i1, double *VL, double *KL,
                 double *VY, double *KY)
{
    int N = m->N;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int i = i0; i < i1; ++i) {
        for (int j = 0; j < N; ++j) {
            double e[4];
            entry(m, i, j, e);
            size_t o = (size_t)(i - i0) * N + j;
            VL[o] = e[0]; KL[o] = e[1]; VY[o] = e[2]; KY[o] = e[3];
        }
    }
}

/* Matrix-free sums for targets [i0, i1):
 *   sVL_i = sum_j V_L[i,j] dphi_j,  sKL_i = sum_j K_L[i,j] phi_j,
 *   sVY_i = sum_j V_Y[i,j] dphi_j,  sKY_i = sum_j K_Y[i,j] phi_j. */
void orc_operator_sums(const orc_mesh *m, int i0, int i1, const double *phi,
                       const double *dphi, double *out /* [(i1-i0)*4] */)
{
    int N = m->N;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int i = i0; i < i1; ++i) {
        double s[4] = {0, 0, 0, 0};
        for (int j = 0; j < N; ++j) {
            double e[4];
            entry(m, i, j, e);
            s[0] += e[0] * dphi[j];
            s[1] += e[1] * phi[j];
            s[2] += e[2] * dphi[j];
            s[3] += e[3] * phi[j];
        }
        for (int k = 0; k < 4; ++k) out[4 * (size_t)(i - i0) + k] = s[k];
    }
}

/* Reaction potential and its first and second derivatives at off-surface
 * points (eq. pot_solvent, eq. Efield_solv, eq. ddphi; appendix with the
 * 1/(4 pi) of G_L kept):
 *   phi_s(x) = sum_j [V_L(x, j) dphi_j - K_L(x, j) phi_j]
 * with derivatives taken in x.  Near rule where |x - c_j| < eta sqrt(A_j).
 * out per point: [phi, d/dx, d/dy, d/dz, xx, xy, xz, yy, yz, zz]. */
void orc_readout(const orc_mesh *m, int M, const double *pts,
                 const double *phi, const double *dphi, double *out)
{
    int N = m->N;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int l = 0; l < M; ++l) {
        const double *x = pts + 3 * (size_t)l;
        double acc[10] = {0};
        for (int j = 0; j < N; ++j) {
            const double *cj = m->cen + 3 * (size_t)j;
            double dd[3] = {x[0] - cj[0], x[1] - cj[1], x[2] - cj[2]};
            double dist = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
            int nq; const double *bary, *w;
            if (dist < m->eta * sqrt(m->area[j])) { nq = m->nn; bary = m->nb; w = m->nw; }
            else { nq = m->nf; bary = m->fb; w = m->fw; }
            double v[3][3];
            for (int k = 0; k < 3; ++k) vert(m, j, k, v[k]);
            const double *n = m->nrm + 3 * (size_t)j;
            double A = m->area[j];
            for (int q = 0; q < nq; ++q) {
                double y[3];
                for (int d = 0; d < 3; ++d)
                    y[d] = bary[3 * q] * v[0][d] + bary[3 * q + 1] * v[1][d] + bary[3 * q + 2] * v[2][d];
                double R[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
                double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
                double r = sqrt(r2);
                double r3 = r2 * r, r5 = r3 * r2, r7 = r5 * r2;
                double nR = n[0] * R[0] + n[1] * R[1] + n[2] * R[2];
                double a = w[q] * A * dphi[j] / FOUR_PI;   /* single layer */
                double b = w[q] * A * phi[j] / FOUR_PI;    /* double layer */
                /* G = 1/r; dG_i = -R_i/r^3; ddG_ik = 3 R_i R_k/r^5 - delta/r^3
                 * H = nR/r^3; dH_i = n_i/r^3 - 3 nR R_i/r^5;
                 * ddH_ik = -3(n_i R_k + n_k R_i + nR delta)/r^5 + 15 nR R_i R_k/r^7 */
                acc[0] += a / r - b * nR / r3;
                for (int i = 0; i < 3; ++i)
                    acc[1 + i] += a * (-R[i] / r3) - b * (n[i] / r3 - 3.0 * nR * R[i] / r5);
                int o = 4;
                for (int i = 0; i < 3; ++i)
                    for (int k = i; k < 3; ++k) {
                        double del = (i == k) ? 1.0 : 0.0;
                        double ddG = 3.0 * R[i] * R[k] / r5 - del / r3;
                        double ddH = -3.0 * (n[i] * R[k] + n[k] * R[i] + nR * del) / r5
                                     + 15.0 * nR * R[i] * R[k] / r7;
                        acc[o++] += a * ddG - b * ddH;
                    }
            }
        }
        for (int k = 0; k < 10; ++k) out[10 * (size_t)l + k] = acc[k];
    }
}

/* Exposed for the singular-integral pins. */
void orc_self_integrals(const orc_mesh *m, int j, const double *c, double *out)
{
    self_integrals(m, j, c, &out[0], &out[1]);
}

/* Near-field corrections for targets [i0, i1): for every pair that the
 * method integrates with a rule other than the far rule (the singular pair
 * j == i and the near-singular pairs |c_i - c_j| < eta sqrt(A_i)), the
 * method's entry minus the far-rule entry, applied to the densities:
 *   out_i = sum_{j near or self} (E_ij - F_ij) * (dphi_j, phi_j, dphi_j, phi_j).
 * A treecode product is its far-rule sum (expansions for accepted boxes,
 * far rule elsewhere) plus these corrections. */
void orc_near_correction_sums(const orc_mesh *m, int i0, int i1, const double *phi,
                              const double *dphi, double *out /* [(i1-i0)*4] */)
{
    int N = m->N;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int i = i0; i < i1; ++i) {
        const double *ci = m->cen + 3 * (size_t)i;
        double s[4] = {0, 0, 0, 0};
        for (int j = 0; j < N; ++j) {
            const double *cj = m->cen + 3 * (size_t)j;
            double d[3] = {ci[0] - cj[0], ci[1] - cj[1], ci[2] - cj[2]};
            double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (j != i && !(dist < m->eta * sqrt(m->area[i])))
                continue;
            double e[4], f[4];
            entry(m, i, j, e);
            rule_entries(m, j, ci, m->nf, m->fb, m->fw, f);
            s[0] += (e[0] - f[0]) * dphi[j];
            s[1] += (e[1] - f[1]) * phi[j];
            s[2] += (e[2] - f[2]) * dphi[j];
            s[3] += (e[3] - f[3]) * phi[j];
        }
        for (int k = 0; k < 4; ++k) out[4 * (size_t)(i - i0) + k] = s[k];
    }
}
