/*
 * Standalone driver of the oracle's C loops for a sanitizer build (test
 * infrastructure only): a regular octahedron refined once (32 panels,
 * radius 1) and a few interior points; every exported loop runs once.
 * Built with -fsanitize=address,undefined by tests/test_sanitizers_cpu.py;
 * exits 0 when every result is finite and the double-layer row sums are
 * close to -1/2 (a consistency check only: the far rule is not exact).
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int N;
    const double *verts; const int *tris;
    const double *cen; const double *nrm; const double *area;
    int nf; const double *fb; const double *fw;
    int nn; const double *nb; const double *nw;
    int ngl; const double *glx; const double *glw;
    double kappa, eta;
} orc_mesh;

void orc_entries(const orc_mesh *m, int i0, int i1, double *VL, double *KL, double *VY, double *KY);
void orc_operator_sums(const orc_mesh *m, int i0, int i1, const double *phi, const double *dphi, double *out);
void orc_near_correction_sums(const orc_mesh *m, int i0, int i1, const double *phi, const double *dphi, double *out);
void orc_readout(const orc_mesh *m, int M, const double *pts, const double *phi, const double *dphi, double *out);
void orc_self_integrals(const orc_mesh *m, int j, const double *c, double *out);

static double V[64][3];
static int T[64][3];
static int nv = 0, nt = 0;

static int midpoint(int a, int b) {
    double p[3];
    for (int d = 0; d < 3; ++d) p[d] = 0.5 * (V[a][d] + V[b][d]);
    double r = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    for (int k = 0; k < nv; ++k) {
        double e = fabs(V[k][0] - p[0] / r) + fabs(V[k][1] - p[1] / r) + fabs(V[k][2] - p[2] / r);
        if (e < 1e-12) return k;
    }
    for (int d = 0; d < 3; ++d) V[nv][d] = p[d] / r;
    return nv++;
}

int main(void) {
    const double o[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    const int f[8][3] = {{0, 2, 4}, {2, 1, 4}, {1, 3, 4}, {3, 0, 4},
                         {2, 0, 5}, {1, 2, 5}, {3, 1, 5}, {0, 3, 5}};
    for (int k = 0; k < 6; ++k) { for (int d = 0; d < 3; ++d) V[k][d] = o[k][d]; }
    nv = 6;
    for (int k = 0; k < 8; ++k) {
        int a = f[k][0], b = f[k][1], c = f[k][2];
        int ab = midpoint(a, b), bc = midpoint(b, c), ca = midpoint(c, a);
        int t[4][3] = {{a, ab, ca}, {ab, b, bc}, {ca, bc, c}, {ab, bc, ca}};
        for (int q = 0; q < 4; ++q) { for (int d = 0; d < 3; ++d) T[nt][d] = t[q][d]; nt++; }
    }
    double *cen = malloc(sizeof(double) * 3 * nt), *nrm = malloc(sizeof(double) * 3 * nt);
    double *area = malloc(sizeof(double) * nt);
    for (int j = 0; j < nt; ++j) {
        const double *a = V[T[j][0]], *b = V[T[j][1]], *c = V[T[j][2]];
        double e1[3], e2[3], cr[3];
        for (int d = 0; d < 3; ++d) { e1[d] = b[d] - a[d]; e2[d] = c[d] - a[d]; cen[3 * j + d] = (a[d] + b[d] + c[d]) / 3; }
        cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
        cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
        cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
        double nn = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        for (int d = 0; d < 3; ++d) nrm[3 * j + d] = cr[d] / nn;
        area[j] = 0.5 * nn;
    }
    const double fb[9] = {2. / 3, 1. / 6, 1. / 6, 1. / 6, 2. / 3, 1. / 6, 1. / 6, 1. / 6, 2. / 3};
    const double fw[3] = {1. / 3, 1. / 3, 1. / 3};
    const double nb[3] = {1. / 3, 1. / 3, 1. / 3}, nw[1] = {1.0};
    const double glx[2] = {-0.5773502691896258, 0.5773502691896258}, glw[2] = {1.0, 1.0};
    orc_mesh m = {nt, &V[0][0], &T[0][0], cen, nrm, area, 3, fb, fw, 1, nb, nw, 2, glx, glw, 0.125, 2.0};
    double *ent = malloc(sizeof(double) * 4 * nt * nt);
    orc_entries(&m, 0, nt, ent, ent + nt * nt, ent + 2 * nt * nt, ent + 3 * nt * nt);
    double *phi = malloc(sizeof(double) * nt), *dphi = malloc(sizeof(double) * nt);
    for (int j = 0; j < nt; ++j) { phi[j] = 1.0; dphi[j] = 0.5 + 0.01 * j; }
    double *s = malloc(sizeof(double) * 4 * nt), *c = malloc(sizeof(double) * 4 * nt);
    orc_operator_sums(&m, 0, nt, phi, dphi, s);
    orc_near_correction_sums(&m, 0, nt, phi, dphi, c);
    const double pts[6] = {0.1, 0.2, -0.1, -0.3, 0.0, 0.25};
    double ro[20], si[2];
    orc_readout(&m, 2, pts, phi, dphi, ro);
    orc_self_integrals(&m, 0, cen, si);
    int bad = 0;
    for (int k = 0; k < 4 * nt * nt; ++k) bad |= !isfinite(ent[k]);
    for (int k = 0; k < 4 * nt; ++k) bad |= !isfinite(s[k]) || !isfinite(c[k]);
    for (int k = 0; k < 20; ++k) bad |= !isfinite(ro[k]);
    bad |= !isfinite(si[0]) || !isfinite(si[1]);
    double worst = 0.0;
    for (int i = 0; i < nt; ++i) worst = fmax(worst, fabs(s[4 * i + 1] + 0.5));
    printf("panels %d, worst |sum_j K_L[i,j] + 1/2| %.3e\n", nt, worst);
    free(cen); free(nrm); free(area); free(ent); free(phi); free(dphi); free(s); free(c);
    return bad || worst > 0.2;
}
