/* Runs every C routine of the oracle on a closed bipyramid whose two poles
 * have valence 80 (more incident triangles than any fixed-size list would
 * hold), so that AddressSanitizer and UndefinedBehaviorSanitizer see every
 * code path: regular, centroid and Sauter-Schwab pair blocks (coincident,
 * edge, vertex pairs), operator rows and columns with V, K and D, mass rows,
 * the right-hand side and the reaction potential.  Exit status 0 and "ok"
 * when all outputs are finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_regular_rule(double *bary, double *w);
int orc_gauss_legendre01(int n, double *x, double *w);
void orc_triangle_geometry(const double *xyz, const int32_t *tri, int nt, double *area, double *normal);
int orc_pair_block(const double *xyz, const int32_t *tri, int t, int s, double kappa, int nss, int kernel_mode,
                   int quad_mode, double *V, double *K);
void orc_operator_rows(int nv, int nt, const double *xyz, const int32_t *tri, double kappa, int nss, int nrows,
                       const int32_t *rows, int mode, double *outV, double *outK, double *outD, int quad_mode);
void orc_mass_rows(int nv, int nt, const double *xyz, const int32_t *tri, int nrows, const int32_t *rows,
                   double *out);
void orc_rhs(int nv, int nt, const double *xyz, const int32_t *tri, int nq, const double *qxyz, const double *q,
             double eps_in, double *bD, double *bN);
void orc_reaction_potential(int nv, int nt, const double *xyz, const int32_t *tri, const double *phi,
                            const double *dphi, int npts, const double *pts, double *out);

static int finite_all(const double *a, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

int main(void)
{
    const int n = 80, nv = n + 2, nt = 2 * n;
    double *xyz = malloc(sizeof(double) * 3 * nv);
    int32_t *tri = malloc(sizeof(int32_t) * 3 * nt);
    xyz[0] = 0.0; xyz[1] = 0.0; xyz[2] = 1.5;     /* top pole */
    xyz[3] = 0.0; xyz[4] = 0.0; xyz[5] = -1.5;    /* bottom pole */
    for (int i = 0; i < n; ++i) {
        const double a = 2.0 * 3.14159265358979323846 * i / n;
        xyz[3 * (i + 2)] = cos(a);
        xyz[3 * (i + 2) + 1] = sin(a);
        xyz[3 * (i + 2) + 2] = 0.0;
    }
    for (int i = 0; i < n; ++i) {
        const int e0 = 2 + i, e1 = 2 + (i + 1) % n;
        tri[6 * i] = 0; tri[6 * i + 1] = e0; tri[6 * i + 2] = e1;           /* counter-clockwise from outside */
        tri[6 * i + 3] = 1; tri[6 * i + 4] = e1; tri[6 * i + 5] = e0;
    }
    int ok = 1;
    double bary[18], w[6], gx[16], gw[16];
    orc_regular_rule(bary, w);
    ok &= orc_gauss_legendre01(16, gx, gw) == 0 && finite_all(gx, 16) && finite_all(gw, 16);
    ok &= orc_gauss_legendre01(0, gx, gw) != 0;
    double *area = malloc(sizeof(double) * nt), *normal = malloc(sizeof(double) * 3 * nt);
    orc_triangle_geometry(xyz, tri, nt, area, normal);
    ok &= finite_all(area, nt) && finite_all(normal, 3 * nt);
    /* coincident, edge (0,1), vertex (0,2), far (0, n + n/2) pairs in both orders, every mode */
    const int pairs[5][2] = {{0, 0}, {0, 1}, {0, 2}, {0, n + n / 2}, {n + n / 2, 0}};
    for (int p = 0; p < 5; ++p)
        for (int km = 0; km < 3; ++km)
            for (int qm = 0; qm < 3; ++qm) {
                /* the regular rule on a coincident pair meets r = 0 with the 1/r kernel: a
                   combination the oracle uses only with the smooth test kernels */
                if (p == 0 && km == 0 && qm == 1) continue;
                double V[9], K[9];
                orc_pair_block(xyz, tri, pairs[p][0], pairs[p][1], 0.125, 3, km, qm, V, K);
                ok &= finite_all(V, 9) && finite_all(K, 9);
            }
    const int32_t rows[3] = {0, 1, 5};
    double *V = malloc(sizeof(double) * 3 * nv), *K = malloc(sizeof(double) * 3 * nv),
           *D = malloc(sizeof(double) * 3 * nv), *M = malloc(sizeof(double) * 3 * nv);
    for (int mode = 0; mode < 2; ++mode)
        for (int qm = 0; qm < 3; qm += 2) {
            orc_operator_rows(nv, nt, xyz, tri, 0.125, 2, 3, rows, mode, V, K, D, qm);
            ok &= finite_all(V, 3 * nv) && finite_all(K, 3 * nv) && finite_all(D, 3 * nv);
        }
    orc_operator_rows(nv, nt, xyz, tri, 0.0, 2, 3, rows, 0, V, NULL, NULL, 0);
    ok &= finite_all(V, 3 * nv);
    orc_mass_rows(nv, nt, xyz, tri, 3, rows, M);
    ok &= finite_all(M, 3 * nv);
    const double qxyz[6] = {0.1, 0.0, 0.2, -0.2, 0.1, -0.3}, q[2] = {1.0, -0.5};
    double *bD = malloc(sizeof(double) * nv), *bN = malloc(sizeof(double) * nv);
    orc_rhs(nv, nt, xyz, tri, 2, qxyz, q, 4.0, bD, bN);
    ok &= finite_all(bD, nv) && finite_all(bN, nv);
    double pr[2];
    orc_reaction_potential(nv, nt, xyz, tri, bD, bN, 2, qxyz, pr);
    ok &= finite_all(pr, 2);
    free(xyz); free(tri); free(area); free(normal); free(V); free(K); free(D); free(M); free(bD); free(bN);
    puts(ok ? "ok" : "non-finite output");
    return ok ? 0 : 1;
}
