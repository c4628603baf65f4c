/*
 * pbm_oracle.c -- plain FP64 CPU oracle for the Galerkin P1 boundary-element
 * discretisation of the linearised Poisson-Boltzmann interface problem
 * (Search, Cooper & van 't Wout, arXiv 2108.10481).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant generator
 * with the GPU library: every rule below is typed in or generated here.
 *
 * What it computes (each function cites the passage it follows):
 *   - the free-space kernels G = exp(-kappa r)/(4 pi r) (kappa = 0: Laplace)
 *     and its normal derivative in the source point (Methodology, Green's
 *     functions and Eq. layer_potentials);
 *   - local 3x3 Galerkin blocks of the single-layer V and double-layer K
 *     operators for one ordered triangle pair, with a regular tensor-product
 *     rule for pairs sharing no vertex and Sauter-Schwab singular quadrature
 *     for pairs sharing a vertex, an edge, or the whole triangle
 *     (Numerical discretization: continuous P1 Galerkin on flat triangles);
 *     the local vertex arrangement of a singular pair is found by searching
 *     the rotations and arrangements of the two triangles for the stated
 *     property;
 *   - the hypersingular D block from the integration-by-parts identity
 *     D = curl.curl G + kappa^2 (n_x . n_y) G;
 *   - rows (or columns) of V, K, D and of the mass matrix M;
 *   - the source projections of the point charges (Eq. sources) tested with
 *     the P1 basis;
 *   - the reaction potential at points from the surface traces
 *     (Eq. phireac_bie), from which Delta G (Eq. dG) follows.
 * Loops are plain loops over triangles and triangle pairs; OpenMP only splits
 * independent output rows across threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------ rules */

/* Symmetric 6-point degree-4 rule on a triangle (Dunavant 1985 / Strang-Fix),
 * generated here from its closed form.  rb[p][k] = barycentric coordinate k of
 * point p; rw[p] = weight relative to the triangle area (sum 1). */
static double rb[6][3], rw[6];
static int rule_ready = 0;

static void init_rule(void)
{
    if (rule_ready) return;
    double s10 = sqrt(10.0);
    double t = sqrt(38.0 - 44.0 * sqrt(2.0 / 5.0));
    double a = (8.0 - s10 + t) / 18.0;
    double b = (8.0 - s10 - t) / 18.0;
    double u = sqrt(213125.0 - 53320.0 * s10);
    double wa = (620.0 + u) / 3720.0;
    double wb = (620.0 - u) / 3720.0;
    for (int p = 0; p < 3; ++p) {
        for (int k = 0; k < 3; ++k) {
            rb[p][k] = (k == p) ? 1.0 - 2.0 * a : a;
            rb[p + 3][k] = (k == p) ? 1.0 - 2.0 * b : b;
        }
        rw[p] = wa;
        rw[p + 3] = wb;
    }
    rule_ready = 1;
}

void orc_regular_rule(double *bary, double *w)
{
    init_rule();
    for (int p = 0; p < 6; ++p) {
        for (int k = 0; k < 3; ++k) bary[3 * p + k] = rb[p][k];
        w[p] = rw[p];
    }
}

/* n-point Gauss-Legendre rule on [0,1]: Newton iteration on the Legendre
 * polynomial P_n evaluated by its three-term recurrence. */
static void legendre(int n, double z, double *pn, double *pm)
{
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    *pn = p1;   /* P_n   */
    *pm = p0;   /* P_n-1 */
}

int orc_gauss_legendre01(int n, double *x, double *w)
{
    if (n < 1 || n > 64) return -1;
    for (int i = 0; i < n; ++i) {
        double z = cos(ORC_PI * (i + 0.75) / (n + 0.5));
        double pn, pm, dp;
        for (int it = 0; it < 100; ++it) {
            legendre(n, z, &pn, &pm);
            dp = n * (z * pn - pm) / (z * z - 1.0);
            double dz = pn / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        legendre(n, z, &pn, &pm);
        dp = n * (z * pn - pm) / (z * z - 1.0);
        x[i] = 0.5 * (1.0 - z);                 /* [-1,1] -> [0,1] */
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp); /* half of 2/((1-z^2) P_n'^2) */
    }
    return 0;
}

/* --------------------------------------------------------------- geometry */

typedef struct {
    double p[3][3];     /* vertex coordinates */
    double n[3];        /* unit normal, (p1-p0) x (p2-p0) normalised */
    double area;
    double curl[3][3];  /* surface curl of the P1 hat of local vertex k */
    int v[3];
} otri;

static void tri_geom(const double *xyz, const int32_t *tri, int t, otri *o)
{
    for (int k = 0; k < 3; ++k) {
        o->v[k] = tri[3 * t + k];
        for (int c = 0; c < 3; ++c) o->p[k][c] = xyz[3 * o->v[k] + c];
    }
    double e1[3], e2[3], cr[3];
    for (int c = 0; c < 3; ++c) {
        e1[c] = o->p[1][c] - o->p[0][c];
        e2[c] = o->p[2][c] - o->p[0][c];
    }
    cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
    cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
    cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double len = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    o->area = 0.5 * len;
    for (int c = 0; c < 3; ++c) o->n[c] = cr[c] / len;
    /* curl of hat k = n x grad(lambda_k) = -(p_{k+2} - p_{k+1}) / (2 area) */
    for (int k = 0; k < 3; ++k) {
        int a = (k + 1) % 3, b = (k + 2) % 3;
        for (int c = 0; c < 3; ++c)
            o->curl[k][c] = -(o->p[b][c] - o->p[a][c]) / (2.0 * o->area);
    }
}

void orc_triangle_geometry(const double *xyz, const int32_t *tri, int nt,
                           double *area, double *normal)
{
    for (int t = 0; t < nt; ++t) {
        otri o;
        tri_geom(xyz, tri, t, &o);
        area[t] = o.area;
        for (int c = 0; c < 3; ++c) normal[3 * t + c] = o.n[c];
    }
}

/* ----------------------------------------------------------------- kernels */

/* kernel_mode 0: g = G(x,y) = exp(-kappa r)/(4 pi r),
 *                d = dG/dn_y = exp(-kappa r)(1 + kappa r) ((x-y).n_y)/(4 pi r^3).
 * kernel_mode 1 and 2: smooth polynomial test kernels (same code path through
 * the quadrature), used only to check that the singular rules integrate
 * polynomials exactly:
 *   mode 1: g = 1 + |x-y|^2,            d = x0*y1 + 2*x2*y2
 *   mode 2: g = x0*x1 + y2*y2 - x1*y0,  d = (x-y).n_y                         */
static inline void kern(int mode, const double *x, const double *y, const double *ny,
                        double kappa, double *g, double *d)
{
    double d0 = x[0] - y[0], d1 = x[1] - y[1], d2 = x[2] - y[2];
    if (mode == 0) {
        double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        double e = exp(-kappa * r);
        double dn = d0 * ny[0] + d1 * ny[1] + d2 * ny[2];
        *g = e / (4.0 * ORC_PI * r);
        *d = e * (1.0 + kappa * r) * dn / (4.0 * ORC_PI * r * r * r);
    } else if (mode == 1) {
        *g = 1.0 + d0 * d0 + d1 * d1 + d2 * d2;
        *d = x[0] * y[1] + 2.0 * x[2] * y[2];
    } else {
        *g = x[0] * x[1] + y[2] * y[2] - x[1] * y[0];
        *d = d0 * ny[0] + d1 * ny[1] + d2 * ny[2];
    }
}

/* ------------------------------------------------- regular pair quadrature */

static void block_regular(const otri *t, const otri *s, double kappa, int mode,
                          double *V, double *K)
{
    for (int i = 0; i < 9; ++i) V[i] = K[i] = 0.0;
    for (int p = 0; p < 6; ++p) {
        double x[3];
        for (int c = 0; c < 3; ++c)
            x[c] = rb[p][0] * t->p[0][c] + rb[p][1] * t->p[1][c] + rb[p][2] * t->p[2][c];
        for (int q = 0; q < 6; ++q) {
            double y[3];
            for (int c = 0; c < 3; ++c)
                y[c] = rb[q][0] * s->p[0][c] + rb[q][1] * s->p[1][c] + rb[q][2] * s->p[2][c];
            double g, d;
            kern(mode, x, y, s->n, kappa, &g, &d);
            double w = rw[p] * rw[q] * t->area * s->area;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) {
                    double bb = w * rb[p][k] * rb[q][l];
                    V[3 * k + l] += bb * g;
                    K[3 * k + l] += bb * d;
                }
        }
    }
}

/* One-point rule (the centroid, weight |t| |s|, every hat 1/3 there): the
 * relaxed regular quadrature of the fast Calderon preconditioner (Discussion,
 * fast Calderon preconditioning). */
static void block_centroid(const otri *t, const otri *s, double kappa, int mode, double *V, double *K)
{
    double x[3], y[3], g, d;
    for (int c = 0; c < 3; ++c) {
        x[c] = (t->p[0][c] + t->p[1][c] + t->p[2][c]) / 3.0;
        y[c] = (s->p[0][c] + s->p[1][c] + s->p[2][c]) / 3.0;
    }
    kern(mode, x, y, s->n, kappa, &g, &d);
    double w = t->area * s->area / 9.0;
    for (int i = 0; i < 9; ++i) {
        V[i] = w * g;
        K[i] = w * d;
    }
}

/* ------------------------------------------ Sauter-Schwab singular quadrature
 *
 * (S. Sauter and C. Schwab, Boundary Element Methods, Springer 2011, sec. 5.2.)
 * Reference triangle {0 <= xh2 <= xh1 <= 1} with chi(xh) = A0 + xh1 (A1 - A0)
 * + xh2 (A2 - A1) for the arranged vertices (A0, A1, A2); the hats of A0, A1, A2
 * are (1 - xh1, xh1 - xh2, xh2) there and the surface element is 2|T| dxh.
 *
 * Arrangement of the two triangles (the reading used throughout): the vertices
 * both triangles share come first and in the same order on both, the free ones
 * after them; the test triangle is only rotated (its leading shared vertices
 * follow its own counter-clockwise order), the trial triangle is arranged to
 * match.  Two identical triangles keep their stored order.  Normals are always
 * the stored outward ones, whatever the arrangement.
 *
 * Each case splits the unit hypercube of (xi, eta1, eta2, eta3) into regions;
 * region r maps onto a pair of reference points xh = xi (X1, X2) and
 * yh = xi (Y1, Y2) with the Jacobian xi^3 J(eta), which cancels the 1/r
 * singularity at the shared set. */

/* The three cyclic rotations first, then the three reflections. */
static const int arrangement[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {0, 2, 1}, {2, 1, 0}, {1, 0, 2}};

static int slot_of(const otri *o, int vertex)
{
    for (int k = 0; k < 3; ++k)
        if (o->v[k] == vertex) return k;
    return -1;
}

/* The arrangement above, found by search: the first rotation of the test
 * triangle whose leading vertices are all shared, then the first arrangement
 * of the trial triangle (a rotation when one vertex is shared) that starts
 * with the same shared vertices in the same order.  Returns the number of
 * shared vertices; at[m] / as[m] = stored slot of arranged vertex m. */
static int arrange_pair(const otri *t, const otri *s, int same, int at[3], int as[3])
{
    int common = 0;
    for (int k = 0; k < 3; ++k) common += slot_of(s, t->v[k]) >= 0;
    if (same) common = 3;
    for (int m = 0; m < 3; ++m) at[m] = as[m] = m;
    if (common == 0 || common == 3) return common;
    for (int r = 0; r < 3; ++r) {
        int lead_shared = 1;
        for (int m = 0; m < common; ++m) lead_shared &= slot_of(s, t->v[arrangement[r][m]]) >= 0;
        if (lead_shared) {
            for (int m = 0; m < 3; ++m) at[m] = arrangement[r][m];
            break;
        }
    }
    const int tries = (common == 1) ? 3 : 6;
    for (int r = 0; r < tries; ++r) {
        int match = 1;
        for (int m = 0; m < common; ++m) match &= s->v[arrangement[r][m]] == t->v[at[m]];
        if (match) {
            for (int m = 0; m < 3; ++m) as[m] = arrangement[r][m];
            break;
        }
    }
    return common;
}

/* Region r of the case with `common` shared vertices at (eta1, eta2, eta3):
 * fills X, Y (the bracketed factors of xh and yh) and returns J(eta). */
static double region(int common, int r, double eta1, double eta2, double eta3, double X[2], double Y[2])
{
    if (common == 3) {                 /* identical triangles, six regions */
        switch (r) {
        case 0: X[0] = 1; X[1] = 1 - eta1 + eta1 * eta2;
                Y[0] = 1 - eta1 * eta2 * eta3; Y[1] = 1 - eta1; break;
        case 1: X[0] = 1 - eta1 * eta2 * eta3; X[1] = 1 - eta1;
                Y[0] = 1; Y[1] = 1 - eta1 + eta1 * eta2; break;
        case 2: X[0] = 1; X[1] = eta1 * (1 - eta2 + eta2 * eta3);
                Y[0] = 1 - eta1 * eta2; Y[1] = eta1 * (1 - eta2); break;
        case 3: X[0] = 1 - eta1 * eta2; X[1] = eta1 * (1 - eta2);
                Y[0] = 1; Y[1] = eta1 * (1 - eta2 + eta2 * eta3); break;
        case 4: X[0] = 1 - eta1 * eta2 * eta3; X[1] = eta1 * (1 - eta2 * eta3);
                Y[0] = 1; Y[1] = eta1 * (1 - eta2); break;
        default: X[0] = 1; X[1] = eta1 * (1 - eta2);
                 Y[0] = 1 - eta1 * eta2 * eta3; Y[1] = eta1 * (1 - eta2 * eta3); break;
        }
        return eta1 * eta1 * eta2;
    }
    if (common == 2) {                 /* shared edge xh2 = 0, five regions */
        switch (r) {
        case 0: X[0] = 1; X[1] = eta1 * eta3;
                Y[0] = 1 - eta1 * eta2; Y[1] = eta1 * (1 - eta2);
                return eta1 * eta1;
        case 1: X[0] = 1; X[1] = eta1;
                Y[0] = 1 - eta1 * eta2 * eta3; Y[1] = eta1 * eta2 * (1 - eta3); break;
        case 2: X[0] = 1 - eta1 * eta2; X[1] = eta1 * (1 - eta2);
                Y[0] = 1; Y[1] = eta1 * eta2 * eta3; break;
        case 3: X[0] = 1 - eta1 * eta2 * eta3; X[1] = eta1 * eta2 * (1 - eta3);
                Y[0] = 1; Y[1] = eta1; break;
        default: X[0] = 1 - eta1 * eta2 * eta3; X[1] = eta1 * (1 - eta2 * eta3);
                 Y[0] = 1; Y[1] = eta1 * eta2; break;
        }
        return eta1 * eta1 * eta2;
    }
    /* shared vertex xh = 0, two regions */
    if (r == 0) { X[0] = 1; X[1] = eta1; Y[0] = eta2; Y[1] = eta2 * eta3; }
    else        { X[0] = eta2; X[1] = eta2 * eta3; Y[0] = 1; Y[1] = eta1; }
    return eta2;
}

static void block_singular(const otri *t, const otri *s, int same, double kappa, int mode,
                           int nss, double *V, double *K)
{
    int at[3], as[3];
    const int common = arrange_pair(t, s, same, at, as);
    const int nregions = (common == 3) ? 6 : (common == 2) ? 5 : 2;
    double gx[64], gw[64];
    orc_gauss_legendre01(nss, gx, gw);
    double A[3][3], B[3][3];           /* arranged vertices of the test / trial triangle */
    for (int m = 0; m < 3; ++m)
        for (int c = 0; c < 3; ++c) { A[m][c] = t->p[at[m]][c]; B[m][c] = s->p[as[m]][c]; }
    double sumV[3][3] = {{0}}, sumK[3][3] = {{0}};   /* indexed by arranged vertices */
    for (int r = 0; r < nregions; ++r)
        for (int i = 0; i < nss; ++i)
            for (int j = 0; j < nss; ++j)
                for (int k = 0; k < nss; ++k)
                    for (int l = 0; l < nss; ++l) {
                        const double xi = gx[i];
                        double X[2], Y[2];
                        const double J = region(common, r, gx[j], gx[k], gx[l], X, Y);
                        const double wt = gw[i] * gw[j] * gw[k] * gw[l] * xi * xi * xi * J;
                        const double xh1 = xi * X[0], xh2 = xi * X[1];
                        const double yh1 = xi * Y[0], yh2 = xi * Y[1];
                        const double hx[3] = {1.0 - xh1, xh1 - xh2, xh2};
                        const double hy[3] = {1.0 - yh1, yh1 - yh2, yh2};
                        double x[3], y[3];
                        for (int c = 0; c < 3; ++c) {
                            x[c] = hx[0] * A[0][c] + hx[1] * A[1][c] + hx[2] * A[2][c];
                            y[c] = hy[0] * B[0][c] + hy[1] * B[1][c] + hy[2] * B[2][c];
                        }
                        double g, d;
                        kern(mode, x, y, s->n, kappa, &g, &d);
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b) {
                                sumV[a][b] += wt * hx[a] * hy[b] * g;
                                sumK[a][b] += wt * hx[a] * hy[b] * d;
                            }
                    }
    /* (2|t|)(2|s|) surface elements; arranged vertex a of t is stored slot at[a] */
    const double jac = 4.0 * t->area * s->area;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            V[3 * at[a] + as[b]] = jac * sumV[a][b];
            K[3 * at[a] + as[b]] = jac * sumK[a][b];
        }
}

/* Local blocks of the ordered pair (test t, trial s):
 *   V[3k+l] = int_t int_s lambda_k(x) g(x,y) lambda_l(y),
 *   K[3k+l] = int_t int_s lambda_k(x) d(x,y) lambda_l(y).
 * quad_mode 0: singular rule with nss points per dimension when the pair shares
 * a vertex, regular rule otherwise; quad_mode 1: regular rule always;
 * quad_mode 2: as 0 with the one-point rule in place of the regular rule.
 * Returns the number of shared vertices. */
int orc_pair_block(const double *xyz, const int32_t *tri, int t, int s, double kappa,
                   int nss, int kernel_mode, int quad_mode, double *V, double *K)
{
    init_rule();
    otri ot, os;
    tri_geom(xyz, tri, t, &ot);
    tri_geom(xyz, tri, s, &os);
    int ns = 0;
    if (t == s) ns = 3;
    else
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) ns += (ot.v[k] == os.v[l]);
    if (ns == 0 && quad_mode == 2) block_centroid(&ot, &os, kappa, kernel_mode, V, K);
    else if (ns == 0 || quad_mode == 1) block_regular(&ot, &os, kappa, kernel_mode, V, K);
    else block_singular(&ot, &os, t == s, kappa, kernel_mode, nss, V, K);
    return ns;
}

/* hypersingular block from the single-layer block of the same pair:
 * D[k][l] = (curl_k(t) . curl_l(s)) * sum(V) + kappa^2 (n_t . n_s) V[k][l] */
static void block_hyper(const otri *t, const otri *s, double kappa, const double *V, double *D)
{
    double S = 0.0;
    for (int i = 0; i < 9; ++i) S += V[i];
    double nn = t->n[0] * s->n[0] + t->n[1] * s->n[1] + t->n[2] * s->n[2];
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
            double cc = t->curl[k][0] * s->curl[l][0] + t->curl[k][1] * s->curl[l][1] +
                        t->curl[k][2] * s->curl[l][2];
            D[3 * k + l] = cc * S + kappa * kappa * nn * V[3 * k + l];
        }
}

/* ---------------------------------------------------------- operator rows */

/* vertex -> incident triangles (plain O(T) scan) */
/* triangles incident to vertex v; out NULL: count only */
static int incident(const int32_t *tri, int nt, int v, int *out)
{
    int n = 0;
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k)
            if (tri[3 * t + k] == v) {
                if (out) out[n] = t;
                ++n;
            }
    return n;
}

/* For each requested vertex i = rows[r]:
 *   mode 0 (rows)   : outX[r*nv + j] = X_ij, i the test vertex;
 *   mode 1 (columns): outX[r*nv + j] = X_ji, i the trial vertex.
 * X in {V, K, D} for the kernel with screening kappa (kappa = 0: Laplace);
 * any output pointer may be NULL; quad_mode as for orc_pair_block (0 or 2).
 * Rows are independent and computed in parallel. */
void orc_operator_rows(int nv, int nt, const double *xyz, const int32_t *tri, double kappa,
                       int nss, int nrows, const int32_t *rows, int mode,
                       double *outV, double *outK, double *outD, int quad_mode)
{
    init_rule();
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < nrows; ++r) {
        int i = rows[r];
        const int ni = incident(tri, nt, i, NULL);
        int *inc = (int *)malloc(sizeof(int) * (ni > 0 ? ni : 1));
        incident(tri, nt, i, inc);
        if (outV) memset(outV + (size_t)r * nv, 0, sizeof(double) * nv);
        if (outK) memset(outK + (size_t)r * nv, 0, sizeof(double) * nv);
        if (outD) memset(outD + (size_t)r * nv, 0, sizeof(double) * nv);
        for (int a = 0; a < ni; ++a) {
            int fixed = inc[a];
            otri of;
            tri_geom(xyz, tri, fixed, &of);
            int kf = 0;
            for (int k = 0; k < 3; ++k) if (of.v[k] == i) kf = k;
            for (int other = 0; other < nt; ++other) {
                int t = (mode == 0) ? fixed : other;
                int s = (mode == 0) ? other : fixed;
                double V[9], K[9], D[9];
                orc_pair_block(xyz, tri, t, s, kappa, nss, 0, quad_mode, V, K);
                otri ot, os;
                tri_geom(xyz, tri, t, &ot);
                tri_geom(xyz, tri, s, &os);
                if (outD) block_hyper(&ot, &os, kappa, V, D);
                for (int m = 0; m < 3; ++m) {
                    int idx = (mode == 0) ? 3 * kf + m : 3 * m + kf;
                    int j = (mode == 0) ? os.v[m] : ot.v[m];
                    if (outV) outV[(size_t)r * nv + j] += V[idx];
                    if (outK) outK[(size_t)r * nv + j] += K[idx];
                    if (outD) outD[(size_t)r * nv + j] += D[idx];
                }
            }
        }
        free(inc);
    }
}

/* rows of the P1 mass matrix M_ij = int phi_i phi_j = sum_t |t|/12 (1 + delta_kl) */
void orc_mass_rows(int nv, int nt, const double *xyz, const int32_t *tri, int nrows,
                   const int32_t *rows, double *out)
{
    for (int r = 0; r < nrows; ++r) {
        int i = rows[r];
        memset(out + (size_t)r * nv, 0, sizeof(double) * nv);
        for (int t = 0; t < nt; ++t) {
            otri o;
            int kf = -1;
            for (int k = 0; k < 3; ++k) if (tri[3 * t + k] == i) kf = k;
            if (kf < 0) continue;
            tri_geom(xyz, tri, t, &o);
            for (int l = 0; l < 3; ++l)
                out[(size_t)r * nv + o.v[l]] += o.area / 12.0 * (l == kf ? 2.0 : 1.0);
        }
    }
}

/* ------------------------------------------------------------------- RHS
 * Eq. sources: phi_D(x) = sum_j q_j / (4 pi eps_in |x - x_j|),
 *              phi_N(x) = d/dn_x of the same = -sum_j q_j (x - x_j).n_x / (4 pi eps_in |x - x_j|^3).
 * Tested with the P1 basis using the regular rule:
 *   bD_i = sum_{t ni i} sum_p w_p |t| lambda_i(x_p) phi_D(x_p), likewise bN. */
void orc_rhs(int nv, int nt, const double *xyz, const int32_t *tri, int nq,
             const double *qxyz, const double *q, double eps_in, double *bD, double *bN)
{
    init_rule();
    double *fD = (double *)malloc(sizeof(double) * 6 * nt);
    double *fN = (double *)malloc(sizeof(double) * 6 * nt);
#pragma omp parallel for schedule(static)
    for (int t = 0; t < nt; ++t) {
        otri o;
        tri_geom(xyz, tri, t, &o);
        for (int p = 0; p < 6; ++p) {
            double x[3];
            for (int c = 0; c < 3; ++c)
                x[c] = rb[p][0] * o.p[0][c] + rb[p][1] * o.p[1][c] + rb[p][2] * o.p[2][c];
            double sD = 0.0, sN = 0.0;
            for (int j = 0; j < nq; ++j) {
                double d0 = x[0] - qxyz[3 * j], d1 = x[1] - qxyz[3 * j + 1], d2 = x[2] - qxyz[3 * j + 2];
                double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                sD += q[j] / (4.0 * ORC_PI * eps_in * r);
                sN += -q[j] * (d0 * o.n[0] + d1 * o.n[1] + d2 * o.n[2]) / (4.0 * ORC_PI * eps_in * r * r * r);
            }
            fD[6 * t + p] = sD;
            fN[6 * t + p] = sN;
        }
    }
    memset(bD, 0, sizeof(double) * nv);
    memset(bN, 0, sizeof(double) * nv);
    for (int t = 0; t < nt; ++t) {
        otri o;
        tri_geom(xyz, tri, t, &o);
        for (int p = 0; p < 6; ++p)
            for (int k = 0; k < 3; ++k) {
                double w = rw[p] * o.area * rb[p][k];
                bD[o.v[k]] += w * fD[6 * t + p];
                bN[o.v[k]] += w * fN[6 * t + p];
            }
    }
    free(fD);
    free(fN);
}

/* ------------------------------------------------------ reaction potential
 * Eq. phireac_bie: phi_reac(x) = V_int[dphi](x) - K_int[phi](x), with the
 * Laplace kernel, phi and dphi the P1 interpolants of the interior traces,
 * integrated with the regular rule:
 *   phi_reac(x) = sum_t sum_p w_p |t| [ G(x,y_p) dphi(y_p) - dG/dn_y(x,y_p) phi(y_p) ]. */
void orc_reaction_potential(int nv, int nt, const double *xyz, const int32_t *tri,
                            const double *phi, const double *dphi, int npts,
                            const double *pts, double *out)
{
    init_rule();
    (void)nv;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < npts; ++k) {
        const double *x = pts + 3 * k;
        double acc = 0.0;
        for (int t = 0; t < nt; ++t) {
            otri o;
            tri_geom(xyz, tri, t, &o);
            for (int p = 0; p < 6; ++p) {
                double y[3], u = 0.0, du = 0.0;
                for (int c = 0; c < 3; ++c)
                    y[c] = rb[p][0] * o.p[0][c] + rb[p][1] * o.p[1][c] + rb[p][2] * o.p[2][c];
                for (int m = 0; m < 3; ++m) {
                    u += rb[p][m] * phi[o.v[m]];
                    du += rb[p][m] * dphi[o.v[m]];
                }
                double g, d;
                kern(0, x, y, o.n, 0.0, &g, &d);
                acc += rw[p] * o.area * (g * du - d * u);
            }
        }
        out[k] = acc;
    }
}
