// Host-side index work for a mesh handle: argument and mesh validation, a
// Morton ordering of the triangles (so that spatially close triangles share a
// wavefront in the far-field kernels), vertex -> triangle incidence, the
// near-pair lists and the sparsity pattern of the near-field vertex blocks.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "pbm_internal.h"

namespace pbm {

// Gauss-Legendre nodes and weights by Golub-Welsch: the nodes are the
// eigenvalues of the symmetric tridiagonal Jacobi matrix of the Legendre
// recurrence (off-diagonal k / sqrt(4k^2 - 1)), the weights 2 v_0^2 from the
// normalised eigenvectors.  The eigenproblem is solved by cyclic Jacobi
// rotations, ample for n <= 32.
void gauss_legendre01(int n, double *x, double *w)
{
    if (n < 1 || n > 32) fail(PB_E_INVALID_ARG, "singular_order must be in [1, 32]");
    std::vector<double> A(n * n, 0.0), Q(n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
    for (int k = 1; k < n; ++k) {
        double b = k / std::sqrt(4.0 * k * k - 1.0);
        A[(k - 1) * n + k] = A[k * n + (k - 1)] = b;
    }
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
        if (off < 1e-34) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {   // A <- A J
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {   // A <- J^T A
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {   // Q <- Q J
                    double qkp = Q[k * n + p], qkq = Q[k * n + q];
                    Q[k * n + p] = c * qkp - s * qkq;
                    Q[k * n + q] = s * qkp + c * qkq;
                }
            }
    }
    std::vector<std::pair<double, double>> nw(n);
    for (int i = 0; i < n; ++i) nw[i] = {A[i * n + i], 2.0 * Q[0 * n + i] * Q[0 * n + i]};
    std::sort(nw.begin(), nw.end());
    for (int i = 0; i < n; ++i) {
        x[i] = 0.5 * (nw[i].first + 1.0);
        w[i] = 0.5 * nw[i].second;
    }
}

static uint32_t spread10(uint32_t v)
{
    v &= 1023u;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

void build_host_mesh(const pb_mesh *m, HostMesh &hm)
{
    if (!m || !m->xyz || !m->tri) fail(PB_E_INVALID_ARG, "mesh pointers must not be NULL");
    const int V = m->n_vertices, T = m->n_triangles;
    if (V < 4 || T < 4) fail(PB_E_MESH, "a closed surface needs at least 4 vertices and 4 triangles");
    if ((int64_t)T > (int64_t)1 << 28) fail(PB_E_INVALID_ARG, "too many triangles");
    hm.V = V;
    hm.T = T;
    hm.xyz.assign(m->xyz, m->xyz + 3 * (size_t)V);
    for (double v : hm.xyz)
        if (!std::isfinite(v)) fail(PB_E_INVALID_ARG, "vertex coordinates must be finite");
    const int32_t *tri = m->tri;
    for (int64_t i = 0; i < 3 * (int64_t)T; ++i)
        if (tri[i] < 0 || tri[i] >= V) fail(PB_E_MESH, "triangle vertex id out of range");

    // closed, oriented 2-manifold: every directed edge once, its reverse once
    std::vector<uint64_t> e(3 * (size_t)T);
    for (int t = 0; t < T; ++t) {
        int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
        if (a == b || b == c || a == c) fail(PB_E_MESH, "triangle with a repeated vertex");
        e[3 * t] = (uint64_t)a * V + b;
        e[3 * t + 1] = (uint64_t)b * V + c;
        e[3 * t + 2] = (uint64_t)c * V + a;
    }
    std::vector<uint64_t> es(e);
    std::sort(es.begin(), es.end());
    for (size_t i = 1; i < es.size(); ++i)
        if (es[i] == es[i - 1]) fail(PB_E_MESH, "directed edge used twice: non-manifold or inconsistently oriented mesh");
    for (uint64_t k : es) {
        uint64_t rev = (k % V) * V + k / V;
        if (!std::binary_search(es.begin(), es.end(), rev))
            fail(PB_E_MESH, "open mesh or inconsistent orientation (edge without an opposite half-edge)");
    }
    std::vector<int> seen(V, 0);
    for (int64_t i = 0; i < 3 * (int64_t)T; ++i) seen[tri[i]] = 1;
    for (int v = 0; v < V; ++v)
        if (!seen[v]) fail(PB_E_MESH, "vertex not used by any triangle");

    // non-degenerate triangles, positive enclosed volume (outward normals)
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int v = 0; v < V; ++v)
        for (int c = 0; c < 3; ++c) {
            lo[c] = std::min(lo[c], hm.xyz[3 * v + c]);
            hi[c] = std::max(hi[c], hm.xyz[3 * v + c]);
        }
    double diag2 = 0.0;
    for (int c = 0; c < 3; ++c) diag2 += (hi[c] - lo[c]) * (hi[c] - lo[c]);
    double vol = 0.0;
    std::vector<uint64_t> key(T);
    for (int t = 0; t < T; ++t) {
        const double *p0 = &hm.xyz[3 * tri[3 * t]], *p1 = &hm.xyz[3 * tri[3 * t + 1]], *p2 = &hm.xyz[3 * tri[3 * t + 2]];
        double e1[3], e2[3], cr[3];
        for (int c = 0; c < 3; ++c) { e1[c] = p1[c] - p0[c]; e2[c] = p2[c] - p0[c]; }
        cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
        cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
        cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
        double a2 = cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2];
        if (!(a2 > 1e-24 * diag2 * diag2)) fail(PB_E_MESH, "degenerate (zero-area) triangle");
        vol += (p0[0] * cr[0] + p0[1] * cr[1] + p0[2] * cr[2]) / 6.0;
        uint32_t q[3];
        for (int c = 0; c < 3; ++c) {
            double cen = (p0[c] + p1[c] + p2[c]) / 3.0;
            double f = (hi[c] > lo[c]) ? (cen - lo[c]) / (hi[c] - lo[c]) : 0.0;
            q[c] = (uint32_t)std::min(1023.0, std::max(0.0, std::floor(f * 1024.0)));
        }
        key[t] = ((uint64_t)(spread10(q[0]) | (spread10(q[1]) << 1) | (spread10(q[2]) << 2)) << 32) | (uint32_t)t;
    }
    if (!(vol > 0.0)) fail(PB_E_MESH, "inverted mesh: enclosed volume is not positive (normals must point outward)");

    // Morton order of the triangle centroids
    std::sort(key.begin(), key.end());
    hm.perm.resize(T);
    hm.iperm.resize(T);
    hm.mkey.resize(T);
    for (int t = 0; t < T; ++t) hm.mkey[t] = (uint32_t)(key[t] >> 32);
    hm.tri.resize(3 * (size_t)T);
    for (int t = 0; t < T; ++t) {
        int orig = (int)(key[t] & 0xffffffffu);
        hm.perm[t] = orig;
        hm.iperm[orig] = t;
        for (int k = 0; k < 3; ++k) hm.tri[3 * t + k] = tri[3 * orig + k];
    }

    // vertex -> (sorted triangle, local index), triangles ascending
    hm.inc_ptr.assign(V + 1, 0);
    for (int t = 0; t < T; ++t)
        for (int k = 0; k < 3; ++k) hm.inc_ptr[hm.tri[3 * t + k] + 1]++;
    for (int v = 0; v < V; ++v) hm.inc_ptr[v + 1] += hm.inc_ptr[v];
    hm.inc_tk.resize(3 * (size_t)T);
    {
        std::vector<int32_t> fill(hm.inc_ptr.begin(), hm.inc_ptr.end() - 1);
        for (int t = 0; t < T; ++t)
            for (int k = 0; k < 3; ++k) hm.inc_tk[fill[hm.tri[3 * t + k]]++] = 4 * t + k;
    }

    // near pairs: for each t, every s sharing at least one vertex (incl. t)
    hm.pair_ptr.assign(T + 1, 0);
    hm.pair_s.clear();
    hm.pair_s.reserve(14 * (size_t)T);
    std::vector<int32_t> buf;
    for (int t = 0; t < T; ++t) {
        buf.clear();
        for (int k = 0; k < 3; ++k) {
            int v = hm.tri[3 * t + k];
            for (int e2 = hm.inc_ptr[v]; e2 < hm.inc_ptr[v + 1]; ++e2) buf.push_back(hm.inc_tk[e2] >> 2);
        }
        std::sort(buf.begin(), buf.end());
        buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
        hm.pair_s.insert(hm.pair_s.end(), buf.begin(), buf.end());
        hm.pair_ptr[t + 1] = (int32_t)hm.pair_s.size();
    }
    const size_t np = hm.pair_s.size();
    if (np > (size_t)INT32_MAX / 2) fail(PB_E_INVALID_ARG, "mesh too large");
    hm.pair_rev.resize(np);
    for (int t = 0; t < T; ++t)
        for (int p = hm.pair_ptr[t]; p < hm.pair_ptr[t + 1]; ++p) {
            int s = hm.pair_s[p];
            auto b = hm.pair_s.begin() + hm.pair_ptr[s], en = hm.pair_s.begin() + hm.pair_ptr[s + 1];
            auto it = std::lower_bound(b, en, t);
            hm.pair_rev[p] = (int32_t)(it - hm.pair_s.begin());
        }

    // near vertex CSR: j appears in row i if some near pair (t ni i, s ni j)
    hm.row_ptr.assign(V + 1, 0);
    hm.col.clear();
    hm.col.reserve(20 * (size_t)V);
    hm.diag_slot.resize(V);
    for (int i = 0; i < V; ++i) {
        buf.clear();
        for (int e2 = hm.inc_ptr[i]; e2 < hm.inc_ptr[i + 1]; ++e2) {
            int t = hm.inc_tk[e2] >> 2;
            for (int p = hm.pair_ptr[t]; p < hm.pair_ptr[t + 1]; ++p) {
                int s = hm.pair_s[p];
                for (int l = 0; l < 3; ++l) buf.push_back(hm.tri[3 * s + l]);
            }
        }
        std::sort(buf.begin(), buf.end());
        buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
        hm.diag_slot[i] = (int32_t)(hm.col.size() + (std::lower_bound(buf.begin(), buf.end(), i) - buf.begin()));
        hm.col.insert(hm.col.end(), buf.begin(), buf.end());
        hm.row_ptr[i + 1] = (int32_t)hm.col.size();
    }

    // per nonzero slot (i, j), its contributions (near pair p, local vertex k
    // of i in t, local vertex l of j in s) in the order row i visits them --
    // incidence, pair, l -- as codes p << 4 | k << 2 | l
    if (np >= ((size_t)1 << 28)) fail(PB_E_INVALID_ARG, "mesh too large");
    const size_t nnz = hm.col.size();
    hm.slot_ptr.assign(nnz + 1, 0);
    for (int pass = 0; pass < 2; ++pass) {
        std::vector<int32_t> fill;
        if (pass == 1) {
            for (size_t a = 0; a < nnz; ++a) hm.slot_ptr[a + 1] += hm.slot_ptr[a];
            hm.slot_code.assign(hm.slot_ptr[nnz], 0);
            fill.assign(hm.slot_ptr.begin(), hm.slot_ptr.end() - 1);
        }
        for (int i = 0; i < V; ++i) {
            const auto cb = hm.col.begin() + hm.row_ptr[i], ce = hm.col.begin() + hm.row_ptr[i + 1];
            for (int e2 = hm.inc_ptr[i]; e2 < hm.inc_ptr[i + 1]; ++e2) {
                const int t = hm.inc_tk[e2] >> 2, k = hm.inc_tk[e2] & 3;
                for (int p = hm.pair_ptr[t]; p < hm.pair_ptr[t + 1]; ++p) {
                    const int s = hm.pair_s[p];
                    for (int l = 0; l < 3; ++l) {
                        const size_t slot = (size_t)(std::lower_bound(cb, ce, hm.tri[3 * s + l]) - hm.col.begin());
                        if (pass == 0) hm.slot_ptr[slot + 1]++;
                        else hm.slot_code[fill[slot]++] = ((uint32_t)p << 4) | ((uint32_t)k << 2) | (uint32_t)l;
                    }
                }
            }
        }
    }
}

}  // namespace pbm
