// Host-side index work for a mesh handle: argument and mesh validation, a
// Morton ordering of the triangles (so that spatially close triangles share a
// wavefront in the far-field kernels), vertex -> triangle incidence, the
// near-pair lists and the sparsity pattern of the near-field vertex blocks.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>
#include <numeric>
#include <system_error>
#include <thread>

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

// Contiguous row ranges of a host loop run on worker threads; the callers
// write disjoint outputs per row (or per worker, joined in row order), so the
// result does not depend on the number of workers.
constexpr int kPrepMaxThreads = 16;
constexpr int kPrepMinRows = 4096;

static int prep_workers(int n, int min_rows)
{
    const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
    return std::max(1, std::min({kPrepMaxThreads, hw, n / min_rows}));
}

// fn(worker, begin, end) over nw contiguous ranges of [0, n); an exception in a
// worker is rethrown on the calling thread.  A range whose thread cannot be
// started runs on the calling thread.
template <typename F>
static void parallel_chunks(int n, int nw, F &&fn)
{
    if (nw <= 1) { fn(0, 0, n); return; }
    std::vector<std::thread> th;
    th.reserve(nw);
    std::exception_ptr err;
    std::mutex mu;
    auto run = [&](int w, int b, int e) {
        try {
            fn(w, b, e);
        } catch (...) {
            std::lock_guard<std::mutex> lk(mu);
            if (!err) err = std::current_exception();
        }
    };
    for (int w = 0; w < nw; ++w) {
        const int b = (int)((int64_t)n * w / nw), e = (int)((int64_t)n * (w + 1) / nw);
        bool started = false;
        try {
            th.emplace_back(run, w, b, e);
            started = true;
        } catch (const std::system_error &) {
        }
        if (!started) run(w, b, e);
    }
    for (auto &t : th) t.join();
    if (err) std::rethrow_exception(err);
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

    // near pairs: for each t, every s sharing at least one vertex (incl. t),
    // ascending
    hm.pair_ptr.assign(T + 1, 0);
    {
        std::vector<std::vector<int32_t>> part(prep_workers(T, kPrepMinRows));
        std::vector<int32_t> cnt(T);
        parallel_chunks(T, (int)part.size(), [&](int w, int b, int e) {
            std::vector<int32_t> stamp(T, -1), buf;
            auto &out = part[w];
            out.reserve(14 * (size_t)(e - b));
            for (int t = b; t < e; ++t) {
                buf.clear();
                for (int k = 0; k < 3; ++k) {
                    const int v = hm.tri[3 * t + k];
                    for (int e2 = hm.inc_ptr[v]; e2 < hm.inc_ptr[v + 1]; ++e2) {
                        const int s = hm.inc_tk[e2] >> 2;
                        if (stamp[s] != t) { stamp[s] = t; buf.push_back(s); }
                    }
                }
                std::sort(buf.begin(), buf.end());
                out.insert(out.end(), buf.begin(), buf.end());
                cnt[t] = (int32_t)buf.size();
            }
        });
        size_t np = 0;
        for (int t = 0; t < T; ++t) np += (size_t)cnt[t];
        if (np > (size_t)INT32_MAX / 2) fail(PB_E_INVALID_ARG, "mesh too large");
        for (int t = 0; t < T; ++t) hm.pair_ptr[t + 1] = hm.pair_ptr[t] + cnt[t];
        hm.pair_s.clear();
        hm.pair_s.reserve(np);
        for (auto &v : part) hm.pair_s.insert(hm.pair_s.end(), v.begin(), v.end());
    }
    const size_t np = hm.pair_s.size();
    hm.pair_rev.resize(np);
    parallel_chunks(T, prep_workers(T, kPrepMinRows), [&](int, int b, int e) {
        for (int t = b; t < e; ++t)
            for (int p = hm.pair_ptr[t]; p < hm.pair_ptr[t + 1]; ++p) {
                const int s = hm.pair_s[p];
                auto bs = hm.pair_s.begin() + hm.pair_ptr[s], es = hm.pair_s.begin() + hm.pair_ptr[s + 1];
                hm.pair_rev[p] = (int32_t)(std::lower_bound(bs, es, t) - hm.pair_s.begin());
            }
    });

    // Near vertex CSR: j appears in row i if some near pair (t ni i, s ni j)
    // does; columns ascending.  Per nonzero slot (i, j), its contributions
    // (near pair p, local vertex k of i in t, local vertex l of j in s) in the
    // order row i visits them -- incidence, pair, l -- as codes
    // p << 4 | k << 2 | l.  Each worker builds its rows' columns, slot counts
    // and codes; the parts are joined in row order.
    if (np >= ((size_t)1 << 28)) fail(PB_E_INVALID_ARG, "mesh too large");
    {
        struct Rows {
            std::vector<int32_t> ncol, col, diag, scount;
            std::vector<uint32_t> code;
        };
        std::vector<Rows> part(prep_workers(V, kPrepMinRows));
        parallel_chunks(V, (int)part.size(), [&](int w, int b, int e) {
            std::vector<int32_t> stamp(V, -1), pos(V, 0), buf, off;
            Rows &r = part[w];
            r.col.reserve(20 * (size_t)(e - b));
            r.scount.reserve(20 * (size_t)(e - b));
            r.code.reserve(240 * (size_t)(e - b));
            auto visit = [&](int i, auto &&f) {
                for (int e2 = hm.inc_ptr[i]; e2 < hm.inc_ptr[i + 1]; ++e2) {
                    const int t = hm.inc_tk[e2] >> 2, k = hm.inc_tk[e2] & 3;
                    for (int p = hm.pair_ptr[t]; p < hm.pair_ptr[t + 1]; ++p) {
                        const int s = hm.pair_s[p];
                        for (int l = 0; l < 3; ++l) f(hm.tri[3 * s + l], ((uint32_t)p << 4) | ((uint32_t)k << 2) | (uint32_t)l);
                    }
                }
            };
            for (int i = b; i < e; ++i) {
                buf.clear();
                visit(i, [&](int j, uint32_t) {
                    if (stamp[j] != i) { stamp[j] = i; buf.push_back(j); }
                });
                std::sort(buf.begin(), buf.end());
                const int nc = (int)buf.size();
                for (int a = 0; a < nc; ++a) pos[buf[a]] = a;
                r.ncol.push_back(nc);
                r.diag.push_back(pos[i]);
                r.col.insert(r.col.end(), buf.begin(), buf.end());
                off.assign(nc + 1, 0);
                visit(i, [&](int j, uint32_t) { off[pos[j] + 1]++; });
                for (int a = 0; a < nc; ++a) {
                    r.scount.push_back(off[a + 1]);
                    off[a + 1] += off[a];
                }
                const size_t base = r.code.size();
                r.code.resize(base + (size_t)off[nc]);
                visit(i, [&](int j, uint32_t c) { r.code[base + (size_t)off[pos[j]]++] = c; });
            }
        });
        // each worker's first row, column and code in the joined arrays
        const int nw = (int)part.size();
        std::vector<size_t> r0(nw + 1, 0), c0(nw + 1, 0), k0(nw + 1, 0);
        for (int w = 0; w < nw; ++w) {
            r0[w + 1] = r0[w] + part[w].ncol.size();
            c0[w + 1] = c0[w] + part[w].col.size();
            k0[w + 1] = k0[w] + part[w].code.size();
        }
        if (c0[nw] > (size_t)INT32_MAX || k0[nw] > (size_t)INT32_MAX) fail(PB_E_INVALID_ARG, "mesh too large");
        hm.row_ptr.assign(V + 1, 0);
        hm.diag_slot.resize(V);
        hm.col.resize(c0[nw]);
        hm.slot_ptr.resize(c0[nw] + 1);
        hm.slot_code.resize(k0[nw]);
        hm.slot_ptr[0] = 0;
        parallel_chunks(nw, nw, [&](int, int b, int e) {
            for (int w = b; w < e; ++w) {
                const Rows &r = part[w];
                int32_t rp = (int32_t)c0[w];
                for (size_t a = 0; a < r.ncol.size(); ++a) {
                    hm.diag_slot[r0[w] + a] = rp + r.diag[a];
                    rp += r.ncol[a];
                    hm.row_ptr[r0[w] + a + 1] = rp;
                }
                std::copy(r.col.begin(), r.col.end(), hm.col.begin() + c0[w]);
                std::copy(r.code.begin(), r.code.end(), hm.slot_code.begin() + k0[w]);
                int32_t sp = (int32_t)k0[w];
                for (size_t a = 0; a < r.scount.size(); ++a) {
                    sp += r.scount[a];
                    hm.slot_ptr[c0[w] + a + 1] = sp;
                }
            }
        });
    }
}

}  // namespace pbm
