// Runs the library's host-side mesh preparation (validation, Morton order,
// incidences, near pairs, near-field sparsity and contribution lists) on a
// closed bipyramid with two vertices of valence 80 and on malformed meshes,
// built for AddressSanitizer and UndefinedBehaviorSanitizer (host code only).
// The malformed meshes must be rejected with PB_E_MESH or PB_E_INVALID_ARG.
// Prints "ok" and exits 0 when every case behaves.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../paper_2108_10481_amd/csrc/pbm_internal.h"

namespace pbm {
// the library's error path (runtime.hip), which the preparation code uses
void fail(pb_status code, const std::string &msg) { throw Error{code, msg}; }
}  // namespace pbm

static std::vector<double> g_xyz;
static std::vector<int32_t> g_tri;

static void bipyramid(int n)
{
    g_xyz = {0.0, 0.0, 1.5, 0.0, 0.0, -1.5};
    for (int i = 0; i < n; ++i) {
        const double a = 2.0 * 3.14159265358979323846 * i / n;
        g_xyz.insert(g_xyz.end(), {std::cos(a), std::sin(a), 0.0});
    }
    g_tri.clear();
    for (int i = 0; i < n; ++i) {
        const int e0 = 2 + i, e1 = 2 + (i + 1) % n;
        g_tri.insert(g_tri.end(), {0, e0, e1, 1, e1, e0});
    }
}

// closed torus (major radius 3, minor 1), n x m vertices, valence 6, outward
// normals; large enough for the preparation's threaded passes
static void torus(int n, int m)
{
    g_xyz.clear();
    g_tri.clear();
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < m; ++j) {
            const double u = 2.0 * 3.14159265358979323846 * i / n, v = 2.0 * 3.14159265358979323846 * j / m;
            g_xyz.insert(g_xyz.end(), {(3.0 + std::cos(v)) * std::cos(u), (3.0 + std::cos(v)) * std::sin(u), std::sin(v)});
        }
    auto id = [&](int i, int j) { return (int32_t)(((i + n) % n) * m + (j + m) % m); };
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < m; ++j) {
            const int32_t a = id(i, j), b = id(i + 1, j), c = id(i + 1, j + 1), d = id(i, j + 1);
            g_tri.insert(g_tri.end(), {a, b, c, a, c, d});
        }
}

// the near-field sparsity and its contribution lists: rows ascending without
// repeats, the diagonal slot on column i, and every contribution code naming
// a near pair (t, s) with vertex i at local k of t and column j at local l of s
static bool csr_consistent(const pbm::HostMesh &hm)
{
    for (int i = 0; i < hm.V; ++i) {
        if (hm.col[hm.diag_slot[i]] != i) return false;
        for (int a = hm.row_ptr[i]; a < hm.row_ptr[i + 1]; ++a) {
            if (a > hm.row_ptr[i] && hm.col[a] <= hm.col[a - 1]) return false;
            if (hm.slot_ptr[a + 1] <= hm.slot_ptr[a]) return false;
            for (int c = hm.slot_ptr[a]; c < hm.slot_ptr[a + 1]; ++c) {
                const uint32_t code = hm.slot_code[c];
                const int p = (int)(code >> 4), k = (code >> 2) & 3, l = code & 3;
                const int t = (int)(std::upper_bound(hm.pair_ptr.begin(), hm.pair_ptr.end(), p) - hm.pair_ptr.begin()) - 1;
                if (hm.tri[3 * t + k] != i || hm.tri[3 * hm.pair_s[p] + l] != hm.col[a]) return false;
            }
        }
    }
    return true;
}

static int run(const char *what, pb_status expect)
{
    pb_mesh m{(int32_t)(g_xyz.size() / 3), (int32_t)(g_tri.size() / 3), g_xyz.data(), g_tri.data()};
    pb_status got = PB_OK;
    try {
        pbm::HostMesh hm;
        pbm::build_host_mesh(&m, hm);
        // every near pair shares a vertex and has its reverse
        for (int t = 0; t < hm.T; ++t)
            for (int p = hm.pair_ptr[t]; p < hm.pair_ptr[t + 1]; ++p)
                if (hm.pair_s[hm.pair_rev[p]] != t) got = PB_E_STATE;
        if (!csr_consistent(hm)) got = PB_E_STATE;
    } catch (const pbm::Error &e) {
        got = e.code;
    }
    if (got != expect) std::printf("%s: status %d, expected %d\n", what, (int)got, (int)expect);
    return got == expect;
}

int main()
{
    int ok = 1;
    bipyramid(80);
    ok &= run("closed bipyramid", PB_OK);
    torus(128, 64);
    ok &= run("closed torus (threaded preparation)", PB_OK);
    bipyramid(80);
    g_tri.resize(g_tri.size() - 3);                       // one triangle missing: open
    ok &= run("open mesh", PB_E_MESH);
    bipyramid(80);
    std::swap(g_tri[1], g_tri[2]);                        // one triangle inverted
    ok &= run("inverted triangle", PB_E_MESH);
    bipyramid(80);
    g_tri[2] = g_tri[1];                                  // repeated vertex
    ok &= run("degenerate triangle", PB_E_MESH);
    bipyramid(80);
    g_tri[4] = (int32_t)(g_xyz.size() / 3) + 7;           // vertex id out of range
    ok &= run("vertex id out of range", PB_E_MESH);
    bipyramid(80);
    g_xyz[5] = std::nan("");                              // non-finite coordinate
    ok &= run("NaN coordinate", PB_E_INVALID_ARG);
    bipyramid(80);
    g_tri.insert(g_tri.end(), g_tri.begin(), g_tri.begin() + 3);   // duplicated triangle: non-manifold
    ok &= run("duplicated triangle", PB_E_MESH);
    std::puts(ok ? "ok" : "failed");
    return ok ? 0 : 1;
}
