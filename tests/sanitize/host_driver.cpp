// Runs the library's host-side mesh preparation (validation, Morton order,
// incidences, near pairs, near-field sparsity and contribution lists) on a
// closed bipyramid with two vertices of valence 80 and on malformed meshes,
// built for AddressSanitizer and UndefinedBehaviorSanitizer (host code only).
// The malformed meshes must be rejected with PB_E_MESH or PB_E_INVALID_ARG.
// Prints "ok" and exits 0 when every case behaves.
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
