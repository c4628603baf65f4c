// Far-field acceleration: a barycentric Lagrange treecode (cluster-particle,
// kernel independent; L. Wang, R. Krasny and S. Tlupova, Commun. Comput. Phys.
// 28 (2020)), the GPU-friendly hierarchical scheme standing in for the
// paper's FMM (Implementation, Results: ExaFMM).
//
// Sources: the 6 regular quadrature points of every triangle with the
// matrix-free weights (b1, b2, curl weights).  A binary tree splits the
// Morton-ordered triangles at the highest differing bit of their Morton codes
// (so every node is an octree-like cell) down to leaves of at most kTreeLeaf
// triangles.  Targets: batches of kTreeBatch consecutive triangles (one
// wavefront, a lane per triangle and its 6 points).  A batch takes a cluster
// through its proxies when r_batch + r_cluster < theta * |c_batch - c_cluster|
// (bounding spheres of the triangles' vertices: triangles sharing a vertex
// never pass, so near pairs are always summed directly) and the cluster has
// more points than proxies; otherwise leaves are summed directly with the
// regular rule, pairs sharing a vertex skipped as in k_far.
//
// Proxies: the (degree+1)^3 tensor Chebyshev points of the second kind on the
// cluster's box.  With L_k the tensor barycentric Lagrange basis, every
// kernel is interpolated in its source variable, G(x, y) ~ sum_k G(x, s_k)
// L_k(y), so per proxy
//   qK = sum_y b1 n_y . grad L_k(y)    (double layer: n_y . grad_y G)
//   qV = sum_y b2 L_k(y)               (single layer; adjoint double layer
//                                       and curl part use the target-side
//                                       kernel at s_k)
//   qC = sum_y w_q C_s L_k(y)          (hypersingular curl part, 3 components)
//   qN = sum_y b1 n_y L_k(y)           (its kappa^2 (n_x . n_y) term)
// and a target point sees every kernel of the formulation evaluated at s_k.
// A batch's interaction list is split into up to `nsplit` pieces of about
// equal work (pieces past a light batch's count stay empty and write zeros);
// each piece writes its own partial sums (the layout of k_far's source
// chunks), which k_far_finish adds in FP64.
#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "far.h"

namespace pbm {

constexpr int kTreeLeaf = 64;
constexpr int kTreeBatch = 64;
constexpr int kTreeBlock = 256;   // four independent wavefronts per block: one-wavefront
                                  // blocks would cap residency at the workgroup slots
constexpr int kMaxPieces = 64;  // pieces of one batch at most
constexpr int kStage = 32;     // near-leaf source records staged per wavefront at a time
constexpr int kProxRec = 12;   // proxy record: position 3, qK, qV, qC 3, qN 3, pad

struct Tree {
    int degree = 0, np = 0, nfar = 0, nbatch = 0, nsplit = 1, nitem = 0;
    double theta = 0.0;
    double evals = 0.0;                 // kernel evaluations per product (point pairs + point-proxy pairs)
    int32_t *node_range = nullptr;      // node -> first, end triangle
    double *box = nullptr;              // node -> centre 3, half-width 3 (interpolation box)
    int32_t *far_node = nullptr;        // far cluster f -> node
    int32_t *far_slot = nullptr;        // far cluster f -> charge slot
    int32_t *piece_ptr = nullptr;       // (batch * nsplit + piece) -> first entry
    int32_t *order = nullptr;           // dispatch order of the (batch, piece) work items, heaviest first
    int32_t *entry = nullptr;           // f << 1 | 1 (proxies of far cluster f) or node << 1 (leaf, direct)
    void *prox = nullptr;               // nfar x np x kProxRec reals (FP64 or FP32 as the handle evaluates)
    int32_t *item = nullptr;            // leaf with charges -> slot, node, first, end triangle
    int32_t *m2m = nullptr;             // parent slot, node, child slots and nodes, deepest level first
    std::vector<int32_t> level_ptr;     // m2m entries per level (host)
    double *charges = nullptr;          // slot x np x 8 proxy charges (FP64)
};

int tree_splits(const Tree &t) { return t.nsplit; }

namespace {

struct Node {
    int b, e, c0 = -1, c1 = -1;
    double lo[3], hi[3];
    double centre(int c) const { return 0.5 * (lo[c] + hi[c]); }
    double radius() const
    {
        double s = 0.0;
        for (int c = 0; c < 3; ++c) s += 0.25 * (hi[c] - lo[c]) * (hi[c] - lo[c]);
        return std::sqrt(s);
    }
};

void tri_box(const HostMesh &hm, int b, int e, double *lo, double *hi)
{
    for (int c = 0; c < 3; ++c) { lo[c] = 1e300; hi[c] = -1e300; }
    for (int t = b; t < e; ++t)
        for (int k = 0; k < 3; ++k) {
            const double *p = &hm.xyz[3 * (size_t)hm.tri[3 * (size_t)t + k]];
            for (int c = 0; c < 3; ++c) { lo[c] = std::min(lo[c], p[c]); hi[c] = std::max(hi[c], p[c]); }
        }
}

}  // namespace

Tree *tree_create(DevMesh &d)
{
    const HostMesh &hm = d.hm;
    const int T = hm.T;
    std::unique_ptr<Tree> tr(new Tree());
    tr->degree = d.opt.tree_degree;
    tr->theta = d.opt.tree_theta;
    const int n1 = tr->degree + 1;
    tr->np = n1 * n1 * n1;

    // source tree
    std::vector<Node> nodes;
    nodes.reserve(4 * (size_t)(T / kTreeLeaf + 1));
    nodes.push_back(Node{0, T});
    for (size_t i = 0; i < nodes.size(); ++i) {
        Node nd = nodes[i];
        tri_box(hm, nd.b, nd.e, nd.lo, nd.hi);
        if (nd.e - nd.b > kTreeLeaf) {
            const uint32_t kb = hm.mkey[nd.b], ke = hm.mkey[nd.e - 1];
            int m = (nd.b + nd.e) / 2;
            if (kb != ke) {
                const int bit = 31 - __builtin_clz(kb ^ ke);
                m = (int)(std::partition_point(hm.mkey.begin() + nd.b, hm.mkey.begin() + nd.e,
                                               [bit](uint32_t k) { return ((k >> bit) & 1u) == 0u; }) -
                          hm.mkey.begin());
                if (m <= nd.b || m >= nd.e) m = (nd.b + nd.e) / 2;
            }
            nd.c0 = (int)nodes.size();
            nd.c1 = nd.c0 + 1;
            nodes.push_back(Node{nd.b, m});
            nodes.push_back(Node{m, nd.e});
        }
        nodes[i] = nd;
    }

    // target batches and their interaction lists
    tr->nbatch = (T + kTreeBatch - 1) / kTreeBatch;
    std::vector<int32_t> far_of(nodes.size(), -1), far_node, list, list_ptr(1, 0);
    std::vector<double> cost, bcost(tr->nbatch);
    std::vector<int> stack;
    double evals = 0.0;
    for (int bt = 0; bt < tr->nbatch; ++bt) {
        const int tb = bt * kTreeBatch, te = std::min(T, tb + kTreeBatch);
        Node bn{tb, te};
        tri_box(hm, tb, te, bn.lo, bn.hi);
        const double rb = bn.radius();
        double total = 0.0;
        stack.assign(1, 0);
        while (!stack.empty()) {
            const int i = stack.back();
            stack.pop_back();
            const Node &nd = nodes[i];
            double dist2 = 0.0;
            for (int c = 0; c < 3; ++c) dist2 += (bn.centre(c) - nd.centre(c)) * (bn.centre(c) - nd.centre(c));
            const bool sep = rb + nd.radius() < tr->theta * std::sqrt(dist2);
            if (sep && 6 * (nd.e - nd.b) > tr->np) {
                if (far_of[i] < 0) {
                    far_of[i] = (int32_t)far_node.size();
                    far_node.push_back(i);
                }
                list.push_back(far_of[i] << 1 | 1);
                cost.push_back((double)tr->np);
            } else if (nd.c0 < 0) {
                list.push_back(i << 1);
                cost.push_back(6.0 * (nd.e - nd.b));
            } else {
                stack.push_back(nd.c1);
                stack.push_back(nd.c0);
                continue;
            }
            total += cost.back();
        }
        list_ptr.push_back((int32_t)list.size());
        bcost[bt] = total;
        evals += 6.0 * (te - tb) * total;
    }
    // Pieces of about equal work over the whole mesh (a batch's list is cut
    // into a number of pieces proportional to its work; about 64 per SIMD in
    // all), dispatched heaviest first so that no long piece starts last: with
    // a fixed number of pieces per batch the uneven batches left most SIMDs
    // idle while a few long wavefronts finished.
    double sum = 0.0;
    for (double c : bcost) sum += c;
    const double target = std::max(sum / 65536.0, 1.0);
    std::vector<int> npc(tr->nbatch);
    tr->nsplit = 1;
    for (int bt = 0; bt < tr->nbatch; ++bt) {
        npc[bt] = std::max(1, std::min(kMaxPieces, (int)std::ceil(bcost[bt] / target)));
        tr->nsplit = std::max(tr->nsplit, npc[bt]);
    }
    const int S = tr->nsplit;
    std::vector<int32_t> piece_ptr(1, 0), entry;
    std::vector<double> pcost((size_t)tr->nbatch * S, 0.0);
    entry.reserve(list.size());
    for (int bt = 0; bt < tr->nbatch; ++bt) {
        double acc = 0.0;
        int k = list_ptr[bt];
        for (int p = 0; p < S; ++p) {
            const double stop = bcost[bt] * (p + 1) / npc[bt];
            const double before = acc;
            while (k < list_ptr[bt + 1] && (acc + 0.5 * cost[k] <= stop || p == npc[bt] - 1)) {
                entry.push_back(list[k]);
                acc += cost[k];
                ++k;
            }
            piece_ptr.push_back((int32_t)entry.size());
            pcost[(size_t)bt * S + p] = acc - before;
        }
    }
    std::vector<int32_t> order((size_t)tr->nbatch * S);
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return pcost[a] > pcost[b]; });
    tr->nfar = (int)far_node.size();
    tr->evals = evals;

    // interpolation boxes of every node: the vertex box, no dimension thinner
    // than 1e-3 of its widest (flat clusters)
    const size_t nn = nodes.size();
    std::vector<double> box(6 * nn, 0.0);
    for (size_t i = 0; i < nn; ++i) {
        const Node &nd = nodes[i];
        double hmax = 0.0;
        for (int c = 0; c < 3; ++c) hmax = std::max(hmax, 0.5 * (nd.hi[c] - nd.lo[c]));
        for (int c = 0; c < 3; ++c) {
            box[6 * i + c] = nd.centre(c);
            box[6 * i + 3 + c] = std::max(0.5 * (nd.hi[c] - nd.lo[c]), 1e-3 * hmax);
        }
    }
    // Upward pass: charges of every far cluster and of everything below it.
    // Leaves from their points; a parent from its two children's proxies
    // (k_tree_m2m): its tensor basis is a polynomial of the interpolation
    // degree in each variable, which the children's interpolation reproduces
    // exactly, so this equals the sum over the parent's points to rounding.
    std::vector<char> need(nn, 0);
    for (int32_t f : far_node) need[f] = 1;
    std::vector<int> depth(nn, 0);
    int maxdepth = 0;
    for (size_t i = 0; i < nn; ++i)   // parents come before their children
        if (nodes[i].c0 >= 0) {
            depth[nodes[i].c0] = depth[nodes[i].c1] = depth[i] + 1;
            maxdepth = std::max(maxdepth, depth[i] + 1);
            if (need[i]) need[nodes[i].c0] = need[nodes[i].c1] = 1;
        }
    std::vector<int32_t> slot(nn, -1);
    int nslot = 0;
    for (size_t i = 0; i < nn; ++i)
        if (need[i]) slot[i] = nslot++;
    std::vector<int32_t> item;   // leaves: slot, node, first, end triangle
    std::vector<std::vector<int32_t>> lev(maxdepth + 1);
    for (size_t i = 0; i < nn; ++i) {
        if (!need[i]) continue;
        const Node &nd = nodes[i];
        if (nd.c0 < 0) {
            item.insert(item.end(), {slot[i], (int32_t)i, nd.b, nd.e});
        } else {
            lev[depth[i]].insert(lev[depth[i]].end(), {slot[i], (int32_t)i, slot[nd.c0], nd.c0, slot[nd.c1], nd.c1});
        }
    }
    tr->nitem = (int)(item.size() / 4);
    std::vector<int32_t> m2m;   // deepest level first
    tr->level_ptr.assign(1, 0);
    for (int L = maxdepth; L >= 0; --L) {
        m2m.insert(m2m.end(), lev[L].begin(), lev[L].end());
        tr->level_ptr.push_back((int32_t)(m2m.size() / 6));
    }
    std::vector<int32_t> far_slot(tr->nfar);
    for (int f = 0; f < tr->nfar; ++f) far_slot[f] = slot[far_node[f]];
    std::vector<int32_t> range(2 * nodes.size());
    for (size_t i = 0; i < nodes.size(); ++i) {
        range[2 * i] = nodes[i].b;
        range[2 * i + 1] = nodes[i].e;
    }
    auto up = [&](const void *src, size_t bytes) {
        void *p = d.alloc(std::max<size_t>(bytes, 4));
        if (bytes) HIPCHECK(hipMemcpyAsync(p, src, bytes, hipMemcpyHostToDevice, d.stream));
        return p;
    };
    tr->node_range = (int32_t *)up(range.data(), sizeof(int32_t) * range.size());
    tr->box = (double *)up(box.data(), sizeof(double) * box.size());
    tr->far_node = (int32_t *)up(far_node.data(), sizeof(int32_t) * far_node.size());
    tr->far_slot = (int32_t *)up(far_slot.data(), sizeof(int32_t) * far_slot.size());
    tr->m2m = (int32_t *)up(m2m.data(), sizeof(int32_t) * m2m.size());
    tr->piece_ptr = (int32_t *)up(piece_ptr.data(), sizeof(int32_t) * piece_ptr.size());
    tr->order = (int32_t *)up(order.data(), sizeof(int32_t) * order.size());
    tr->entry = (int32_t *)up(entry.data(), sizeof(int32_t) * entry.size());
    const size_t rsz = d.prm.precision == PB_FP64 ? sizeof(double) : sizeof(float);
    tr->prox = d.alloc(rsz * kProxRec * (size_t)tr->np * std::max(tr->nfar, 1));
    tr->item = (int32_t *)up(item.data(), sizeof(int32_t) * item.size());
    tr->charges = (double *)d.alloc(sizeof(double) * 8 * (size_t)tr->np * std::max(nslot, 1));
    HIPCHECK(hipStreamSynchronize(d.stream));   // host vectors go out of scope
    return tr.release();
}

void tree_destroy(DevMesh &d)
{
    delete d.tree;   // device memory belongs to the handle's allocation list
    d.tree = nullptr;
}

// ------------------------------------------------------------ upward pass
// Leaves (k_tree_charges, one block per leaf): 64 source points at a time are
// staged in LDS; threads (point, dimension) form the 1-D barycentric basis
// values and derivatives at the Chebyshev nodes, then each thread accumulates
// the charges of its proxies.  Parents (k_tree_m2m, level by level from the
// deepest): their children's charges carried by the parent's basis evaluated
// at the children's proxies.  FP64 throughout.
constexpr int kUpPts = 64;

__device__ inline double cheb_node(int m, int deg) { return cos(kPi * m / deg); }

// 1-D barycentric Lagrange basis at the deg+1 Chebyshev nodes tn (weights wb)
// of normalised coordinate t: values L[m] and derivatives dL[m] (dL may be null)
__device__ inline void bary_basis(int deg, double t, const double *tn, const double *wb, double *L, double *dL)
{
    const int n1 = deg + 1;
    int hit = -1;
    for (int m = 0; m < n1; ++m)
        if (fabs(t - tn[m]) < 1e-13) hit = m;
    if (hit < 0) {
        double S = 0.0, S2 = 0.0;
        for (int m = 0; m < n1; ++m) {
            const double r = wb[m] / (t - tn[m]);
            S += r;
            S2 += r / (t - tn[m]);
        }
        for (int m = 0; m < n1; ++m) {
            const double v = wb[m] / (t - tn[m]) / S;
            L[m] = v;
            if (dL) dL[m] = v * (S2 / S - 1.0 / (t - tn[m]));
        }
    } else {
        // at a node: Kronecker values, the differentiation matrix row
        double diag = 0.0;
        for (int m = 0; m < n1; ++m) {
            L[m] = m == hit ? 1.0 : 0.0;
            if (dL && m != hit) {
                const double v = (wb[m] / wb[hit]) / (tn[hit] - tn[m]);
                dL[m] = v;
                diag -= v;
            }
        }
        if (dL) dL[hit] = diag;
    }
}

__global__ __launch_bounds__(256) void k_tree_charges(int deg, int np, const int32_t *__restrict__ item,
                                                      const double *__restrict__ box,
                                                      const double *__restrict__ stat,
                                                      const double *__restrict__ dyn, double *__restrict__ charges,
                                                      DevCtl ctl)
{
    __shared__ double tn[kTreeMaxDegree + 1], wb[kTreeMaxDegree + 1];
    __shared__ double pt[kUpPts][11];                            // t 3, b1, b2, w C 3, n 3
    __shared__ double la[kUpPts][3][kTreeMaxDegree + 1], lb[kUpPts][3][kTreeMaxDegree + 1];
    if (ctl_skip(ctl)) return;
    const int tid = threadIdx.x, n1 = deg + 1;
    const int32_t *it = item + 4 * (size_t)blockIdx.x;
    const int sl = it[0], b = it[2], e = it[3];
    const double *bx = box + 6 * (size_t)it[1];
    if (tid < n1) {
        tn[tid] = cheb_node(tid, deg);
        wb[tid] = ((tid & 1) ? -1.0 : 1.0) * ((tid == 0 || tid == deg) ? 0.5 : 1.0);
    }
    double acc[2][8];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[a][c] = 0.0;
    const int npts = 6 * (e - b);
    for (int base = 0; base < npts; base += kUpPts) {
        __syncthreads();   // previous chunk consumed (and tn, wb written)
        if (tid < kUpPts) {
            const int p = base + tid;
            if (p < npts) {
                const int s = b + p / 6, q = p % 6;
                const double *st = stat + (size_t)s * kStat;
                const double *sd = dyn + (size_t)s * kDyn;
                for (int c = 0; c < 3; ++c) pt[tid][c] = (st[3 * q + c] - bx[c]) / bx[3 + c];
                pt[tid][3] = sd[q];
                pt[tid][4] = sd[6 + q];
                for (int c = 0; c < 3; ++c) pt[tid][5 + c] = rule_w(q) * sd[12 + c];
                for (int c = 0; c < 3; ++c) pt[tid][8 + c] = st[18 + c];
            } else {
                for (int c = 0; c < 11; ++c) pt[tid][c] = 0.0;
                pt[tid][0] = pt[tid][1] = pt[tid][2] = 0.5;   // any point in the box; weights are zero
            }
        }
        __syncthreads();
        if (tid < 3 * kUpPts) {
            const int pp = tid / 3, dim = tid % 3;
            bary_basis(deg, pt[pp][dim], tn, wb, la[pp][dim], lb[pp][dim]);
        }
        __syncthreads();
        const int cnt = min(kUpPts, npts - base);
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int k = tid + 256 * a;
            if (k >= np) break;
            const int i = k / (n1 * n1), j = (k / n1) % n1, l = k % n1;
            for (int pp = 0; pp < cnt; ++pp) {
                const double Lx = la[pp][0][i], Ly = la[pp][1][j], Lz = la[pp][2][l];
                const double L = Lx * Ly * Lz;
                const double gx = lb[pp][0][i] * Ly * Lz / bx[3], gy = Lx * lb[pp][1][j] * Lz / bx[4],
                             gz = Lx * Ly * lb[pp][2][l] / bx[5];
                const double *P = pt[pp];
                acc[a][0] += P[3] * (P[8] * gx + P[9] * gy + P[10] * gz);
                acc[a][1] += P[4] * L;
                acc[a][2] += P[5] * L;
                acc[a][3] += P[6] * L;
                acc[a][4] += P[7] * L;
                acc[a][5] += P[3] * P[8] * L;
                acc[a][6] += P[3] * P[9] * L;
                acc[a][7] += P[3] * P[10] * L;
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int k = tid + 256 * a;
        if (k >= np) break;
        double *o = charges + ((size_t)sl * np + k) * 8;
        for (int c = 0; c < 8; ++c) o[c] = acc[a][c];
    }
}

// One block per parent of one level: q_P[k] = sum over both children c and
// their proxies k' of L^P_k(s^c_k') q_c[k'].  The parent's tensor basis at the
// child's tensor grid factorises, so the sum is applied one dimension at a
// time (z, then y, then x) through LDS: 3 (deg+1) instead of (deg+1)^3
// products per proxy and charge.
__global__ __launch_bounds__(256) void k_tree_m2m(int deg, int np, const int32_t *__restrict__ m2m,
                                                  const double *__restrict__ box, double *__restrict__ charges,
                                                  DevCtl ctl)
{
    constexpr int kMaxNp = (kTreeMaxDegree + 1) * (kTreeMaxDegree + 1) * (kTreeMaxDegree + 1);
    __shared__ double tn[kTreeMaxDegree + 1], wb[kTreeMaxDegree + 1];
    __shared__ double tab[2][3][kTreeMaxDegree + 1][kTreeMaxDegree + 1];   // [child][dim][child node][parent basis]
    __shared__ double buf[2][kMaxNp][8];
    if (ctl_skip(ctl)) return;
    const int tid = threadIdx.x, n1 = deg + 1, n2 = n1 * n1;
    const int32_t *en = m2m + 6 * (size_t)blockIdx.x;
    const int ps = en[0];
    const double *pb = box + 6 * (size_t)en[1];
    if (tid < n1) {
        tn[tid] = cheb_node(tid, deg);
        wb[tid] = ((tid & 1) ? -1.0 : 1.0) * ((tid == 0 || tid == deg) ? 0.5 : 1.0);
    }
    __syncthreads();
    if (tid < 2 * 3 * n1) {
        const int c = tid / (3 * n1), dim = (tid / n1) % 3, m = tid % n1;
        const double *cb = box + 6 * (size_t)en[3 + 2 * c];
        // the child's node m in dimension dim, in the parent's normalised coordinate
        const double t = (cb[dim] + cb[3 + dim] * tn[m] - pb[dim]) / pb[3 + dim];
        bary_basis(deg, t, tn, wb, tab[c][dim][m], nullptr);
    }
    double acc[2][8];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int v = 0; v < 8; ++v) acc[a][v] = 0.0;
    for (int c = 0; c < 2; ++c) {
        const double *cq = charges + (size_t)en[2 + 2 * c] * np * 8;
        __syncthreads();   // tables ready; the previous child's buffers consumed
        for (int e = tid; e < np * 8; e += blockDim.x) buf[0][e / 8][e % 8] = cq[e];
        __syncthreads();
        // z: buf1[i', j', l] = sum_l' T_z[l'][l] buf0[i', j', l']
        for (int k = tid; k < np; k += blockDim.x) {
            const int l = k % n1, base = k - l;
            double q[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int lc = 0; lc < n1; ++lc) {
                const double w = tab[c][2][lc][l];
#pragma unroll
                for (int v = 0; v < 8; ++v) q[v] += w * buf[0][base + lc][v];
            }
#pragma unroll
            for (int v = 0; v < 8; ++v) buf[1][k][v] = q[v];
        }
        __syncthreads();
        // y: buf0[i', j, l] = sum_j' T_y[j'][j] buf1[i', j', l]
        for (int k = tid; k < np; k += blockDim.x) {
            const int j = (k / n1) % n1, base = k - j * n1;
            double q[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int jc = 0; jc < n1; ++jc) {
                const double w = tab[c][1][jc][j];
#pragma unroll
                for (int v = 0; v < 8; ++v) q[v] += w * buf[1][base + jc * n1][v];
            }
#pragma unroll
            for (int v = 0; v < 8; ++v) buf[0][k][v] = q[v];
        }
        __syncthreads();
        // x: q_P[i, j, l] += sum_i' T_x[i'][i] buf0[i', j, l]
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int k = tid + 256 * a;
            if (k >= np) break;
            const int i = k / n2, base = k - i * n2;
            for (int ic = 0; ic < n1; ++ic) {
                const double w = tab[c][0][ic][i];
#pragma unroll
                for (int v = 0; v < 8; ++v) acc[a][v] += w * buf[0][base + ic * n2][v];
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int k = tid + 256 * a;
        if (k >= np) break;
        double *o = charges + ((size_t)ps * np + k) * 8;
#pragma unroll
        for (int v = 0; v < 8; ++v) o[v] = acc[a][v];
    }
}

// proxy records of far cluster f: positions and charges, in the evaluation precision
template <typename RP>
__global__ __launch_bounds__(256) void k_tree_proxies(int deg, int np, const int32_t *__restrict__ far_node,
                                                      const int32_t *__restrict__ far_slot,
                                                      const double *__restrict__ box,
                                                      const double *__restrict__ charges, RP *__restrict__ prox,
                                                      DevCtl ctl)
{
    if (ctl_skip(ctl)) return;
    const int f = blockIdx.x, n1 = deg + 1;
    const double *bx = box + 6 * (size_t)far_node[f];
    for (int k = threadIdx.x; k < np; k += blockDim.x) {
        const double *q = charges + ((size_t)far_slot[f] * np + k) * 8;
        const int i = k / (n1 * n1), j = (k / n1) % n1, l = k % n1;
        RP *o = prox + ((size_t)f * np + k) * kProxRec;
        o[0] = (RP)(bx[0] + bx[3] * cheb_node(i, deg));
        o[1] = (RP)(bx[1] + bx[4] * cheb_node(j, deg));
        o[2] = (RP)(bx[2] + bx[5] * cheb_node(l, deg));
        for (int c = 0; c < 8; ++c) o[3 + c] = (RP)q[c];
        o[11] = (RP)0;
    }
}

// ------------------------------------------------------------- evaluation
// One wavefront per (batch, piece), four per block: lanes own target triangles; list entries
// are wavefront-uniform, so proxy records and source triangles come through
// scalar loads.  Sums in R, as the direct kernel's chunks (a piece holds a
// few thousand sources at most); pieces are added in FP64 by k_far_finish.
// FP32: 5 wavefronts per SIMD (at most 96 VGPRs, no spills), which hides the
// per-source scalar loads of the direct sums; the Yukawa-only form (FORM 3)
// needs 97 VGPRs and runs 4.
template <typename R, int FORM>
__global__ __launch_bounds__(kTreeBlock) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? (FORM == 3 ? 4 : 5) : 1))) void k_tree_eval(int T, int nsplit, int nwork, int np, FarCoef<R> cf,
                                                          const int32_t *__restrict__ tri,
                                                          const R *__restrict__ stat, const R *__restrict__ dyn,
                                                          const int32_t *__restrict__ node_range,
                                                          const int32_t *__restrict__ piece_ptr,
                                                          const int32_t *__restrict__ order,
                                                          const int32_t *__restrict__ entry,
                                                          const R *__restrict__ prox, R *__restrict__ part,
                                                          DevCtl ctl)
{
    __shared__ R srec[kTreeBlock / kTreeBatch][kStage][42];
    __shared__ int4 sid[kTreeBlock / kTreeBatch][kStage];
    if (ctl_skip(ctl)) return;
    // four independent wavefronts per block, one (batch, piece) each
    // wavefront-uniform (readfirstlane), so the list walk stays on scalar loads
    const int wi = blockIdx.x * (kTreeBlock / kTreeBatch) +
                   __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kTreeBatch));
    if (wi >= nwork) return;
    const int item = order[wi];
    const int bt = item / nsplit, piece = item % nsplit;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kTreeBatch)), lane = threadIdx.x % kTreeBatch;
    const int t = bt * kTreeBatch + (int)(threadIdx.x % kTreeBatch);
    const int tc = t < T ? t : T - 1;   // lanes past the end compute, never store
    const R *ts = stat + (size_t)tc * kStat;
    R tx[6], ty[6], tz[6];
#pragma unroll
    for (int p = 0; p < 6; ++p) { tx[p] = ts[3 * p]; ty[p] = ts[3 * p + 1]; tz[p] = ts[3 * p + 2]; }
    const R ntx = ts[18], nty = ts[19], ntz = ts[20];
    const R ot = ts[21];   // plane offset x . n_t, the same for the six points
    const int v0 = tri[3 * tc], v1 = tri[3 * tc + 1], v2 = tri[3 * tc + 2];
    R a1[6], a2[6], W0 = 0, W1 = 0, W2 = 0;
#pragma unroll
    for (int p = 0; p < 6; ++p) { a1[p] = 0; a2[p] = 0; }
    for (int en = piece_ptr[item]; en < piece_ptr[item + 1]; ++en) {
        const int code = entry[en];
        if (code & 1) {
            const R *P = prox + (size_t)(code >> 1) * np * kProxRec;
            for (int k = 0; k < np; ++k) {
                const R *cur = P + (size_t)k * kProxRec;
                const R sx = cur[0], sy = cur[1], sz = cur[2];
                const R qK = cur[3], qV = cur[4];
                // per proxy: row 1 = ri (cKL qK + cVL qV) + e ri (cKY qK + cVY qV); row 2 =
                // (d.n_t) qV (cTL R3 + cTY E) + ntqN e ri with R3 = r^-3, E = e (R3 +
                // kappa r^-2) and d.n_t = ot - z.n_t the same for the six target points;
                // the curl part's G sums (GL, GY) take their coefficients once
                R ntqN = 0, AL = 0, AY = 0, CL = 0, CY = 0, GL = 0, GY = 0;
                if (FORM == 0) {
                    AL = cf.kL * qK + cf.vL * qV;
                    AY = cf.kY * qK + cf.vY * qV;
                } else {
                    ntqN = cf.cDY * cf.k2 * (ntx * cur[8] + nty * cur[9] + ntz * cur[10]);
                    const R dq = (ot - (sx * ntx + sy * nty + sz * ntz)) * qV;
                    AL = cf.cKL * qK + cf.cVL * qV;
                    AY = cf.cKY * qK + cf.cVY * qV;
                    CL = cf.cTL * dq;
                    CY = cf.cTY * dq;
                }
#pragma unroll
                for (int p = 0; p < 6; ++p) {
                    const R dx = tx[p] - sx, dy = ty[p] - sy, dz = tz[p] - sz;
                    const R r2 = dx * dx + dy * dy + dz * dz;
                    const R ri = rsqrt_r(r2);
                    const R r = r2 * ri;
                    const R e = expneg(cf.kexp, r);
                    const R gy = e * ri;
                    if (FORM == 0) {
                        a1[p] += ri * AL;
                        a2[p] += gy * AY;
                    } else {
                        const R ri2 = ri * ri, R3 = ri2 * ri;
                        const R E = e * fma(cf.kappa, ri2, R3);
                        if (FORM == 3) {
                            a1[p] = fma(gy, AY, a1[p]);
                            a2[p] = fma(CY, E, fma(ntqN, gy, a2[p]));
                        } else {
                            a1[p] = fma(ri, AL, fma(gy, AY, a1[p]));
                            a2[p] = fma(CL, R3, fma(CY, E, fma(ntqN, gy, a2[p])));
                            GL = fma(R(rule_w(p)), ri, GL);
                        }
                        GY = fma(R(rule_w(p)), gy, GY);
                    }
                }
                if (FORM >= 1) {
                    const R gw = FORM == 3 ? cf.cDY * GY : cf.cDL * GL + cf.cDY * GY;
                    W0 += gw * cur[5];
                    W1 += gw * cur[6];
                    W2 += gw * cur[7];
                }
            }
        } else {
            const int nd = code >> 1;
            const int sb = node_range[2 * nd], se = node_range[2 * nd + 1];
            // kStage source records at a time staged in the wavefront's own LDS
            // slice (one lane per source, all loads in flight together), then read
            // back as broadcasts: the leaves differ from wavefront to wavefront,
            // so a scalar-load walk would wait on every source
            for (int s0 = sb; s0 < se; s0 += kStage) {
                const int ns = min(kStage, se - s0);
                __builtin_amdgcn_wave_barrier();   // the previous records are consumed
                if (lane < ns) {
                    const R *st = stat + (size_t)(s0 + lane) * kStat, *sd = dyn + (size_t)(s0 + lane) * kDyn;
#pragma unroll
                    for (int c = 0; c < 27; ++c) srec[wv][lane][c] = st[c];
#pragma unroll
                    for (int c = 0; c < 15; ++c) srec[wv][lane][27 + c] = sd[c];
                    sid[wv][lane] = make_int4(tri[3 * (s0 + lane)], tri[3 * (s0 + lane) + 1], tri[3 * (s0 + lane) + 2], 0);
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                for (int k = 0; k < ns; ++k) {
                    const int4 j = sid[wv][k];
                    const bool adj = (j.x == v0) | (j.x == v1) | (j.x == v2) | (j.y == v0) | (j.y == v1) |
                                     (j.y == v2) | (j.z == v0) | (j.z == v1) | (j.z == v2);
                    if (adj) continue;
                    far_source<R, FORM>(cf, srec[wv][k], srec[wv][k] + 27, tx, ty, tz, ot, ntx, nty, ntz, a1, a2, W0,
                                        W1, W2);
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
        }
    }
    if (t >= T) return;
    R *o = part + ((size_t)piece * T + t) * 16;
#pragma unroll
    for (int p = 0; p < 6; ++p) { o[p] = a1[p]; o[6 + p] = a2[p]; }
    o[12] = W0; o[13] = W1; o[14] = W2; o[15] = 0;
}

template <typename R>
static void tree_launch(DevMesh &d, const R *stat, const R *dyn)
{
    Tree &tr = *d.tree;
    if (tr.nfar > 0) {
        hipLaunchKernelGGL(k_tree_charges, dim3(tr.nitem), dim3(256), 0, d.stream, tr.degree, tr.np, tr.item, tr.box,
                           d.stat64, d.dyn64, tr.charges, d.ctl);
        for (size_t L = 0; L + 1 < tr.level_ptr.size(); ++L) {
            const int n = tr.level_ptr[L + 1] - tr.level_ptr[L];
            if (n > 0)
                hipLaunchKernelGGL(k_tree_m2m, dim3(n), dim3(256), 0, d.stream, tr.degree, tr.np,
                                   tr.m2m + 6 * (size_t)tr.level_ptr[L], tr.box, tr.charges, d.ctl);
        }
        hipLaunchKernelGGL(k_tree_proxies<R>, dim3(tr.nfar), dim3(256), 0, d.stream, tr.degree, tr.np, tr.far_node,
                           tr.far_slot, tr.box, tr.charges, (R *)tr.prox, d.ctl);
    }
    FarCoef<R> cf;
    const int form = far_coef(d, cf);
    const int nwork = tr.nbatch * tr.nsplit, per = kTreeBlock / kTreeBatch;
    const dim3 grid((nwork + per - 1) / per), block(kTreeBlock);
#define TREE_EVAL(F)                                                                                              \
    hipLaunchKernelGGL((k_tree_eval<R, F>), grid, block, 0, d.stream, d.hm.T, tr.nsplit, nwork, tr.np, cf, d.tri, \
                       stat, dyn, tr.node_range, tr.piece_ptr, tr.order, tr.entry, (const R *)tr.prox, (R *)d.part, \
                       d.ctl)
    if (form == 0) TREE_EVAL(0);
    else if (form == 1) TREE_EVAL(1);
    else TREE_EVAL(3);
#undef TREE_EVAL
    HIPCHECK(hipGetLastError());
}

void launch_tree_far(DevMesh &d, bool fp32)
{
    Profiler &pf = d.prof;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (pf.on(0)) {
        HIPCHECK(hipEventCreate(&e0));
        HIPCHECK(hipEventCreate(&e1));
        HIPCHECK(hipEventRecord(e0, d.stream));
    }
    if (fp32) tree_launch<float>(d, d.stat32, d.dyn32);
    else tree_launch<double>(d, d.stat64, d.dyn64);
    if (pf.on(0)) {
        HIPCHECK(hipEventRecord(e1, d.stream));
        pf.record(0, e0, e1, d.tree->evals);   // point-pair and point-proxy kernel evaluations
    }
}

}  // namespace pbm
