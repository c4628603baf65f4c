"""Pins of the oracle's singular quadrature and of its sampled-row checker.

The Sauter-Schwab blocks are compared entry by entry with the Laplace single-
and double-layer integrals of flat triangles computed another way: closed-form
inner potentials (Wilton et al. 1984, Graglia 1993, van Oosterom-Strackee
1983) and a tanh-sinh outer rule (tests/flat_triangle.py), which shares no
map, ordering or rule with the oracle.  A wrong region map, Jacobian, local
vertex arrangement or scatter of the arranged block back to the stored
vertices either stops the convergence in the Gauss order or leaves an O(1e-2)
error (both checked on planted mistakes while writing these tests).

The checker used by the full-size GPU parity tests (``oracle.system_rows``,
``oracle.calderon_rows``, and through them the column mode of
``orc_operator_rows``) is pinned against the dense matrices it samples.
"""
import numpy as np
import pytest

import inputs
import oracle
from flat_triangle import laplace_blocks


class _Mesh:
    def __init__(self, xyz, tri):
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32)
        self.n_vertices = len(self.xyz)
        self.n_triangles = len(self.tri)


@pytest.fixture(scope="module")
def skew_pairs():
    """Skewed, non-coplanar pairs of a coarse star surface: one coincident,
    edge and vertex pair in each order (test/trial)."""
    m, _ = inputs.star_surface(7, 2, 3.0)
    tri = m.tri
    pairs = [(0, 0, 3), (9, 9, 3)]
    for a, b in ((0, None), (None, 7)):
        found = set()
        for s in range(len(tri)):
            t_, s_ = (a, s) if a is not None else (s, b)
            k = len(set(tri[t_]) & set(tri[s_]))
            if k in (1, 2) and k not in found:
                pairs.append((t_, s_, k))
                found.add(k)
    return m, pairs


# Gauss order 4 error bounds per case (the rule's own convergence, about three
# times the errors observed for these pairs) and the order-10 bound
ORDER4 = {3: 6e-5, 2: 6e-5, 1: 2e-5}


def test_singular_blocks_match_closed_form(skew_pairs):
    """Every entry of V_L and K_L converges exponentially in the Gauss order to
    the independently computed integral."""
    m, pairs = skew_pairs
    assert sorted({k for _, _, k in pairs}) == [1, 2, 3]
    for t, s, k in pairs:
        Vr, Kr = laplace_blocks(m.xyz[m.tri[t]], m.xyz[m.tri[s]], step=1.0 / 32)
        scale = np.abs(Vr).max()
        errs = []
        for n in (3, 4, 6, 8, 10):
            V, K, ns = oracle.pair_block(m, t, s, 0.0, n)
            assert ns == k
            errs.append((np.abs(V - Vr).max() / scale, np.abs(K - Kr).max() / scale))
        ev = [e[0] for e in errs]
        ek = [e[1] for e in errs]
        assert ev[1] < ORDER4[k] and ek[1] < ORDER4[k], (t, s, k, errs)
        assert ev[-1] < 5e-11 and ek[-1] < 1e-10, (t, s, k, errs)
        assert ev[0] > ev[1] > ev[2] > ev[3], (t, s, k, errs)
        if k < 3:   # K_L of a flat coincident pair is zero on both sides
            assert ek[0] > ek[1] > ek[2] > ek[3], (t, s, k, errs)
        else:
            assert ek[-1] < 1e-13


def test_skinny_high_valence_pairs_converge():
    """Valence-80 apexes: triangles of aspect ratio about 25 sharing the apex,
    a spoke edge (coplanar neighbours) or a ring edge (sharp fold).  The rule
    converges more slowly on such pairs, but to the independently computed
    integral."""
    m = inputs.bipyramid(80)
    cases = {(0, 0): 3, (0, 2): 2, (0, 1): 2, (0, 10): 1, (0, 3): 1, (1, 3): 2}
    for (t, s), k in cases.items():
        Vr, Kr = laplace_blocks(m.xyz[m.tri[t]], m.xyz[m.tri[s]], step=1.0 / 32)
        scale = np.abs(Vr).max()
        errs = []
        for n in (4, 8, 12):
            V, K, ns = oracle.pair_block(m, t, s, 0.0, n)
            assert ns == k
            errs.append(max(np.abs(V - Vr).max(), np.abs(K - Kr).max()) / scale)
        assert errs[0] > errs[1] > errs[2] or errs[0] < 1e-13, ((t, s), errs)
        assert errs[2] < 1e-3, ((t, s), errs)
        assert errs[0] < 0.6, ((t, s), errs)


def test_blocks_invariant_under_relabelling():
    """Renumbering the vertices and rotating each triangle's stored vertex
    list (orientation kept) changes no block of a pair sharing an edge or a
    vertex beyond rounding: the local arrangement depends only on which
    vertices are shared and on the triangles' orientation.  Identical
    triangles keep their stored order, so a rotation moves their quadrature
    points; the 6-region rule is nearly symmetric and stays within 1e-8."""
    m, _ = inputs.star_surface(7, 2, 3.0)
    rng = np.random.default_rng(3)
    perm = rng.permutation(m.n_vertices)          # old id -> new id
    rot = rng.integers(0, 3, m.n_triangles)
    xyz2 = np.zeros_like(m.xyz)
    xyz2[perm] = m.xyz
    m2 = _Mesh(xyz2, [np.roll(perm[tr], -r) for tr, r in zip(m.tri, rot)])
    worst = {1: 0.0, 2: 0.0, 3: 0.0}
    for t in range(0, m.n_triangles, 3):
        for s in range(m.n_triangles):
            k = len(set(m.tri[t]) & set(m.tri[s]))
            if k == 0:
                continue
            for kap in (0.0, 0.125):
                V, K, _ = oracle.pair_block(m, t, s, kap, 4)
                V2, K2, _ = oracle.pair_block(m2, t, s, kap, 4)
                it = [(a + rot[t]) % 3 for a in range(3)]   # new slot a = old slot a + rot
                js = [(b + rot[s]) % 3 for b in range(3)]
                e = max(np.abs(V2 - V[np.ix_(it, js)]).max(), np.abs(K2 - K[np.ix_(it, js)]).max())
                worst[k] = max(worst[k], e / np.abs(V).max())
    assert worst[1] < 1e-14 and worst[2] < 1e-14, worst
    assert worst[3] < 1e-8, worst


# --------------------------------------------------------- sampled-row checker
@pytest.fixture(scope="module")
def checker_meshes():
    star, _ = inputs.star_surface(11, 3, 4.0)
    return {"sphere": inputs.icosphere(3, 1.5), "star": star}


@pytest.mark.parametrize("name", ["sphere", "star"])
def test_system_rows_equal_dense_rows(checker_meshes, name):
    """oracle.system_rows (operator rows, and columns of K for T = K^T) gives
    the sampled entries of A x for every formulation, to rounding."""
    m = checker_meshes[name]
    nv = m.n_vertices
    rng = np.random.default_rng(5)
    x = rng.standard_normal(2 * nv)
    rows = np.sort(rng.choice(nv, 9, replace=False))
    for form in oracle.FORMULATIONS:
        A = oracle.system_matrix(m, 4.0, 80.0, 0.125, form)
        y = A @ x
        y1, y2 = oracle.system_rows(m, 4.0, 80.0, 0.125, form, rows, x)
        got = np.concatenate([y1, y2])
        ref = np.concatenate([y[rows], y[nv + rows]])
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(y).max(), form


def test_operator_columns_are_transposed_rows(checker_meshes):
    """Column mode of the operator routine: column i of V, K, D equals row i
    of their transposes from the dense assembly, for both kernels."""
    m = checker_meshes["star"]
    cols = np.array([0, 5, m.n_vertices - 1], dtype=np.int32)
    for kap in (0.0, 0.125):
        dense = oracle.assemble(m, kap)
        got = oracle.operator_rows(m, kap, cols, 1)
        for op in ("V", "K", "D"):
            ref = dense[op][:, cols].T
            assert np.abs(got[op] - ref).max() <= 1e-15 * np.abs(dense[op]).max(), (kap, op)


@pytest.mark.parametrize("fast", [False, True])
def test_calderon_rows_equal_dense_rows(checker_meshes, fast):
    """oracle.calderon_rows samples P x for both PMCHWT systems and every part
    of the Calderon operator, with the accurate or the relaxed quadrature."""
    m = checker_meshes["star"]
    nv = m.n_vertices
    rng = np.random.default_rng(6)
    x = rng.standard_normal(2 * nv)
    rows = np.sort(rng.choice(nv, 7, replace=False))
    for form in (oracle.PMCHWT_INT, oracle.PMCHWT_EXT):
        for part in ("full", "int", "ext"):
            P = oracle.calderon_matrix(m, 4.0, 80.0, 0.125, form, part, fast=fast)
            y = P @ x
            y1, y2 = oracle.calderon_rows(m, 4.0, 80.0, 0.125, form, part, rows, x, fast=fast)
            got = np.concatenate([y1, y2])
            ref = np.concatenate([y[rows], y[nv + rows]])
            assert np.abs(got - ref).max() <= 1e-13 * np.abs(y).max(), (form, part)
