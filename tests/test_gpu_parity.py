"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances (from the arithmetic); every vector comparison (_rel) checks the
relative 2-norm error and, per block row, the largest entry error against ten
times the bound:
  * FP64 operator products, source projections, reaction potentials,
    preconditioner blocks: 1e-12 relative (2-norm).  Both sides evaluate the
    same quadrature sums in FP64; only the summation order differs.
  * Near-field Sauter-Schwab blocks: 1e-13 relative to the block's largest entry.
  * FP32 far-field evaluation: 1e-5 relative on the operator product.
  * Delta G: 1e-6 relative in FP64 at the solver tolerance 1e-5 (the GPU and
    the oracle run the same Krylov iteration; rounding differences stay far
    below the stopping tolerance), 1e-4 in reduced precision.
Sizes: small meshes span several 256-triangle tiles with a ragged tail
(T = 720, 980, 1280); the full-size sphere (20480 triangles) is checked on
sampled rows the oracle computes one by one.
"""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

pbm = pytest.importorskip("paper_2108_10481_amd")


def _opts(form=0, precision=0, **kw):
    return pbm.pb_default_options(formulation=form, precision=precision, **kw)


def _rel(a, b):
    """Relative error in the 2-norm, combined with an entrywise check: each
    half of the vector (the two block rows of a [trace_D; trace_N] vector)
    must also have its largest entry error within ten times the same bound
    relative to its own largest entry, so a single wrong entry cannot hide in
    the norm of a long vector.  Returns the larger of the 2-norm error and a
    tenth of the entrywise one."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    norm = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    entry = 0.0
    for x, y in zip(np.array_split(a, 2), np.array_split(b, 2)):
        scale = np.abs(y).max() if y.size else 0.0
        if scale > 0:
            entry = max(entry, float(np.abs(x - y).max() / scale))
    return max(norm, 0.1 * entry)


@pytest.fixture(scope="module")
def meshes():
    m1 = inputs.icosphere(6, 2.0)                 # T = 720
    m2, _ = inputs.star_surface(5, 7, 6.0)        # T = 980
    return {"sphere6": m1, "star7": m2}


@pytest.fixture(scope="module")
def dense_systems(meshes):
    out = {}
    for name, m in meshes.items():
        for form in (0, 1):
            out[(name, form)] = oracle.system_matrix(m, 4.0, 80.0, 0.125, form)
    return out


def test_library_sees_gpu():
    assert pbm.pb_device_count() >= 1


@pytest.mark.parametrize("name", ["sphere6", "star7"])
def test_near_field_blocks(meshes, name):
    """Sauter-Schwab local blocks of coincident, edge and vertex pairs."""
    m = meshes[name]
    tri = m.tri
    ts, ss = [], []
    for t in (0, 17, 311, m.n_triangles - 1):
        for s in range(m.n_triangles):
            if len(set(tri[t]) & set(tri[s])) > 0:
                ts.append(t)
                ss.append(s)
    with pbm.MeshHandle(m.xyz, m.tri, _opts()) as h:
        got = pbm.pb_mesh_near_blocks(h, ts, ss)
    for k, (t, s) in enumerate(zip(ts, ss)):
        VL, KL, _ = oracle.pair_block(m, t, s, 0.0, 4)
        VY, KY, _ = oracle.pair_block(m, t, s, 0.125, 4)
        ref = np.stack([VL, KL, VY, KY])
        scale = np.abs(ref[0]).max()
        assert np.abs(got[k] - ref).max() < 1e-13 * scale, (t, s)


@pytest.mark.parametrize("name", ["sphere6", "star7"])
@pytest.mark.parametrize("form", [0, 1])
def test_operator_fp64(meshes, dense_systems, name, form):
    m = meshes[name]
    A = dense_systems[(name, form)]
    rng = np.random.default_rng(11)
    x = rng.standard_normal(2 * m.n_vertices)
    with pbm.MeshHandle(m.xyz, m.tri, _opts(form)) as h:
        y = pbm.pb_mesh_apply(h, x)
        y2 = pbm.pb_mesh_apply(h, x)
        yf = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_FAR_ONLY)
        yn = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_NEAR_ONLY)
        yp = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_PRECOND)
        pinv = pbm.pb_mesh_preconditioner(h)
    ref = A @ x
    assert _rel(y, ref) < 1e-12
    assert np.array_equal(y, y2), "operator product must be deterministic"
    assert _rel(yf + yn, ref) < 1e-12
    inv = oracle.block_diagonal_inverse(A, m.n_vertices)
    assert np.abs(pinv - inv).max() < 1e-12 * np.abs(inv).max()
    assert _rel(yp, oracle.apply_block_diag(inv, ref)) < 1e-12


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("sym", [0, 1])
def test_operator_fp32(meshes, dense_systems, form, sym):
    """FP32 matrix-free products of a 980-triangle mesh against the oracle's
    dense system: each ordered triangle pair evaluated (far_symmetric 0, the
    automatic choice at this size) or each unordered pair once for both
    directions (far_symmetric 1); the two agree to FP32 rounding."""
    m = meshes["star7"]
    A = dense_systems[("star7", form)]
    x = np.random.default_rng(5).standard_normal(2 * m.n_vertices)
    with pbm.MeshHandle(m.xyz, m.tri, _opts(form, pbm.PB_FP32, far_symmetric=sym)) as h:
        y = pbm.pb_mesh_apply(h, x)
        y2 = pbm.pb_mesh_apply(h, x)
    assert _rel(y, A @ x) < 1e-5
    assert np.array_equal(y, y2), "FP32 products must be deterministic"


def test_far_symmetric_option():
    """far_symmetric -1 on a mesh the automatic choice splits symmetrically
    (5120 triangles) gives the per-ordered-pair product to FP32 rounding of
    the symmetric one and of FP64; the mesh info reports the choice (also for
    kappa = 0, never for FP64 or the assembled field); values outside
    {-1, 0, 1} are refused."""
    m, _ = inputs.star_surface(9, 16, 9.0)                     # T = 5120
    x = np.random.default_rng(17).standard_normal(2 * m.n_vertices)
    ys = {}
    for sym in (0, 1, -1):
        with pbm.MeshHandle(m.xyz, m.tri, _opts(1, pbm.PB_FP32, far_symmetric=sym)) as h:
            ys[sym] = pbm.pb_mesh_apply(h, x)
            assert h.info()["far_symmetric"] == (0 if sym < 0 else 1), sym
    with pbm.MeshHandle(m.xyz, m.tri, _opts(1)) as h:
        y64 = pbm.pb_mesh_apply(h, x)
        assert h.info()["far_symmetric"] == 0
    for extra, want in ((dict(kappa=0.0), 1), (dict(operator_mode=pbm.PB_ASSEMBLED), 0)):
        with pbm.MeshHandle(m.xyz, m.tri, _opts(1, pbm.PB_FP32, far_symmetric=1, **extra)) as h:
            assert h.info()["far_symmetric"] == want, extra
    assert np.array_equal(ys[0], ys[1]), "5120 triangles take the symmetric split automatically"
    for sym in (0, -1):
        assert _rel(ys[sym], y64) < 2e-6, (sym, _rel(ys[sym], y64))
    with pytest.raises(pbm.PbError) as e:
        pbm.MeshHandle(m.xyz, m.tri, _opts(1, pbm.PB_FP32, far_symmetric=2))
    assert e.value.code == pbm.PB_E_INVALID_ARG


@pytest.mark.parametrize("name", ["sphere6", "star7"])
def test_rhs_and_reaction_potential(meshes, name):
    m = meshes[name]
    ch = inputs.charges_ball(3, 13, 1.0)
    bD, bN = oracle.rhs(m, ch, 4.0)
    rng = np.random.default_rng(2)
    phi, dphi = rng.standard_normal(m.n_vertices), rng.standard_normal(m.n_vertices)
    ref_pr = oracle.reaction_potential(m, phi, dphi, ch.xyz)
    with pbm.MeshHandle(m.xyz, m.tri, _opts()) as h:
        b = pbm.pb_mesh_rhs(h, ch.xyz, ch.q)
        pr = pbm.pb_mesh_reaction_potential(h, phi, dphi, ch.xyz)
    assert _rel(b[:m.n_vertices], bD) < 1e-12
    assert _rel(b[m.n_vertices:], bN) < 1e-12
    assert _rel(pr, ref_pr) < 1e-12


@pytest.mark.parametrize("form", [0, 1])
def test_kirkwood_solve_parity(form):
    """Sphere of radius 2 A, 320 triangles, central +1 e: GPU Delta G equals the
    oracle's within 1e-6 (FP64) and 1e-4 (FP32), same iteration count."""
    m, ch = inputs.config_kirkwood(4, 2.0)
    ref = oracle.solve(m, ch, formulation=form)
    got = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form))
    assert got["status"] == pbm.PB_OK
    assert abs(got["dG"] - ref["dG"]) < 1e-6 * abs(ref["dG"])
    assert got["iterations"] == ref["iterations"]
    assert _rel(np.concatenate([got["phi"], got["dphi"]]), np.concatenate([ref["phi"], ref["dphi"]])) < 1e-6
    tight = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, tol=1e-11))
    reft = oracle.solve(m, ch, formulation=form, tol=1e-11, A=ref["A"])
    assert abs(tight["dG"] - reft["dG"]) < 1e-10 * abs(reft["dG"])
    g32 = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, pbm.PB_FP32))
    assert abs(g32["dG"] - ref["dG"]) < 1e-4 * abs(ref["dG"])


@pytest.mark.parametrize("form", [0, 1])
def test_small_solve_parity_multi_charge(meshes, dense_systems, form):
    m = meshes["star7"]
    ch = inputs.charges_ball(9, 20, 2.5)
    ref = oracle.solve(m, ch, formulation=form, A=dense_systems[("star7", form)])
    got = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form))
    assert abs(got["dG"] - ref["dG"]) < 1e-6 * abs(ref["dG"])
    assert abs(got["iterations"] - ref["iterations"]) <= 1


@pytest.fixture(scope="module")
def sphere32():
    return inputs.config_sphere()   # 20480 triangles, 10242 vertices, 50 charges


@pytest.mark.parametrize("form", [0, 1])
def test_full_size_sampled_rows(sphere32, form):
    """Radius-10 sphere, 20480 triangles: sampled rows of A x, in the launch
    configuration the benchmark uses, against rows the oracle computes."""
    m, _ = sphere32
    rng = np.random.default_rng(21)
    x = rng.standard_normal(2 * m.n_vertices)
    rows = np.sort(rng.choice(m.n_vertices, 12, replace=False))
    r1, r2 = oracle.system_rows(m, 4.0, 80.0, 0.125, form, rows, x)
    for prec, tol in ((pbm.PB_FP64, 1e-12), (pbm.PB_FP32, 2e-5)):
        with pbm.MeshHandle(m.xyz, m.tri, _opts(form, prec)) as h:
            y = pbm.pb_mesh_apply(h, x)
        nv = m.n_vertices
        got = np.concatenate([y[rows], y[nv + rows]])
        ref = np.concatenate([r1, r2])
        assert _rel(got, ref) < tol, (prec, _rel(got, ref))


@pytest.mark.parametrize("form,a,b,kappa", [(pbm.PB_DIRECT_INT, 1.0, 1.0, 0.125), (pbm.PB_JUFFER, 1.0, 1.0, 0.125),
                                             (pbm.PB_DIRECT_EXT, 1.0, 1.0, 0.125),
                                             (pbm.PB_MULLER_INT, 1.0, 1.0, 0.125),
                                             (pbm.PB_CFIE_EXT, 0.0, 1.0, 0.125), (pbm.PB_CFIE_EXT, 0.0, 0.0, 0.125),
                                             (pbm.PB_DIRECT_INT, 1.0, 1.0, 0.0), (pbm.PB_JUFFER, 1.0, 1.0, 0.0)])
def test_symmetric_far_field_full_size(sphere32, form, a, b, kappa):
    """20480-triangle sphere: the FP32 matrix-free far field, which evaluates
    every unordered pair once for both directions on coordinates scaled by
    kappa log2(e), against the FP64 one, which evaluates every ordered pair
    (the direct, second-kind and Yukawa-only kernel forms; a zero
    combined-field constant leaves a row without Laplace terms, both zero no
    Laplace term at all), within FP32 rounding; and its sampled rows against
    the oracle's.  kappa = 0 (no screening) takes the kernel's unscreened
    variant (coordinates as they are, no exponential) and is held to the same
    bounds."""
    m, _ = sphere32
    nv = m.n_vertices
    rng = np.random.default_rng(83)
    x = rng.standard_normal(2 * nv)
    with pbm.MeshHandle(m.xyz, m.tri, _opts(form, pbm.PB_FP32, cfie_alpha=a, cfie_beta=b, kappa=kappa)) as h:
        y32 = pbm.pb_mesh_apply(h, x)
        y32b = pbm.pb_mesh_apply(h, x)
        yf = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_FAR_ONLY)
    with pbm.MeshHandle(m.xyz, m.tri, _opts(form, cfie_alpha=a, cfie_beta=b, kappa=kappa)) as h:
        y64 = pbm.pb_mesh_apply(h, x)
        yf64 = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_FAR_ONLY)
    assert np.array_equal(y32, y32b), "the symmetric product must be deterministic"
    assert _rel(y32, y64) < 2e-6, (form, a, b, _rel(y32, y64))
    # the far part alone: second-kind rows combine -V_L + V_Y, which cancel to
    # (1 - exp(-kappa r))/r, about a tenth of either term at the pairs' distances,
    # so FP32 rounding weighs up to ten times more: the FP32 far-field bound
    assert _rel(yf, yf64) < 2e-5, (form, a, b, _rel(yf, yf64))
    rows = np.sort(rng.choice(nv, 4, replace=False))
    oform = {pbm.PB_DIRECT_INT: oracle.DIRECT, pbm.PB_JUFFER: oracle.JUFFER, pbm.PB_DIRECT_EXT: oracle.DIRECT_EXT,
             pbm.PB_MULLER_INT: oracle.MULLER_INT, pbm.PB_CFIE_EXT: oracle.CFIE_EXT}[form]
    r1, r2 = oracle.system_rows(m, 4.0, 80.0, kappa, oform, rows, x, alpha=a, beta=b)
    assert _rel(np.concatenate([y32[rows], y32[nv + rows]]), np.concatenate([r1, r2])) < 2e-5


def test_full_size_solve_kirkwood(sphere32):
    """Full-size sphere: FP64 and FP32 GPU solves agree to 1e-4 on Delta G and
    both sit within the discretisation error of the Kirkwood series."""
    from kirkwood import kirkwood_energy
    m, ch = sphere32
    ref = kirkwood_energy(10.0, ch.xyz, ch.q)
    for form in (0, 1):
        g64 = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form))
        g32 = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, pbm.PB_FP32))
        assert g64["status"] == pbm.PB_OK
        assert abs(g64["dG"] - ref) < 5e-3 * abs(ref), (g64["dG"], ref)
        assert abs(g32["dG"] - g64["dG"]) < 1e-4 * abs(g64["dG"])


def _golden_sphere20480():
    """Oracle Delta G on the 20480-triangle sphere workload, per (formulation,
    GMRES tolerance): (dG, iterations), from tests/golden/sphere20480_dG.txt."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sphere20480_dG.txt")
    out = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        name, tol, dG, its, _ = line.split()
        out[({"direct": 0, "juffer": 1}[name], float(tol))] = (float(dG), int(its))
    return out


def test_full_size_dG_against_oracle(sphere32):
    """20480-triangle sphere, 50 charges: Delta G against the FP64 oracle's
    (tests/golden, written by a script that calls only the oracle) -- FP64
    matrix-free and assembled within 1e-6 at the paper's tolerance and 1e-8 at
    tolerance 1e-10, FP32 and the mixed 16-bit modes within 1e-4."""
    m, ch = sphere32
    gold = _golden_sphere20480()
    for form in (0, 1):
        ref, its = gold[(form, 1e-5)]
        for mode in (pbm.PB_MATRIX_FREE, pbm.PB_ASSEMBLED):
            g = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, operator_mode=mode))
            assert g["status"] == pbm.PB_OK and abs(g["iterations"] - its) <= 1, (form, mode, g["iterations"], its)
            assert abs(g["dG"] - ref) < 1e-6 * abs(ref), (form, mode, g["dG"], ref)
        reft, _ = gold[(form, 1e-10)]
        g = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, tol=1e-10))
        assert abs(g["dG"] - reft) < 1e-8 * abs(reft), (form, g["dG"], reft)
        for prec, mode in ((pbm.PB_FP32, pbm.PB_MATRIX_FREE), (pbm.PB_FP32, pbm.PB_ASSEMBLED),
                           (pbm.PB_MIXED_BF16, pbm.PB_ASSEMBLED), (pbm.PB_MIXED_FP16, pbm.PB_ASSEMBLED)):
            g = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, prec, operator_mode=mode))
            assert g["status"] == pbm.PB_OK
            assert abs(g["dG"] - ref) < 1e-4 * abs(ref), (form, prec, mode, g["dG"], ref)


def test_tetrahedron_all_near():
    """Every pair of a tetrahedron shares a vertex: the far field is empty."""
    xyz = np.array([[1, 1, 1], [-1, -1, 1], [-1, 1, -1], [1, -1, -1]], dtype=float)
    tri = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], dtype=np.int32)
    m = inputs.Mesh(xyz, tri)
    A = oracle.system_matrix(m, 4.0, 80.0, 0.125, 1)
    x = np.random.default_rng(0).standard_normal(8)
    with pbm.MeshHandle(xyz, tri, _opts(1)) as h:
        y = pbm.pb_mesh_apply(h, x)
        yf = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_FAR_ONLY)
    assert _rel(y, A @ x) < 1e-12
    assert np.abs(yf).max() == 0.0


def test_high_valence_skinny_mesh_parity():
    """Bipyramid over an 80-gon: two vertices of valence 80, 160 triangles of
    aspect ratio about 25 and a sharp fold along the ring.  Near-field blocks,
    FP64 and FP32 operator products and both formulations' solves against the
    oracle (dense, every pair)."""
    m = inputs.bipyramid(80, 3.0, 3.0)
    tri = m.tri
    ts, ss = [], []
    for t in (0, 1, 79, 158):
        for s_ in range(m.n_triangles):
            if len(set(tri[t]) & set(tri[s_])) > 0:
                ts.append(t)
                ss.append(s_)
    ch = inputs.Charges(np.array([[0.0, 0.0, 0.0], [0.3, -0.2, 0.5], [-0.4, 0.1, -0.6]]),
                        np.array([1.0, -0.5, 0.7]))
    with pbm.MeshHandle(m.xyz, m.tri, _opts()) as h:
        got = pbm.pb_mesh_near_blocks(h, ts, ss)
    for k, (t, s_) in enumerate(zip(ts, ss)):
        VL, KL, _ = oracle.pair_block(m, t, s_, 0.0, 4)
        VY, KY, _ = oracle.pair_block(m, t, s_, 0.125, 4)
        ref = np.stack([VL, KL, VY, KY])
        assert np.abs(got[k] - ref).max() < 1e-13 * np.abs(ref[0]).max(), (t, s_)
    x = np.random.default_rng(17).standard_normal(2 * m.n_vertices)
    for form in (0, 1):
        A = oracle.system_matrix(m, 4.0, 80.0, 0.125, form)
        ref = A @ x
        for prec, tol in ((pbm.PB_FP64, 1e-12), (pbm.PB_FP32, 1e-5)):
            with pbm.MeshHandle(m.xyz, m.tri, _opts(form, prec)) as h:
                y = pbm.pb_mesh_apply(h, x)
            assert _rel(y, ref) < tol, (form, prec, _rel(y, ref))
        r = oracle.solve(m, ch, formulation=form, A=A)
        g = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form))
        assert g["status"] == pbm.PB_OK and g["iterations"] == r["iterations"]
        assert abs(g["dG"] - r["dG"]) < 1e-6 * abs(r["dG"]), (form, g["dG"], r["dG"])


def test_error_paths_on_device():
    m, ch = inputs.config_kirkwood(4, 2.0)
    with pytest.raises(pbm.PbError) as e:
        pbm.pb_solve(m.xyz, m.tri, np.array([[0.0, 0.0, 5.0]]), np.array([1.0]), _opts())
    assert e.value.code == pbm.PB_E_CHARGES
    with pytest.raises(pbm.PbError) as e:
        pbm.pb_solve(m.xyz, m.tri, np.array([[0.0, 0.0, np.nan]]), np.array([1.0]), _opts())
    assert e.value.code == pbm.PB_E_INVALID_ARG
    r = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(max_iter=1))
    assert r["status"] == pbm.PB_NOT_CONVERGED and r["iterations"] == 1


# ------------------------------------------------------------ assembled modes
@pytest.mark.parametrize("name", ["sphere6", "star7"])
@pytest.mark.parametrize("form", [0, 1])
def test_assembled_operator(meshes, dense_systems, name, form):
    """The dense far field (assembled once, vertex basis) reproduces the
    oracle's operator: 1e-12 with FP64 storage, 1e-5 with FP32 storage."""
    m = meshes[name]
    A = dense_systems[(name, form)]
    x = np.random.default_rng(13).standard_normal(2 * m.n_vertices)
    ref = A @ x
    for prec, tol in ((pbm.PB_FP64, 1e-12), (pbm.PB_FP32, 1e-5), (pbm.PB_MIXED_BF16, 1e-5),
                      (pbm.PB_MIXED_FP16, 1e-5)):
        with pbm.MeshHandle(m.xyz, m.tri, _opts(form, prec, operator_mode=pbm.PB_ASSEMBLED)) as h:
            assert h.info()["assembled"] == 1
            y = pbm.pb_mesh_apply(h, x)
            yf = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_FAR_ONLY)
            yn = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_NEAR_ONLY)
        assert _rel(y, ref) < tol, (prec, _rel(y, ref))
        assert _rel(yf + yn, ref) < tol


@pytest.mark.parametrize("prec", [pbm.PB_MIXED_BF16, pbm.PB_MIXED_FP16, pbm.PB_FP32])
@pytest.mark.parametrize("form", [0, 1])
def test_mixed_precision_solves(meshes, dense_systems, prec, form):
    """16-bit far field in the inner solves, FP64 iterative refinement on the
    accurate operator: Delta G within 1e-4 of the FP64 oracle."""
    m = meshes["star7"]
    ch = inputs.charges_ball(9, 20, 2.5)
    ref = oracle.solve(m, ch, formulation=form, A=dense_systems[("star7", form)])
    got = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, prec, operator_mode=pbm.PB_ASSEMBLED))
    assert got["status"] == pbm.PB_OK
    assert got["rel_residual"] <= 1e-5 * 1.001
    assert abs(got["dG"] - ref["dG"]) < 1e-4 * abs(ref["dG"]), (got["dG"], ref["dG"])
    if prec != pbm.PB_FP32:
        assert got["outer_iterations"] >= 1


def test_assembled_full_size_sampled_rows(sphere32):
    m, _ = sphere32
    rng = np.random.default_rng(23)
    x = rng.standard_normal(2 * m.n_vertices)
    rows = np.sort(rng.choice(m.n_vertices, 8, replace=False))
    r1, r2 = oracle.system_rows(m, 4.0, 80.0, 0.125, 0, rows, x)
    ref = np.concatenate([r1, r2])
    for prec, tol in ((pbm.PB_FP64, 1e-12), (pbm.PB_FP32, 2e-5)):
        with pbm.MeshHandle(m.xyz, m.tri, _opts(0, prec, operator_mode=pbm.PB_ASSEMBLED)) as h:
            y = pbm.pb_mesh_apply(h, x)
        nv = m.n_vertices
        assert _rel(np.concatenate([y[rows], y[nv + rows]]), ref) < tol


def test_full_size_mixed_solve(sphere32):
    """20480-triangle sphere: mixed BF16 / FP16 solves within 1e-4 of the FP64
    matrix-free GPU solve (whose Delta G test_full_size_dG_against_oracle
    checks against the oracle's)."""
    m, ch = sphere32
    for form in (0, 1):
        g64 = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form))
        for prec in (pbm.PB_MIXED_BF16, pbm.PB_MIXED_FP16):
            g = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, prec, operator_mode=pbm.PB_ASSEMBLED))
            assert g["status"] == pbm.PB_OK
            assert abs(g["dG"] - g64["dG"]) < 1e-4 * abs(g64["dG"]), (form, prec, g["dG"], g64["dG"])


# ------------------------------------------------------- several charge sets
def _sets(k0, n, nq=12, radius=2.5):
    return [inputs.charges_ball(k0 + k, nq, radius) for k in range(n)]


def test_solve_multi_fp32_bitwise_equals_single(meshes):
    """Batched lock-step GMRES runs each system's arithmetic exactly as a lone
    solve does: FP32 assembled results are bitwise identical alone and in the batch."""
    m = meshes["star7"]
    sets = _sets(100, 5)
    opt = _opts(1, pbm.PB_FP32, operator_mode=pbm.PB_ASSEMBLED)
    with pbm.MeshHandle(m.xyz, m.tri, opt) as h:
        multi = pbm.pb_solve_multi(h, [(c.xyz, c.q) for c in sets])
        single = [pbm.pb_mesh_solve(h, c.xyz, c.q) for c in sets]
    for a, b in zip(multi, single):
        assert a["dG"] == b["dG"] and a["iterations"] == b["iterations"]
        assert np.array_equal(a["phi"], b["phi"]) and np.array_equal(a["dphi"], b["dphi"])


@pytest.mark.parametrize("prec", [pbm.PB_MIXED_BF16, pbm.PB_MIXED_FP16])
@pytest.mark.parametrize("form", [0, 1])
def test_solve_multi_mfma_matches_oracle(meshes, dense_systems, prec, form):
    """16 right-hand sides through the MFMA GEMM (16-bit far field) with FP64
    refinement: every set's Delta G within 1e-4 of the oracle."""
    m = meshes["star7"]
    sets = _sets(200, 16)
    A = dense_systems[("star7", form)]
    with pbm.MeshHandle(m.xyz, m.tri, _opts(form, prec, operator_mode=pbm.PB_ASSEMBLED)) as h:
        multi = pbm.pb_solve_multi(h, [(c.xyz, c.q) for c in sets])
    for c, r in zip(sets, multi):
        ref = oracle.solve(m, c, formulation=form, A=A)
        assert r["status"] == pbm.PB_OK and r["rel_residual"] <= 1e-5 * 1.001
        assert abs(r["dG"] - ref["dG"]) < 1e-4 * abs(ref["dG"]), (r["dG"], ref["dG"])


def test_solve_multi_ragged_batch_and_full_size(sphere32):
    """20480-triangle sphere, 19 charge sets (a batch of 16 plus a ragged 3):
    mixed BF16 MFMA solves within 1e-4 of FP64 matrix-free GPU solves."""
    m, _ = sphere32
    sets = [inputs.charges_ball(40 + k, 50, 8.0) for k in range(19)]
    with pbm.MeshHandle(m.xyz, m.tri, _opts(0, pbm.PB_MIXED_BF16, operator_mode=pbm.PB_ASSEMBLED)) as h:
        multi = pbm.pb_solve_multi(h, [(c.xyz, c.q) for c in sets])
    with pbm.MeshHandle(m.xyz, m.tri, _opts(0)) as h64:
        for k in (0, 7, 15, 16, 18):
            ref = pbm.pb_mesh_solve(h64, sets[k].xyz, sets[k].q)
            assert abs(multi[k]["dG"] - ref["dG"]) < 1e-4 * abs(ref["dG"]), (k, multi[k]["dG"], ref["dG"])


def test_sixteen_sets_at_40962_vertices():
    """The 16-charge-set workload at its own size (frequency-64 sphere of radius
    10 A, 40962 vertices, 16 sets of 50 charges): the MFMA GEMM path with BF16
    and FP16 storage.  Anchors: the FP64 GPU operator matches oracle rows on
    this mesh; every set's solution leaves a preconditioned residual of at most
    the tolerance (plus the FP32 far field's rounding) under that FP64
    operator; two sets' Delta G within 1e-4 of FP64 GPU solves."""
    m, sets = inputs.config_sphere_multi()
    nv = m.n_vertices
    rng = np.random.default_rng(41)
    x = rng.standard_normal(2 * nv)
    rows = np.sort(rng.choice(nv, 6, replace=False))
    r1, r2 = oracle.system_rows(m, 4.0, 80.0, 0.125, 0, rows, x)
    with pbm.MeshHandle(m.xyz, m.tri, _opts(0)) as h64:
        y = pbm.pb_mesh_apply(h64, x)
        assert _rel(np.concatenate([y[rows], y[nv + rows]]), np.concatenate([r1, r2])) < 1e-12
        pinv = pbm.pb_mesh_preconditioner(h64)
        refs = {k: pbm.pb_mesh_solve(h64, sets[k].xyz, sets[k].q) for k in (0, 15)}
        for prec in (pbm.PB_MIXED_BF16, pbm.PB_MIXED_FP16):
            with pbm.MeshHandle(m.xyz, m.tri, _opts(0, prec, operator_mode=pbm.PB_ASSEMBLED)) as h:
                multi = pbm.pb_solve_multi(h, [(c.xyz, c.q) for c in sets])
            for k, (c, r) in enumerate(zip(sets, multi)):
                assert r["status"] == pbm.PB_OK and r["rel_residual"] <= 1e-5 * 1.001, (prec, k)
                b = pbm.pb_mesh_rhs(h64, c.xyz, c.q)
                b[nv:] = 0.0                      # the direct formulation's right-hand side [b_D; 0]
                u = np.concatenate([r["phi"], r["dphi"]])
                res = oracle.apply_block_diag(pinv.reshape(nv, 2, 2), b - pbm.pb_mesh_apply(h64, u))
                pb = oracle.apply_block_diag(pinv.reshape(nv, 2, 2), b)
                assert np.linalg.norm(res) <= 1.2e-5 * np.linalg.norm(pb), (prec, k)
                if k in refs:
                    assert abs(r["dG"] - refs[k]["dG"]) < 1e-4 * abs(refs[k]["dG"]), (prec, k)


# ------------------------------------------------------------------ serving
def _requests():
    out = []
    for k, (f, prec, form) in enumerate([(4, pbm.PB_MIXED_BF16, 0), (9, pbm.PB_FP32, 1), (6, pbm.PB_MIXED_FP16, 1),
                                         (12, pbm.PB_MIXED_BF16, 1), (5, pbm.PB_FP32, 0), (10, pbm.PB_MIXED_BF16, 0)]):
        base = 18.0 * (20 * f * f / 81920.0) ** 0.5
        mesh, shape = inputs.star_surface(300 + k, f, base)
        ch = inputs.charges_in_star(400 + k, 30 + 10 * k, shape, values="uniform")
        opt = pbm.pb_default_options(formulation=form, precision=prec, operator_mode=pbm.PB_ASSEMBLED)
        out.append((mesh, ch, opt))
    return out


def test_server_same_alone_and_in_the_mix():
    """Requests of different sizes, formulations and precisions run together on
    the server (overlapping on the device) give bitwise the results they give
    alone."""
    reqs = _requests()
    alone = []
    for mesh, ch, opt in reqs:
        o = pbm.pb_default_options()
        for f, _ in pbm.pb_options._fields_:
            setattr(o, f, getattr(opt, f))
        o.memory_budget = pbm.pb_estimate_device_bytes(mesh.xyz, mesh.tri, opt)
        alone.append(pbm.pb_solve(mesh.xyz, mesh.tri, ch.xyz, ch.q, o))
    with pbm.Server(max_slots=4) as s:
        tickets = [s.submit(m.xyz, m.tri, c.xyz, c.q, o) for m, c, o in reqs]
        mixed = [s.wait(t) for t in tickets]
        st = s.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["peak_running"] >= 2, st
    for a, b in zip(alone, mixed):
        assert a["dG"] == b["dG"] and a["iterations"] == b["iterations"]
        assert np.array_equal(a["phi"], b["phi"]) and np.array_equal(a["dphi"], b["dphi"])
    # and every served result against the FP64 oracle on the same inputs
    # (FP32 and mixed 16-bit far fields: the reduced-precision bound 1e-4)
    for (mesh, ch, opt), b in zip(reqs, mixed):
        ref = oracle.solve(mesh, ch, formulation=opt.formulation)
        assert abs(b["dG"] - ref["dG"]) < 1e-4 * abs(ref["dG"]), (mesh.n_triangles, b["dG"], ref["dG"])


def test_server_reused_blocks_change_nothing():
    """Requests large enough for the server's block cache (assembled far fields
    of 0.5 to 1.7 GB, near-field blocks above 64 MiB), repeated and interleaved
    so that later ones run in blocks earlier ones left (of the same or another
    size, holding their stale values): bitwise the results they give alone."""
    reqs = []
    for k, (f, prec, form) in enumerate([(24, pbm.PB_MIXED_BF16, 1), (32, pbm.PB_FP32, 0), (28, pbm.PB_MIXED_FP16, 0)]):
        base = 18.0 * (20 * f * f / 81920.0) ** 0.5
        mesh, shape = inputs.star_surface(500 + k, f, base)
        ch = inputs.charges_in_star(600 + k, 40, shape, values="uniform")
        reqs.append((mesh, ch, pbm.pb_default_options(formulation=form, precision=prec,
                                                      operator_mode=pbm.PB_ASSEMBLED)))
    alone = []
    for mesh, ch, opt in reqs:
        o = pbm.pb_default_options()
        for f, _ in pbm.pb_options._fields_:
            setattr(o, f, getattr(opt, f))
        o.memory_budget = pbm.pb_estimate_device_bytes(mesh.xyz, mesh.tri, opt)
        alone.append(pbm.pb_solve(mesh.xyz, mesh.tri, ch.xyz, ch.q, o))
    order = [0, 1, 2, 0, 1, 2, 1]
    with pbm.Server(max_slots=2) as s:
        got = []
        for k in order:   # one at a time, so every later request finds idle blocks
            m, c, o = reqs[k]
            got.append(s.wait(s.submit(m.xyz, m.tri, c.xyz, c.q, o)))
        tickets = [s.submit(reqs[k][0].xyz, reqs[k][0].tri, reqs[k][1].xyz, reqs[k][1].q, reqs[k][2])
                   for k in order]
        got += [s.wait(t) for t in tickets]
        st = s.stats()
    assert st["failed"] == 0
    for k, b in zip(order + order, got):
        a = alone[k]
        assert a["dG"] == b["dG"] and a["iterations"] == b["iterations"]
        assert np.array_equal(a["phi"], b["phi"]) and np.array_equal(a["dphi"], b["dphi"])


def test_server_admission_by_footprint_and_cancel():
    """Equal-size requests under a budget that fits only one of them run one
    at a time; a queued request can be cancelled; results stay correct."""
    mesh, ch, opt = _requests()[3]
    sets = [inputs.charges_ball(500 + k, 20, 2.0) for k in range(3)]
    est = pbm.pb_estimate_device_bytes(mesh.xyz, mesh.tri, opt)
    with pbm.Server(hbm_budget=int(est * 1.5), max_slots=4) as s:
        tickets = [s.submit(mesh.xyz, mesh.tri, c.xyz, c.q, opt) for c in sets]
        extra = s.submit(mesh.xyz, mesh.tri, ch.xyz, ch.q, opt)
        try:
            s.cancel(extra)
            cancelled = True
        except pbm.PbError as e:
            assert e.code == pbm.PB_E_STATE     # it had already started
            cancelled = False
        res = [s.wait(t) for t in tickets]
        if not cancelled:
            s.wait(extra)
        st = s.stats()
    assert st["peak_running"] == 1, st
    assert st["peak_inflight_bytes"] <= int(est * 1.5)
    for r in res:
        assert r["status"] == pbm.PB_OK
    spans = sorted((r["t_start"], r["t_end"]) for r in res)
    for (s0, e0), (s1, e1) in zip(spans, spans[1:]):
        assert s1 >= e0 - 1e-3, spans     # never two requests on the device at once


def test_star_full_size_sampled_rows():
    """Star surface, 81920 triangles / 40962 vertices (the matrix-free FP32
    configuration): sampled rows of A x for both formulations against rows the
    oracle computes, in the launch configuration the benchmark uses."""
    m, _ = inputs.config_star()
    rng = np.random.default_rng(31)
    x = rng.standard_normal(2 * m.n_vertices)
    rows = np.sort(rng.choice(m.n_vertices, 4, replace=False))
    nv = m.n_vertices
    for form in (0, 1):
        r1, r2 = oracle.system_rows(m, 4.0, 80.0, 0.125, form, rows, x)
        ref = np.concatenate([r1, r2])
        for prec, tol in ((pbm.PB_FP32, 2e-5), (pbm.PB_FP64, 1e-12)):
            with pbm.MeshHandle(m.xyz, m.tri, _opts(form, prec)) as h:
                y = pbm.pb_mesh_apply(h, x)
            assert _rel(np.concatenate([y[rows], y[nv + rows]]), ref) < tol, (form, prec)


# ---------------------------------------------------------- captured GMRES
@pytest.mark.parametrize("prec,mode", [(pbm.PB_FP64, pbm.PB_MATRIX_FREE), (pbm.PB_FP32, pbm.PB_ASSEMBLED),
                                       (pbm.PB_MIXED_BF16, pbm.PB_ASSEMBLED)])
@pytest.mark.parametrize("form", [0, 1])
def test_graph_gmres_matches_eager(meshes, prec, mode, form):
    """GMRES iterations replayed from a captured HIP graph (device Givens) give
    the eager solve's iterations and Delta G; the graph is replayed across
    several solves on one handle with eager work between them."""
    m = meshes["star7"]
    sets = [inputs.charges_ball(600 + k, 15, 2.5) for k in range(3)]
    x = np.random.default_rng(3).standard_normal(2 * m.n_vertices)
    og = _opts(form, prec, operator_mode=mode)
    oe = _opts(form, prec, operator_mode=mode, use_graph=0)
    with pbm.MeshHandle(m.xyz, m.tri, og) as hg, pbm.MeshHandle(m.xyz, m.tri, oe) as he:
        for c in sets:
            rg = pbm.pb_mesh_solve(hg, c.xyz, c.q)
            yg = pbm.pb_mesh_apply(hg, x)          # eager work between graph replays
            re = pbm.pb_mesh_solve(he, c.xyz, c.q)
            ye = pbm.pb_mesh_apply(he, x)
            assert np.array_equal(yg, ye)
            assert rg["iterations"] == re["iterations"] and rg["outer_iterations"] == re["outer_iterations"]
            assert abs(rg["dG"] - re["dG"]) <= 1e-12 * abs(re["dG"])
            assert rg["status"] == pbm.PB_OK


def test_graph_gmres_small_and_nonconverged():
    """Kirkwood sphere (tiny, launch-latency bound) through the graph path, and
    a max_iter stop inside a replay batch."""
    m, ch = inputs.config_kirkwood(4, 2.0)
    ref = oracle.solve(m, ch)
    r = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts())
    assert abs(r["dG"] - ref["dG"]) < 1e-6 * abs(ref["dG"]) and r["iterations"] == ref["iterations"]
    r3 = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(max_iter=3))
    assert r3["status"] == pbm.PB_NOT_CONVERGED and r3["iterations"] == 3


# ------------------------------------------- (scaled) mass preconditioners
_MASS_CASES = [(0, pbm.PB_MASS), (1, pbm.PB_MASS), (1, pbm.PB_SCALED_MASS)]


def _mass_ref(m, form, prec):
    a, b = oracle.mass_scales(4.0, 80.0, form, prec == pbm.PB_SCALED_MASS)
    return oracle.mass_preconditioner(m, a, b)


@pytest.mark.parametrize("form,prec", _MASS_CASES)
@pytest.mark.parametrize("name", ["sphere6", "star7"])
def test_mass_preconditioner_product(meshes, dense_systems, name, form, prec):
    """blockdiag(aM, bM)^-1 A x (Eqs. prec:mass, prec:mass:scaled): the GPU's
    fixed-degree Chebyshev inverse of the mass matrix is within 2 (1/3)^20 of
    the oracle's Cholesky solve; checked on the whole preconditioned product."""
    m = meshes[name]
    A = dense_systems[(name, form)]
    x = np.random.default_rng(31).standard_normal(2 * m.n_vertices)
    P = _mass_ref(m, form, prec)
    with pbm.MeshHandle(m.xyz, m.tri, _opts(form, preconditioner=prec)) as h:
        y = pbm.pb_mesh_apply(h, x)
        yp = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_PRECOND)
        yp2 = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_PRECOND)
    assert _rel(y, A @ x) < 1e-12
    assert np.array_equal(yp, yp2)
    assert _rel(yp, P(A @ x)) < 2e-9


@pytest.mark.parametrize("form,prec", _MASS_CASES)
def test_mass_preconditioned_solve_parity(meshes, dense_systems, form, prec):
    """Kirkwood sphere and a 980-triangle star: the mass-preconditioned GPU
    solve takes the oracle's iterations and gives its Delta G (FP64 1e-6,
    FP32 assembled 1e-4); at tight tolerance the traces agree to 1e-8."""
    sp = "scaled_mass" if prec == pbm.PB_SCALED_MASS else "mass"
    m, ch = inputs.config_kirkwood(4, 2.0)
    ref = oracle.solve(m, ch, formulation=form, preconditioner=sp)
    got = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, preconditioner=prec))
    assert got["status"] == pbm.PB_OK
    assert got["iterations"] == ref["iterations"]
    assert abs(got["dG"] - ref["dG"]) < 1e-6 * abs(ref["dG"])
    tight = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, preconditioner=prec, tol=1e-11))
    reft = oracle.solve(m, ch, formulation=form, preconditioner=sp, tol=1e-11, A=ref["A"])
    u = np.concatenate([tight["phi"], tight["dphi"]])
    assert _rel(u, np.concatenate([reft["phi"], reft["dphi"]])) < 1e-8
    ms = meshes["star7"]
    chs = inputs.charges_ball(9, 20, 2.5)
    refs = oracle.solve(ms, chs, formulation=form, preconditioner=sp, A=dense_systems[("star7", form)])
    for p, mode, tol in ((pbm.PB_FP64, pbm.PB_MATRIX_FREE, 1e-6), (pbm.PB_FP32, pbm.PB_ASSEMBLED, 1e-4),
                         (pbm.PB_MIXED_BF16, pbm.PB_ASSEMBLED, 1e-4)):
        g = pbm.pb_solve(ms.xyz, ms.tri, chs.xyz, chs.q, _opts(form, p, preconditioner=prec, operator_mode=mode))
        assert g["status"] == pbm.PB_OK
        assert abs(g["dG"] - refs["dG"]) < tol * abs(refs["dG"]), (p, g["dG"], refs["dG"])
        if p == pbm.PB_FP64:
            assert abs(g["iterations"] - refs["iterations"]) <= 1


def test_mass_preconditioner_graph_batch_and_options(meshes):
    """Captured and eager GMRES give the same iterations and Delta G with the
    scaled mass preconditioner; batched solves are bitwise the single ones;
    the scaled mass matrix is refused for the direct formulation."""
    m = meshes["star7"]
    sets = _sets(700, 3)
    og = _opts(1, pbm.PB_FP32, preconditioner=pbm.PB_SCALED_MASS, operator_mode=pbm.PB_ASSEMBLED)
    oe = _opts(1, pbm.PB_FP32, preconditioner=pbm.PB_SCALED_MASS, operator_mode=pbm.PB_ASSEMBLED, use_graph=0)
    with pbm.MeshHandle(m.xyz, m.tri, og) as hg, pbm.MeshHandle(m.xyz, m.tri, oe) as he:
        multi = pbm.pb_solve_multi(hg, [(c.xyz, c.q) for c in sets])
        for c, mb in zip(sets, multi):
            rg = pbm.pb_mesh_solve(hg, c.xyz, c.q)
            re = pbm.pb_mesh_solve(he, c.xyz, c.q)
            assert rg["iterations"] == re["iterations"] and abs(rg["dG"] - re["dG"]) <= 1e-12 * abs(re["dG"])
            assert mb["dG"] == re["dG"] and np.array_equal(mb["phi"], re["phi"])
    with pytest.raises(pbm.PbError):
        pbm.pb_solve(m.xyz, m.tri, sets[0].xyz, sets[0].q, _opts(0, preconditioner=pbm.PB_SCALED_MASS))


def test_mass_preconditioner_full_size_rows(sphere32):
    """20480-triangle sphere, Juffer, scaled mass, FP32 assembled: a M y_p
    equals the unpreconditioned product y on sampled rows (M rows from the
    oracle); the solve converges in fewer iterations than with the
    block-diagonal preconditioner (the paper's Case 10)."""
    m, ch = sphere32
    nv = m.n_vertices
    rng = np.random.default_rng(41)
    x = rng.standard_normal(2 * nv)
    rows = np.sort(rng.choice(nv, 12, replace=False))
    Mr = oracle.mass_rows(m, rows)
    a, b = oracle.mass_scales(4.0, 80.0, 1, True)
    opt = _opts(1, pbm.PB_FP32, preconditioner=pbm.PB_SCALED_MASS, operator_mode=pbm.PB_ASSEMBLED)
    with pbm.MeshHandle(m.xyz, m.tri, opt) as h:
        y = pbm.pb_mesh_apply(h, x)
        yp = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_PRECOND)
        r = pbm.pb_mesh_solve(h, ch.xyz, ch.q)
    got = np.concatenate([a * (Mr @ yp[:nv]), b * (Mr @ yp[nv:])])
    ref = np.concatenate([y[rows], y[nv + rows]])
    assert _rel(got, ref) < 1e-8
    bd = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(1, pbm.PB_FP32, operator_mode=pbm.PB_ASSEMBLED))
    assert r["status"] == pbm.PB_OK and r["iterations"] < bd["iterations"], (r["iterations"], bd["iterations"])
    assert abs(r["dG"] - bd["dG"]) < 1e-4 * abs(bd["dG"])


# ------------------------------------------------------ every formulation
_FORMS = [pbm.PB_DIRECT_INT, pbm.PB_JUFFER, pbm.PB_DIRECT_EXT, pbm.PB_DIRECT_INT_PERM, pbm.PB_DIRECT_EXT_PERM,
          pbm.PB_MULLER_INT, pbm.PB_MULLER_EXT, pbm.PB_LU, pbm.PB_PMCHWT_INT, pbm.PB_PMCHWT_EXT]
_DIRECT_FAMILY = (pbm.PB_DIRECT_INT, pbm.PB_DIRECT_EXT, pbm.PB_DIRECT_INT_PERM, pbm.PB_DIRECT_EXT_PERM)


@pytest.fixture(scope="module")
def base_operators(meshes):
    """V, K, D, T = K^T of both kernels and M on the 980-triangle star, from
    which every formulation's system is composed as the paper prints it."""
    m = meshes["star7"]
    oL = oracle.assemble(m, 0.0, ("V", "K", "D"))
    oY = oracle.assemble(m, 0.125, ("V", "K", "D"))
    for o in (oL, oY):
        o["T"] = o["K"].T.copy()
    return oL, oY, oracle.mass(m)


def _system(base, form):
    A11, A12, A21, A22 = oracle.system_blocks(base[0], base[1], base[2], 4.0, 80.0, form)
    return np.block([[A11, A12], [A21, A22]])


@pytest.mark.parametrize("form", _FORMS)
def test_formulation_operator(meshes, base_operators, form):
    """The library's coefficient model of each formulation (combination of the
    interior and exterior trace equations) against the oracle's systems typed
    in as printed: matrix-free FP64 (1e-12), assembled FP64 (1e-12), assembled
    FP32 one evaluation per pair (1e-5) and matrix-free FP32 (1e-5)."""
    m = meshes["star7"]
    A = _system(base_operators, form)
    x = np.random.default_rng(71 + form).standard_normal(2 * m.n_vertices)
    ref = A @ x
    for prec, mode, tol in ((pbm.PB_FP64, pbm.PB_MATRIX_FREE, 1e-12), (pbm.PB_FP64, pbm.PB_ASSEMBLED, 1e-12),
                            (pbm.PB_FP32, pbm.PB_ASSEMBLED, 1e-5), (pbm.PB_FP32, pbm.PB_MATRIX_FREE, 1e-5)):
        with pbm.MeshHandle(m.xyz, m.tri, _opts(form, prec, operator_mode=mode)) as h:
            y = pbm.pb_mesh_apply(h, x)
        assert _rel(y, ref) < tol, (form, prec, mode, _rel(y, ref))


@pytest.mark.parametrize("form", _FORMS)
def test_formulation_solve_parity(form):
    """Kirkwood sphere: each formulation (block-diagonal preconditioner for the
    direct ones, mass matrix for the others, as the paper pairs them) takes the
    oracle's iterations and gives its Delta G and interior traces; exterior
    unknowns come back as interior traces."""
    m, ch = inputs.config_kirkwood(4, 2.0)
    direct = form in _DIRECT_FAMILY
    ref = oracle.solve(m, ch, formulation=form, preconditioner=True if direct else "mass")
    got = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q,
                       _opts(form, preconditioner=pbm.PB_BLOCK_DIAG if direct else pbm.PB_MASS))
    assert got["status"] == pbm.PB_OK
    assert got["iterations"] == ref["iterations"], (form, got["iterations"], ref["iterations"])
    assert abs(got["dG"] - ref["dG"]) < 1e-6 * abs(ref["dG"])
    assert _rel(np.concatenate([got["phi"], got["dphi"]]), np.concatenate([ref["phi"], ref["dphi"]])) < 1e-5
    g32 = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q,
                       _opts(form, pbm.PB_FP32, operator_mode=pbm.PB_ASSEMBLED,
                             preconditioner=pbm.PB_BLOCK_DIAG if direct else pbm.PB_MASS))
    assert abs(g32["dG"] - ref["dG"]) < 1e-4 * abs(ref["dG"])


@pytest.mark.parametrize("form", [0, 1])
def test_one_point_regular_rule(meshes, form):
    """regular_order 1: the one-point rule on every pair sharing no vertex,
    matrix-free in FP64 (1e-12) and FP32 (1e-5) against the oracle's system
    with the same rule; the solve's iterations and Delta G (1e-6) against the
    oracle's; the modes that cannot take it are refused."""
    m = meshes["star7"]
    A = oracle.system_matrix(m, 4.0, 80.0, 0.125, form, centroid=True)
    x = np.random.default_rng(93).standard_normal(2 * m.n_vertices)
    ref = A @ x
    for prec, tol in ((pbm.PB_FP64, 1e-12), (pbm.PB_FP32, 1e-5)):
        with pbm.MeshHandle(m.xyz, m.tri, _opts(form, prec, regular_order=1)) as h:
            assert _rel(pbm.pb_mesh_apply(h, x), ref) < tol, (form, prec)
    with pbm.MeshHandle(m.xyz, m.tri, _opts(form, pbm.PB_FP32, operator_mode=pbm.PB_AUTO, regular_order=1)) as h:
        assert h.info()["assembled"] == 0
    ch = inputs.charges_ball(9, 20, 2.5)
    r = oracle.solve(m, ch, formulation=form, A=A)
    g = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, regular_order=1))
    assert g["status"] == pbm.PB_OK and abs(g["iterations"] - r["iterations"]) <= 1
    assert abs(g["dG"] - r["dG"]) < 1e-6 * abs(r["dG"]), (g["dG"], r["dG"])
    for kw in ({"operator_mode": pbm.PB_ASSEMBLED}, {"operator_mode": pbm.PB_TREECODE},
               {"precision": pbm.PB_MIXED_BF16}):
        with pytest.raises(pbm.PbError) as e:
            pbm.MeshHandle(m.xyz, m.tri, _opts(form, regular_order=1, **kw))
        assert e.value.code == pbm.PB_E_INVALID_ARG


_CFIE_CASES = [(pbm.PB_CFIE_INT, 0.5, 2.0), (pbm.PB_CFIE_INT, 0.0, 3.0), (pbm.PB_CFIE_EXT, 3.0, 0.25),
               (pbm.PB_CFIE_EXT, 0.0, 1.0), (pbm.PB_CFIE_EXT, 1.0, 0.0), (pbm.PB_CFIE_EXT, 0.0, 0.0)]


def _degenerate(form, a, b):
    """External combined field with one zero constant: one block row without a
    Laplace term, the other with one."""
    return form == pbm.PB_CFIE_EXT and (a == 0.0) != (b == 0.0)


@pytest.mark.parametrize("form,a,b", _CFIE_CASES)
def test_cfie_operator(meshes, base_operators, form, a, b):
    """Combined-field systems with general and zero constants (Eqs.
    bie:combined:int, bie:combined:ext) against the oracle's typed system:
    matrix-free and assembled FP64 (1e-12) and FP32 (1e-5), and the treecode
    without separated clusters
    (the direct sums, 1e-12).  A zero constant leaves blocks without a
    Laplace term, which the assembly takes with both coefficients inside the
    kernel values (PB_AUTO assembles them too)."""
    m = meshes["star7"]
    A11, A12, A21, A22 = oracle.system_blocks(base_operators[0], base_operators[1], base_operators[2], 4.0, 80.0,
                                              form, a, b)
    A = np.block([[A11, A12], [A21, A22]])
    x = np.random.default_rng(91).standard_normal(2 * m.n_vertices)
    ref = A @ x
    modes = [(pbm.PB_FP64, pbm.PB_MATRIX_FREE, 1e-12), (pbm.PB_FP32, pbm.PB_MATRIX_FREE, 1e-5),
             (pbm.PB_FP64, pbm.PB_ASSEMBLED, 1e-12), (pbm.PB_FP32, pbm.PB_ASSEMBLED, 1e-5)]
    for prec, mode, tol in modes:
        with pbm.MeshHandle(m.xyz, m.tri, _opts(form, prec, operator_mode=mode, cfie_alpha=a, cfie_beta=b)) as h:
            assert h.info()["assembled"] == (1 if mode == pbm.PB_ASSEMBLED else 0)
            y = pbm.pb_mesh_apply(h, x)
        assert _rel(y, ref) < tol, (form, a, b, prec, mode, _rel(y, ref))
    with pbm.MeshHandle(m.xyz, m.tri, _opts(form, operator_mode=pbm.PB_TREECODE, tree_theta=1e-3,
                                            cfie_alpha=a, cfie_beta=b)) as h:
        assert _rel(pbm.pb_mesh_apply(h, x), ref) < 1e-12
    if _degenerate(form, a, b):
        with pbm.MeshHandle(m.xyz, m.tri, _opts(form, pbm.PB_FP32, operator_mode=pbm.PB_AUTO,
                                                cfie_alpha=a, cfie_beta=b)) as h:
            assert h.info()["assembled"] == 1
            assert _rel(pbm.pb_mesh_apply(h, x), ref) < 1e-5


def test_cfie_without_coupling_is_applied_not_solved():
    """alpha = beta = 0 keeps one side's trace equations only: the operator is
    applied (checked against the oracle above), every solve entry point
    refuses it with PB_E_STATE."""
    m, ch = inputs.config_kirkwood(4, 2.0)
    for form in (pbm.PB_CFIE_INT, pbm.PB_CFIE_EXT):
        opt = pbm.pb_default_options(formulation=form, cfie_alpha=0.0, cfie_beta=0.0)
        with pbm.MeshHandle(m.xyz, m.tri, opt) as h:
            assert np.all(np.isfinite(pbm.pb_mesh_apply(h, np.ones(2 * m.n_vertices))))
            for call in (lambda: pbm.pb_mesh_solve(h, ch.xyz, ch.q),
                         lambda: pbm.pb_solve_multi(h, [(ch.xyz, ch.q)]),
                         lambda: pbm.pb_solve_batch([h], [(ch.xyz, ch.q)])):
                with pytest.raises(pbm.PbError) as e:
                    call()
                assert e.value.code == pbm.PB_E_STATE
        with pytest.raises(pbm.PbError) as e:
            pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, opt)
        assert e.value.code == pbm.PB_E_STATE


@pytest.mark.parametrize("form,a,b", [c for c in _CFIE_CASES if c[1:] != (0.0, 0.0)])
def test_cfie_solve_parity(form, a, b):
    """Kirkwood sphere with the mass preconditioner: the oracle's iterations
    and Delta G (1e-6 in FP64, 1e-4 in FP32)."""
    m, ch = inputs.config_kirkwood(4, 2.0)
    ref = oracle.solve(m, ch, formulation=form, preconditioner="mass", alpha=a, beta=b)
    got = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, preconditioner=pbm.PB_MASS, cfie_alpha=a,
                                                          cfie_beta=b))
    assert got["status"] == pbm.PB_OK
    assert got["iterations"] == ref["iterations"], (form, a, b, got["iterations"], ref["iterations"])
    assert abs(got["dG"] - ref["dG"]) < 1e-6 * abs(ref["dG"]), (form, a, b, got["dG"], ref["dG"])
    g32 = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, pbm.PB_FP32, preconditioner=pbm.PB_MASS,
                                                          cfie_alpha=a, cfie_beta=b))
    assert abs(g32["dG"] - ref["dG"]) < 1e-4 * abs(ref["dG"])


def test_lu_full_size(sphere32):
    """20480-triangle sphere, Lu formulation (exterior unknowns) with the mass
    preconditioner (the paper's Case 12): sampled rows of A x in FP32 assembled
    against the oracle, and the FP32 / BF16 solves within 1e-4 of the FP64
    matrix-free GPU solve."""
    m, ch = sphere32
    nv = m.n_vertices
    rng = np.random.default_rng(29)
    x = rng.standard_normal(2 * nv)
    rows = np.sort(rng.choice(nv, 8, replace=False))
    r1, r2 = oracle.system_rows(m, 4.0, 80.0, 0.125, oracle.LU, rows, x)
    ref = np.concatenate([r1, r2])
    with pbm.MeshHandle(m.xyz, m.tri, _opts(pbm.PB_LU, pbm.PB_FP32, operator_mode=pbm.PB_ASSEMBLED,
                                            preconditioner=pbm.PB_MASS)) as h:
        y = pbm.pb_mesh_apply(h, x)
        r32 = pbm.pb_mesh_solve(h, ch.xyz, ch.q)
    assert _rel(np.concatenate([y[rows], y[nv + rows]]), ref) < 2e-5
    g64 = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(pbm.PB_LU, preconditioner=pbm.PB_MASS))
    gbf = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(pbm.PB_LU, pbm.PB_MIXED_BF16, operator_mode=pbm.PB_ASSEMBLED,
                                                          preconditioner=pbm.PB_MASS))
    for g in (r32, gbf):
        assert g["status"] == pbm.PB_OK and abs(g["dG"] - g64["dG"]) < 1e-4 * abs(g64["dG"])


# ------------------------------------------- Calderon preconditioners (PMCHWT)
_CALDERON = [(pbm.PB_CALDERON, "calderon"), (pbm.PB_CALDERON_INT, "calderon_int"),
             (pbm.PB_CALDERON_EXT, "calderon_ext"), (pbm.PB_SCALED_CALDERON_INT, "scaled_calderon_int"),
             (pbm.PB_SCALED_CALDERON_EXT, "scaled_calderon_ext")]


def _calderon_ref(m, base, form, name):
    part = oracle.calderon_part(name)
    Pb = oracle.calderon_blocks(base[0], base[1], base[2], 4.0, 80.0, form, part)
    a, b = oracle.calderon_scales(4.0, 80.0, form, part) if name.startswith("scaled") else (1.0, 1.0)
    return oracle.calderon_preconditioner(m, np.block([[Pb[0], Pb[1]], [Pb[2], Pb[3]]]), a, b)


@pytest.mark.parametrize("prec,name", _CALDERON)
@pytest.mark.parametrize("form", [pbm.PB_PMCHWT_INT, pbm.PB_PMCHWT_EXT])
def test_calderon_product(meshes, base_operators, form, prec, name):
    """B A x with B = blockdiag(aM, bM)^-1 P blockdiag(M, M)^-1 (Eqs.
    prec:calderon:int, prec:calderon:ext) on the 980-triangle star, against
    the oracle's dense P, A and Cholesky mass solves: FP64 matrix-free and
    assembled within the two Chebyshev mass inverses (2e-9), FP32 within the
    FP32 far field's 1e-5 carried through M^-1 P M^-1, where the rounding of
    the far field is spread over all frequencies (2e-6; 2.5e-7 measured)."""
    m = meshes["star7"]
    A = _system(base_operators, form)
    B = _calderon_ref(m, base_operators, form, name)
    x = np.random.default_rng(91 + prec).standard_normal(2 * m.n_vertices)
    ref = B(A @ x)
    for p, mode, tol in ((pbm.PB_FP64, pbm.PB_MATRIX_FREE, 2e-9), (pbm.PB_FP64, pbm.PB_ASSEMBLED, 2e-9),
                         (pbm.PB_FP32, pbm.PB_ASSEMBLED, 2e-6), (pbm.PB_FP32, pbm.PB_MATRIX_FREE, 2e-6)):
        with pbm.MeshHandle(m.xyz, m.tri, _opts(form, p, operator_mode=mode, preconditioner=prec)) as h:
            y = pbm.pb_mesh_apply(h, x)
            yp = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_PRECOND)
            yp2 = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_PRECOND)
        assert np.array_equal(yp, yp2)
        assert _rel(y, A @ x) < (1e-12 if p == pbm.PB_FP64 else 1e-5)
        print(f"calderon product form {form} {name} prec {p} mode {mode}: rel {_rel(yp, ref):.2e}")
        assert _rel(yp, ref) < tol, (p, mode, _rel(yp, ref))


@pytest.mark.parametrize("prec,name", _CALDERON)
@pytest.mark.parametrize("form", [pbm.PB_PMCHWT_INT, pbm.PB_PMCHWT_EXT])
def test_calderon_solve_parity(form, prec, name):
    """Kirkwood sphere: each Calderon variant takes the oracle's iterations and
    gives its Delta G; at tight tolerance the traces agree with the oracle's;
    FP32 assembled and BF16 mixed solves land within 1e-4."""
    m, ch = inputs.config_kirkwood(4, 2.0)
    ref = oracle.solve(m, ch, formulation=form, preconditioner=name)
    got = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, preconditioner=prec))
    assert got["status"] == pbm.PB_OK
    assert got["iterations"] == ref["iterations"], (got["iterations"], ref["iterations"])
    assert abs(got["dG"] - ref["dG"]) < 1e-6 * abs(ref["dG"])
    tight = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, preconditioner=prec, tol=1e-11))
    reft = oracle.solve(m, ch, formulation=form, preconditioner=name, tol=1e-11, A=ref["A"])
    u = np.concatenate([tight["phi"], tight["dphi"]])
    assert _rel(u, np.concatenate([reft["phi"], reft["dphi"]])) < 1e-8
    for p in (pbm.PB_FP32, pbm.PB_MIXED_BF16):
        g = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, p, operator_mode=pbm.PB_ASSEMBLED,
                                                            preconditioner=prec))
        assert g["status"] == pbm.PB_OK and abs(g["dG"] - ref["dG"]) < 1e-4 * abs(ref["dG"]), (p, g["dG"])


def test_calderon_graph_and_refusals(meshes):
    """Captured and eager GMRES agree with a half Calderon preconditioner on the
    star (FP32 assembled, two dense operators); Calderon preconditioners are
    refused for other formulations and for batched solves."""
    m = meshes["star7"]
    sets = _sets(900, 2)
    for prec in (pbm.PB_CALDERON, pbm.PB_SCALED_CALDERON_EXT):
        og = _opts(pbm.PB_PMCHWT_INT, pbm.PB_FP32, preconditioner=prec, operator_mode=pbm.PB_ASSEMBLED)
        oe = _opts(pbm.PB_PMCHWT_INT, pbm.PB_FP32, preconditioner=prec, operator_mode=pbm.PB_ASSEMBLED,
                   use_graph=0)
        with pbm.MeshHandle(m.xyz, m.tri, og) as hg, pbm.MeshHandle(m.xyz, m.tri, oe) as he:
            for c in sets:
                rg = pbm.pb_mesh_solve(hg, c.xyz, c.q)
                re = pbm.pb_mesh_solve(he, c.xyz, c.q)
                assert rg["status"] == pbm.PB_OK
                assert rg["iterations"] == re["iterations"] and abs(rg["dG"] - re["dG"]) <= 1e-12 * abs(re["dG"])
            with pytest.raises(pbm.PbError):
                pbm.pb_solve_multi(hg, [(c.xyz, c.q) for c in sets])
    with pytest.raises(pbm.PbError):
        pbm.pb_solve(m.xyz, m.tri, sets[0].xyz, sets[0].q, _opts(pbm.PB_JUFFER, preconditioner=pbm.PB_CALDERON))


def test_calderon_full_size(sphere32):
    """20480-triangle sphere, internal PMCHWT, FP32 assembled: with
    z = blockdiag(M, M)^-1 A x from the mass-preconditioned handle, sampled
    rows of M (B A x) equal the oracle's rows of P z for the full and both half
    operators; B_int A x + B_ext A x = B_full A x at every row; the full
    Calderon solve needs fewer iterations than the mass-preconditioned one and
    reaches the same Delta G."""
    m, ch = sphere32
    nv = m.n_vertices
    form = pbm.PB_PMCHWT_INT
    rng = np.random.default_rng(53)
    x = rng.standard_normal(2 * nv)
    rows = np.sort(rng.choice(nv, 6, replace=False))
    Mr = oracle.mass_rows(m, rows)
    base = dict(operator_mode=pbm.PB_ASSEMBLED)
    with pbm.MeshHandle(m.xyz, m.tri, _opts(form, pbm.PB_FP32, preconditioner=pbm.PB_MASS, **base)) as h:
        z = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_PRECOND)
        rm = pbm.pb_mesh_solve(h, ch.xyz, ch.q)
    out = {}
    for prec, part in ((pbm.PB_CALDERON, "full"), (pbm.PB_CALDERON_INT, "int"), (pbm.PB_CALDERON_EXT, "ext")):
        with pbm.MeshHandle(m.xyz, m.tri, _opts(form, pbm.PB_FP32, preconditioner=prec, **base)) as h:
            out[part] = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_PRECOND)
            if part == "full":
                rc = pbm.pb_mesh_solve(h, ch.xyz, ch.q)
        r1, r2 = oracle.calderon_rows(m, 4.0, 80.0, 0.125, oracle.PMCHWT_INT, part, rows, z)
        got = np.concatenate([Mr @ out[part][:nv], Mr @ out[part][nv:]])
        print(f"calderon full size {part}: rel {_rel(got, np.concatenate([r1, r2])):.2e}")
        assert _rel(got, np.concatenate([r1, r2])) < 2e-6, part
    assert _rel(out["int"] + out["ext"], out["full"]) < 1e-6
    print(f"calderon full size iterations: mass {rm['iterations']} calderon {rc['iterations']}")
    assert rc["status"] == pbm.PB_OK and rc["iterations"] < rm["iterations"]
    assert abs(rc["dG"] - rm["dG"]) < 1e-4 * abs(rm["dG"])


@pytest.fixture(scope="module")
def fast_operators(meshes):
    """Fast Calderon's P on the star: V, K, D, T of both kernels with the
    one-point rule on far pairs and Sauter-Schwab order 3 on near pairs."""
    m = meshes["star7"]
    oL = oracle.assemble(m, 0.0, ("V", "K", "D"), oracle.FAST_NSS, centroid=True)
    oY = oracle.assemble(m, 0.125, ("V", "K", "D"), oracle.FAST_NSS, centroid=True)
    for o in (oL, oY):
        o["T"] = o["K"].T.copy()
    return oL, oY, oracle.mass(m)


@pytest.mark.parametrize("prec,name", [(pbm.PB_CALDERON, "calderon"), (pbm.PB_SCALED_CALDERON_INT,
                                                                        "scaled_calderon_int"),
                                       (pbm.PB_CALDERON_EXT, "calderon_ext")])
@pytest.mark.parametrize("form", [pbm.PB_PMCHWT_INT, pbm.PB_PMCHWT_EXT])
def test_fast_calderon_product(meshes, base_operators, fast_operators, form, prec, name):
    """Fast Calderon (one-point rule far field evaluated in FP32, Sauter-Schwab
    order 3): B A x against the oracle's relaxed P on the 980-triangle star,
    for FP64 matrix-free and FP32 assembled handles (the relaxed P is the same
    in both): within the FP32 evaluation of P's far field (2e-6)."""
    m = meshes["star7"]
    A = _system(base_operators, form)
    B = _calderon_ref(m, fast_operators, form, name)
    x = np.random.default_rng(97 + prec).standard_normal(2 * m.n_vertices)
    ref = B(A @ x)
    for p, mode in ((pbm.PB_FP64, pbm.PB_MATRIX_FREE), (pbm.PB_FP32, pbm.PB_ASSEMBLED)):
        with pbm.MeshHandle(m.xyz, m.tri, _opts(form, p, operator_mode=mode, preconditioner=prec,
                                                calderon_fast=1)) as h:
            yp = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_PRECOND)
        print(f"fast calderon product form {form} {name} prec {p}: rel {_rel(yp, ref):.2e}")
        assert _rel(yp, ref) < 2e-6, (p, mode, _rel(yp, ref))


@pytest.mark.parametrize("prec,name", [(pbm.PB_CALDERON, "calderon"), (pbm.PB_SCALED_CALDERON_INT,
                                                                        "scaled_calderon_int")])
@pytest.mark.parametrize("form", [pbm.PB_PMCHWT_INT, pbm.PB_PMCHWT_EXT])
def test_fast_calderon_solve_parity(form, prec, name):
    """Kirkwood sphere, fast Calderon (the paper's Cases 20b and 23b): the
    oracle's iterations, Delta G within 1e-5 (the preconditioner differs from
    the oracle's by its FP32 far field, the solution does not), the oracle's
    traces at tolerance 1e-11 to within the conditioning of B A times that
    tolerance (1e-7; 1.4e-8 measured)."""
    m, ch = inputs.config_kirkwood(4, 2.0)
    ref = oracle.solve(m, ch, formulation=form, preconditioner=name, fast=True)
    got = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, preconditioner=prec, calderon_fast=1))
    assert got["status"] == pbm.PB_OK
    assert got["iterations"] == ref["iterations"], (got["iterations"], ref["iterations"])
    assert abs(got["dG"] - ref["dG"]) < 1e-5 * abs(ref["dG"])
    tight = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, preconditioner=prec, calderon_fast=1, tol=1e-11))
    reft = oracle.solve(m, ch, formulation=form, preconditioner=name, tol=1e-11, A=ref["A"], fast=True)
    u = np.concatenate([tight["phi"], tight["dphi"]])
    assert _rel(u, np.concatenate([reft["phi"], reft["dphi"]])) < 1e-7
    with pytest.raises(pbm.PbError):
        pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, preconditioner=pbm.PB_MASS, calderon_fast=1))


def test_fast_calderon_full_size(sphere32):
    """20480-triangle sphere, internal PMCHWT, FP32 assembled, fast full and
    scaled-interior Calderon: sampled rows of M (B A x) against the oracle's
    relaxed P applied to z = blockdiag(M, M)^-1 A x; the solves reach the mass
    preconditioner's Delta G with at most two iterations more than the
    accurately integrated Calderon preconditioner."""
    m, ch = sphere32
    nv = m.n_vertices
    form = pbm.PB_PMCHWT_INT
    rng = np.random.default_rng(59)
    x = rng.standard_normal(2 * nv)
    rows = np.sort(rng.choice(nv, 6, replace=False))
    Mr = oracle.mass_rows(m, rows)
    base = dict(operator_mode=pbm.PB_ASSEMBLED)
    with pbm.MeshHandle(m.xyz, m.tri, _opts(form, pbm.PB_FP32, preconditioner=pbm.PB_MASS, **base)) as h:
        z = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_PRECOND)
        rm = pbm.pb_mesh_solve(h, ch.xyz, ch.q)
    for prec, part in ((pbm.PB_CALDERON, "full"), (pbm.PB_SCALED_CALDERON_INT, "int")):
        with pbm.MeshHandle(m.xyz, m.tri, _opts(form, pbm.PB_FP32, preconditioner=prec, calderon_fast=1,
                                                **base)) as h:
            yp = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_PRECOND)
            rf = pbm.pb_mesh_solve(h, ch.xyz, ch.q)
        ra = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, pbm.PB_FP32, preconditioner=prec, **base))
        a, b = (1.0, 1.0) if part == "full" else oracle.calderon_scales(4.0, 80.0, oracle.PMCHWT_INT, "int")
        r1, r2 = oracle.calderon_rows(m, 4.0, 80.0, 0.125, oracle.PMCHWT_INT, part, rows, z, fast=True)
        got = np.concatenate([a * (Mr @ yp[:nv]), b * (Mr @ yp[nv:])])
        print(f"fast calderon full size {part}: rel {_rel(got, np.concatenate([r1, r2])):.2e} "
              f"iterations fast {rf['iterations']} accurate {ra['iterations']} mass {rm['iterations']}")
        assert _rel(got, np.concatenate([r1, r2])) < 2e-6, part
        assert rf["status"] == pbm.PB_OK and ra["iterations"] <= rf["iterations"] <= ra["iterations"] + 2
        assert abs(rf["dG"] - rm["dG"]) < 1e-4 * abs(rm["dG"])


# ------------------------------------------------------- treecode far field
@pytest.fixture(scope="module")
def sphere16():
    return inputs.icosphere(16, 10.0)


@pytest.mark.parametrize("form", [pbm.PB_DIRECT_INT, pbm.PB_JUFFER, pbm.PB_MULLER_INT, pbm.PB_PMCHWT_INT])
def test_treecode_without_separated_clusters_is_direct(meshes, sphere16, form):
    """With a separation ratio so small that no cluster qualifies, every pair
    is summed directly: the treecode product equals the direct matrix-free
    one to FP64 rounding (same sums, other order) and to FP32 rounding."""
    for m in (meshes["star7"], sphere16):
        x = np.random.default_rng(7).standard_normal(2 * m.n_vertices)
        for p, tol in ((pbm.PB_FP64, 1e-13), (pbm.PB_FP32, 2e-7)):
            with pbm.MeshHandle(m.xyz, m.tri, _opts(form, p)) as h:
                ref = pbm.pb_mesh_apply(h, x)
            with pbm.MeshHandle(m.xyz, m.tri, _opts(form, p, operator_mode=pbm.PB_TREECODE, tree_theta=0.01)) as h:
                y = pbm.pb_mesh_apply(h, x)
            assert _rel(y, ref) < tol, (form, p, _rel(y, ref))


@pytest.mark.parametrize("form", [pbm.PB_DIRECT_INT, pbm.PB_JUFFER, pbm.PB_LU, pbm.PB_PMCHWT_EXT])
def test_treecode_converges_with_degree(sphere16, form):
    """5120-triangle sphere: the treecode's error against the exact product
    (the FP64 direct matrix-free product, itself equal to the oracle's to
    1e-12) falls geometrically with the interpolation degree, by at least 5x
    per degree, and is below 1e-6 at degree 5 with theta 0.5."""
    m = sphere16
    x = np.random.default_rng(11).standard_normal(2 * m.n_vertices)
    with pbm.MeshHandle(m.xyz, m.tri, _opts(form)) as h:
        ref = pbm.pb_mesh_apply(h, x)
    errs = []
    for deg in (2, 3, 4, 5, 6, 7):
        with pbm.MeshHandle(m.xyz, m.tri, _opts(form, operator_mode=pbm.PB_TREECODE, tree_degree=deg,
                                                tree_theta=0.5)) as h:
            errs.append(_rel(pbm.pb_mesh_apply(h, x), ref))
    print(f"treecode form {form}: errors by degree 2..7 {['%.1e' % e for e in errs]}")
    assert all(errs[k + 1] < errs[k] / 5.0 for k in range(len(errs) - 1)), errs
    assert errs[3] < 1e-6 and errs[-1] < 1e-9


# Accuracy target of the treecode at its defaults (degree 6, theta 0.7): a
# relative operator error of at most 5e-6 (the _rel measure), below the FP32
# direct far field's own bound (2e-5), so that the treecode leaves the reduced
# precision Delta G contract (1e-4) a margin of 10 over the FP32 rounding.
TREE_TARGET = 5e-6


def test_treecode_full_size_rows_and_solve(sphere32):
    """20480-triangle sphere, FP32 treecode at its defaults: the whole product
    of the direct, Juffer and internal PMCHWT systems within the accuracy
    target of the FP64 direct matrix-free product, sampled rows of the Juffer
    and PMCHWT products within it of the oracle's rows; the Juffer solve
    (scaled mass) and the direct one reach the FP64 direct matrix-free Delta G
    within 1e-5 with the same iterations."""
    m, ch = sphere32
    nv = m.n_vertices
    rng = np.random.default_rng(61)
    x = rng.standard_normal(2 * nv)
    rows = np.sort(rng.choice(nv, 6, replace=False))
    for form in (oracle.DIRECT, oracle.JUFFER, oracle.PMCHWT_INT):
        with pbm.MeshHandle(m.xyz, m.tri, _opts(form, pbm.PB_FP32, operator_mode=pbm.PB_TREECODE)) as h:
            y = pbm.pb_mesh_apply(h, x)
        with pbm.MeshHandle(m.xyz, m.tri, _opts(form)) as h:
            yd = pbm.pb_mesh_apply(h, x)
        print(f"treecode full size form {form}: product rel {_rel(y, yd):.2e}")
        assert _rel(y, yd) < TREE_TARGET, (form, _rel(y, yd))
        if form == oracle.DIRECT:
            continue
        r1, r2 = oracle.system_rows(m, 4.0, 80.0, 0.125, form, rows, x)
        got = np.concatenate([y[rows], y[nv + rows]])
        assert _rel(got, np.concatenate([r1, r2])) < TREE_TARGET
    for form, prec in ((pbm.PB_JUFFER, pbm.PB_SCALED_MASS), (pbm.PB_DIRECT_INT, pbm.PB_BLOCK_DIAG)):
        ref = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, preconditioner=prec))
        got = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, _opts(form, pbm.PB_FP32, preconditioner=prec,
                                                              operator_mode=pbm.PB_TREECODE))
        assert got["status"] == pbm.PB_OK and abs(got["iterations"] - ref["iterations"]) <= 1
        assert abs(got["dG"] - ref["dG"]) < 1e-5 * abs(ref["dG"]), (form, got["dG"], ref["dG"])


@pytest.mark.parametrize("prec", [pbm.PB_CALDERON_EXT, pbm.PB_SCALED_CALDERON_INT])
def test_treecode_calderon(sphere16, prec):
    """Calderon preconditioners on the treecode far field (P's far field through
    the same tree, the Yukawa-only kernels for the exterior part): B A x within
    1e-6 of the direct matrix-free chain; the captured solve equals the eager one."""
    m = sphere16
    x = np.random.default_rng(13).standard_normal(2 * m.n_vertices)
    with pbm.MeshHandle(m.xyz, m.tri, _opts(pbm.PB_PMCHWT_INT, preconditioner=prec)) as h:
        ref = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_PRECOND)
    ot = _opts(pbm.PB_PMCHWT_INT, preconditioner=prec, operator_mode=pbm.PB_TREECODE)
    with pbm.MeshHandle(m.xyz, m.tri, ot) as h:
        y = pbm.pb_mesh_apply(h, x, pbm.PB_APPLY_PRECOND)
    assert _rel(y, ref) < 1e-6, _rel(y, ref)
    ch = inputs.charges_ball(5, 20, 8.0)
    rg = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, ot)
    ot.use_graph = 0
    re = pbm.pb_solve(m.xyz, m.tri, ch.xyz, ch.q, ot)
    assert rg["status"] == pbm.PB_OK and rg["iterations"] == re["iterations"]
    assert abs(rg["dG"] - re["dG"]) <= 1e-12 * abs(re["dG"])
