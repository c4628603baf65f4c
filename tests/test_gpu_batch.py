"""GPU checks of pb_solve_batch: requests of uneven size on different meshes
solved together, their far fields fused into one persistent launch per kernel
form and GMRES iteration.

Each request's arithmetic is that of its own pb_mesh_solve (same source split,
same per-lane sums, same Krylov kernels and host Givens code), so results are
compared bit for bit with single solves; one FP64 request is also checked
against the oracle (Delta G within 1e-6, as for single solves)."""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

pbm = pytest.importorskip("paper_2108_10481_amd")


def _requests():
    """(mesh, charges, formulation, preconditioner): four sizes (320 to 2000
    triangles, ragged against the 64-triangle wavefronts), four kernel forms'
    worth of formulations, three preconditioners."""
    star, shape = inputs.star_surface(5, 7, 6.0)                      # T = 980
    return [
        (inputs.icosphere(4, 2.0), inputs.charges_ball(1, 1, 0.5), pbm.PB_DIRECT_INT, pbm.PB_BLOCK_DIAG),
        (star, inputs.charges_in_star(6, 9, shape), pbm.PB_JUFFER, pbm.PB_SCALED_MASS),
        (inputs.icosphere(6, 2.0), inputs.charges_ball(2, 5, 1.0), pbm.PB_PMCHWT_INT, pbm.PB_MASS),
        (inputs.icosphere(10, 5.0), inputs.charges_ball(3, 7, 3.0), pbm.PB_DIRECT_EXT, pbm.PB_BLOCK_DIAG),
    ]


def _handles(reqs, precision, mode=None, use_graph=1, far_symmetric=0, kappas=None):
    """kappas: one screening constant per request (default: the paper's 0.125)."""
    mode = pbm.PB_MATRIX_FREE if mode is None else mode
    kappas = kappas or [0.125] * len(reqs)
    return [pbm.MeshHandle(m.xyz, m.tri, pbm.pb_default_options(formulation=f, preconditioner=p,
                                                                precision=precision, operator_mode=mode,
                                                                use_graph=use_graph, far_symmetric=far_symmetric,
                                                                kappa=k))
            for (m, _, f, p), k in zip(reqs, kappas)]


def _same(a, b):
    assert a["status"] == b["status"] and a["iterations"] == b["iterations"]
    assert a["dG"] == b["dG"] and a["rel_residual"] == b["rel_residual"]
    assert np.array_equal(a["phi"], b["phi"]) and np.array_equal(a["dphi"], b["dphi"])


@pytest.mark.parametrize("precision,sym,unscreened", [(pbm.PB_FP64, 0, False), (pbm.PB_FP32, 0, False),
                                                      (pbm.PB_FP32, 1, False), (pbm.PB_FP32, 1, True)])
def test_batch_equals_single_solves(precision, sym, unscreened):
    """sym = 1: every request's far field evaluated once per unordered
    triangle pair (far_symmetric 1) in its single solve and in the batch;
    unscreened: two of the requests have kappa = 0, so the batch runs the
    screened and the unscreened symmetric kernels side by side."""
    reqs = _requests()
    hs = _handles(reqs, precision, far_symmetric=sym, kappas=[0.0, 0.125, 0.125, 0.0] if unscreened else None)
    try:
        single = [pbm.pb_mesh_solve(h, c.xyz, c.q) for h, (_, c, _, _) in zip(hs, reqs)]
        batch = pbm.pb_solve_batch(hs, [(c.xyz, c.q) for _, c, _, _ in reqs])
        for a, b in zip(batch, single):
            _same(a, b)
            assert a["status"] == pbm.PB_OK and a["iterations"] > 0
        # another order and a subset: each request's result does not depend on its co-tenants
        order = [3, 1, 0]
        again = pbm.pb_solve_batch([hs[k] for k in order], [(reqs[k][1].xyz, reqs[k][1].q) for k in order])
        for k, a in zip(order, again):
            _same(a, single[k])
    finally:
        for h in hs:
            h.close()
    if precision == pbm.PB_FP64:
        m, c, f, _ = reqs[0]
        ref = oracle.solve(m, c, formulation=oracle.DIRECT)
        assert abs(batch[0]["dG"] - ref["dG"]) < 1e-6 * abs(ref["dG"])
        assert batch[0]["iterations"] == ref["iterations"]


def test_batch_repeated_calls_reuse_graph():
    """The captured batch graph is kept for the next call with the same
    requests: repeated calls, calls on other subsets in between, and a batch
    after a handle was closed and another created (possibly at the same
    addresses, with another formulation) all give bitwise the single solves."""
    reqs = _requests()
    hs = _handles(reqs, pbm.PB_FP32)
    extra = []
    try:
        sets = [(c.xyz, c.q) for _, c, _, _ in reqs]
        single = [pbm.pb_mesh_solve(h, *st) for h, st in zip(hs, sets)]
        for _ in range(2):
            for a, b in zip(pbm.pb_solve_batch(hs, sets), single):
                _same(a, b)
        sub = [2, 0]
        for k, a in zip(sub, pbm.pb_solve_batch([hs[k] for k in sub], [sets[k] for k in sub])):
            _same(a, single[k])
        for a, b in zip(pbm.pb_solve_batch(hs, sets), single):
            _same(a, b)
        # the same charges on other charge values: a new right-hand side, same graph
        q2 = [(x, 0.5 * q) for x, q in sets]
        single2 = [pbm.pb_mesh_solve(h, *st) for h, st in zip(hs, q2)]
        for a, b in zip(pbm.pb_solve_batch(hs, q2), single2):
            _same(a, b)
        hs[1].close()
        m1, c1 = reqs[1][0], reqs[1][1]
        extra.append(pbm.MeshHandle(m1.xyz, m1.tri, pbm.pb_default_options(
            formulation=pbm.PB_DIRECT_INT, precision=pbm.PB_FP32, operator_mode=pbm.PB_MATRIX_FREE)))
        hs2 = [hs[0], extra[0], hs[2], hs[3]]
        single3 = [pbm.pb_mesh_solve(h, *st) for h, st in zip(hs2, sets)]
        for a, b in zip(pbm.pb_solve_batch(hs2, sets), single3):
            _same(a, b)
    finally:
        for h in hs + extra:
            h.close()


def test_batch_eager_lockstep_equals_single_solves():
    """With use_graph = 0 the lockstep runs eagerly (host Givens, one
    synchronisation per iteration): still bitwise the single solves."""
    reqs = _requests()
    hs = _handles(reqs, pbm.PB_FP32, use_graph=0)
    try:
        single = [pbm.pb_mesh_solve(h, c.xyz, c.q) for h, (_, c, _, _) in zip(hs, reqs)]
        batch = pbm.pb_solve_batch(hs, [(c.xyz, c.q) for _, c, _, _ in reqs])
        for a, b in zip(batch, single):
            _same(a, b)
    finally:
        for h in hs:
            h.close()


def test_batch_degenerate_requests():
    """A batch of one equals the single solve; a request with zero charge
    (right-hand side 0) takes no iteration and returns u = 0 beside others."""
    reqs = _requests()[:2]
    hs = _handles(reqs, pbm.PB_FP32)
    try:
        m0, c0 = reqs[0][0], reqs[0][1]
        one = pbm.pb_solve_batch(hs[:1], [(c0.xyz, c0.q)])
        _same(one[0], pbm.pb_mesh_solve(hs[0], c0.xyz, c0.q))
        zero = np.zeros_like(c0.q)
        c1 = reqs[1][1]
        out = pbm.pb_solve_batch(hs, [(c0.xyz, zero), (c1.xyz, c1.q)])
        assert out[0]["iterations"] == 0 and out[0]["dG"] == 0.0
        assert not np.any(out[0]["phi"]) and not np.any(out[0]["dphi"])
        _same(out[1], pbm.pb_mesh_solve(hs[1], c1.xyz, c1.q))
    finally:
        for h in hs:
            h.close()


def test_batch_refusals():
    reqs = _requests()[:2]
    sets = [(c.xyz, c.q) for _, c, _, _ in reqs]
    mf = _handles(reqs, pbm.PB_FP32)
    other = _handles(reqs, pbm.PB_FP64)
    dense = _handles(reqs, pbm.PB_FP32, pbm.PB_ASSEMBLED)
    tree = _handles(reqs, pbm.PB_FP32, pbm.PB_TREECODE)
    try:
        for hs, code in (([mf[0], other[1]], pbm.PB_E_STATE), ([mf[0], dense[1]], pbm.PB_E_STATE),
                         ([tree[0], mf[1]], pbm.PB_E_STATE), ([mf[0], mf[0]], pbm.PB_E_INVALID_ARG)):
            with pytest.raises(pbm.PbError) as e:
                pbm.pb_solve_batch(hs, sets)
            assert e.value.code == code
        # a charge outside one request's surface fails the call and names the request
        far = np.array([[100.0, 0.0, 0.0]])
        with pytest.raises(pbm.PbError) as e:
            pbm.pb_solve_batch(mf, [sets[0], (far, np.ones(1))])
        assert e.value.code == pbm.PB_E_CHARGES and "request 1" in pbm.pb_last_error()
        # the refused calls left the handles usable
        _same(pbm.pb_solve_batch(mf, sets)[1], pbm.pb_mesh_solve(mf[1], *sets[1]))
    finally:
        for h in mf + other + dense + tree:
            h.close()


def test_batch_full_size_mix():
    """The bench's mix at full size: the 20480-triangle sphere beside serving-
    trace star surfaces of 1280 to 20480 triangles, FP32 matrix-free, direct and
    Juffer; bitwise equal to single solves."""
    trace = inputs.serving_trace(seed=5, n_requests=6, fmax=32)
    items = [inputs.build_request(r) + (r["formulation"],) for r in trace]
    m, ch = inputs.config_sphere()
    items.append((m, ch, pbm.PB_JUFFER))
    hs = [pbm.MeshHandle(mm.xyz, mm.tri, pbm.pb_default_options(formulation=f, precision=pbm.PB_FP32,
                                                                 operator_mode=pbm.PB_MATRIX_FREE))
          for mm, _, f in items]
    try:
        batch = pbm.pb_solve_batch(hs, [(c.xyz, c.q) for _, c, _ in items])
        for h, (_, c, _), a in zip(hs, items, batch):
            _same(a, pbm.pb_mesh_solve(h, c.xyz, c.q))
    finally:
        for h in hs:
            h.close()
