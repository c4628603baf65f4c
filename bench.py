#!/usr/bin/env python3
"""Benchmark: complete boundary-element Poisson-Boltzmann solves on one MI355X.

Default workload (the configuration the headline metric is quoted on):
protein-shaped star surface r = 18 A (1 + 0.15 f), f a random sum of real
spherical harmonics of degree <= 6 (seed 3), frequency-64 icosphere mapping
(81920 flat triangles, 40962 vertices), 2000 charges N(0, 0.4) e inside
0.8 r, eps_in 4, eps_out 80, kappa 0.125 / A, matrix-free FP32 far field with
the FP64 Sauter-Schwab near field, block-diagonal preconditioner, GMRES
tolerance 1e-5 without restart.

Step k = one complete solve with the internal direct formulation (k even)
or the Juffer formulation (k odd), covering every stage of the hot path:
geometry, near field, mass terms, preconditioner, right-hand side, GMRES with
the far-field operator, reaction potential and Delta G.  The mesh's host-side
index plan (validation, Morton order, sparsity) is built once before timing
(its cost is reported as the cold solve); every device stage is redone in
every step.  value = operator-product kernel pairs per second over the timed
solves; solves/s, p50 / p99 latency, the far-field kernel's roofline, the
first requests of the serving trace (served vs serial plain FP64) and the
oracle's CPU rate are reported beside it.  --workload sphere runs the
20480-triangle sphere the same way; the other workloads are listed in parse().

Prints one JSON line (rank 0; there is only one GPU).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import inputs  # noqa: E402

METRIC = ("operator matvec kernel-pairs/s; solves/s + p99 latency at ΔG rel err ≤1e-4")
# algorithmic flops per kernel pair of the fused far-field formula (FMA = 2,
# exp and rsqrt = 1 each), counted from the kernel formula
FLOPS_PER_PAIR = {0: 28, 1: 38}
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}   # MI355X published vector peaks
# far-field assembly, per ordered far point pair (the recorded work), counted
# from the assembly formula: each unordered point pair is evaluated once and
# yields six values (the four of the (t, s) block and the two non-symmetric
# ones of (s, t)): kernel values direct 25.7 flops / 22 lane operations,
# Juffer 32.5 / 26.5, plus the basis contraction in the two-orbit form of the
# 6-point rule (4.33 flops / 3 lane operations per value); halved per ordered pair
ASM_FLOPS_PER_PP = {0: 25.83, 1: 29.25}
# VALU issue: a SIMD issues one wave64 VALU instruction per 4 cycles, so the
# device's issue capacity is 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane
# instructions per second.  The rocprofv3 counters show the far-field kernels'
# transcendentals (v_rsq_f32, v_exp_f32) overlapping the other VALU work there
# (SQ_ACTIVE_INST_VALU, which counts each of them as two quad-cycles, exceeds
# the kernel's SIMD cycles), so the issue fraction charges the executed
# non-transcendental instructions and the transcendentals are reported beside
# it against the measured v_exp_f32 rate.  Executed non-transcendental VALU
# lane instructions per ordered kernel pair, from SQ_INSTS_VALU -
# SQ_INSTS_VALU_TRANS_F32 (profiles/k_far_star81920_trace_and_counters.md,
# profiles/sphere20480_fp32_assembled_trace_and_traffic.md):
ISSUE_PEAK = 256 * 4 * 16 * 2.4e9
FAR_VALU_PER_PAIR = {0: 11.79, 1: 16.70}   # k_far_sym<FORM>, one transcendental per pair
FAR_TRANS_PER_PAIR = 1.0
ASM_VALU_PER_PP = {0: 22.50, 1: 25.76}     # far-field assembly, one transcendental per pair
ASM_TRANS_PER_PP = 1.0


def valu_issue(pairs_by_form, valu_per_pair, trans_per_pair, seconds, peaks):
    """Issue fraction of executed non-transcendental VALU lane instructions and
    the transcendental rate against the measured v_exp_f32 rate."""
    if seconds <= 0:
        return None
    lane = sum(w * valu_per_pair[f] for f, w in pairs_by_form.items()) / seconds
    trans = sum(w * trans_per_pair for w in pairs_by_form.values()) / seconds
    out = {"lane_instr_per_s": round(lane, 1), "peak_lane_instr_per_s": ISSUE_PEAK,
           "frac": round(lane / ISSUE_PEAK, 4), "transcendentals_per_s": round(trans, 1)}
    if peaks:
        out["trans_frac_of_measured_exp_rate"] = round(trans / peaks["exp32_lane_ops_per_s"], 4)
        out["fma_microbenchmark_lane_instr_per_s"] = peaks["fma32_lane_ops_per_s"]
        out["source"] = "profiles/peaks.json"
    return out


def measured_traffic(workload_key: str, kernel: str = "assembly"):
    """HBM bytes per launch of the dominant kernel from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs summarised in profiles/traffic.json, scaled by the copy-kernel
    calibration stored there; None when the kernel's source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        t = json.load(open(path))
        if kernel != "assembly":
            t = t["kernels"][kernel]
        src = open(os.path.join(ROOT, t["source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    if t.get("workload") != workload_key or hashlib.sha256(src).hexdigest() != t.get("source_sha256"):
        return None
    return t


def measured_peaks():
    """Peaks measured on gfx950 by ``bench.py --measure-peaks`` (profiles/peaks.json):
    FP32 FMA lane instructions/s, the issue cost of v_exp_f32 / v_rsq_f32 in
    FMA slots, FP64 FMA/s, BF16 MFMA flop/s, HBM read and copy bytes/s."""
    try:
        return json.load(open(os.path.join(ROOT, "profiles", "peaks.json")))
    except (OSError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "mixed-bf16", "mixed-fp16"])
    ap.add_argument("--operator-mode", default=None, choices=["matrix-free", "assembled", "auto"],
                    help="default: matrix-free for the star workload, auto for the sphere")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=24, help="oracle rows per formulation in the CPU sample")
    ap.add_argument("--workload", default="star",
                    choices=["star", "sphere", "multi", "serving", "calderon", "large", "batch"])
    ap.add_argument("--serving-requests", type=int, default=48,
                    help="requests of the serving trace replayed after the timed steps (0: none)")
    ap.add_argument("--no-reference", action="store_true",
                    help="skip the FP64 reference solves of the accuracy gate")
    ap.add_argument("--far-symmetric", type=int, default=0, choices=[0, 1, -1],
                    help="FP32 matrix-free far field: 0 automatic (the library default), 1 the symmetric "
                         "kernel at every size, -1 the per-ordered-pair kernel")
    ap.add_argument("--preconditioner", default="block-diag", choices=["block-diag", "scaled-mass"],
                    help="scaled-mass: the Juffer solves use blockdiag(aM, bM)^-1 (the paper's Case 10), "
                         "the direct ones keep the block-diagonal preconditioner (Case 2)")
    return ap.parse_known_args()[0]


def _pct(values, q):
    v = sorted(values)
    return v[min(len(v) - 1, max(0, int(math.ceil(q * len(v))) - 1))]


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library runs on one GPU; it has no multi-GPU path, so only --gpus 1 "
              "is measured", file=sys.stderr)
        sys.exit(2)
    import paper_2108_10481_amd as pbm
    if pbm.pb_device_count() < 1:
        print("bench.py: no GPU visible to the HIP library", file=sys.stderr)
        sys.exit(1)

    prec = {"fp64": pbm.PB_FP64, "fp32": pbm.PB_FP32, "mixed-bf16": pbm.PB_MIXED_BF16,
            "mixed-fp16": pbm.PB_MIXED_FP16}[a.precision]
    mode_name = a.operator_mode or ("matrix-free" if a.workload == "star" else "auto")
    mode = {"matrix-free": pbm.PB_MATRIX_FREE, "assembled": pbm.PB_ASSEMBLED, "auto": pbm.PB_AUTO}[mode_name]
    if a.workload == "star":
        mesh, ch = inputs.config_star()
        workload = ("star surface R=18 A (1 + 0.15 sum Y_lm, l<=6, seed 3), 81920 triangles / 40962 vertices, "
                    "2000 charges N(0,0.4) e inside 0.8 r (seed 1003), eps 4/80, kappa 0.125, GMRES tol 1e-5; "
                    "step k = one complete solve (every device stage redone) with the direct formulation "
                    "(k even) or the Juffer formulation (k odd)")
        key = "star81920"
    else:
        mesh, ch = inputs.config_sphere()
        workload = ("sphere R=10 A, icosphere 20480 triangles / 10242 vertices, 50 charges U[-1,1] e in r<8 A "
                    "(seed 2), eps 4/80, kappa 0.125, GMRES tol 1e-5; step k = one complete solve (every "
                    "device stage redone) with the direct (k even) or the Juffer (k odd) formulation")
        key = "sphere20480"
    T = mesh.n_triangles
    P = 6 * T
    forms = (pbm.PB_DIRECT_INT, pbm.PB_JUFFER)
    print(f"bench: {key}, {a.precision} {mode_name}", file=sys.stderr, flush=True)

    precs = {f: pbm.PB_SCALED_MASS if (a.preconditioner == "scaled-mass" and f == pbm.PB_JUFFER)
             else pbm.PB_BLOCK_DIAG for f in forms}
    opts = {f: pbm.pb_default_options(formulation=f, precision=prec, operator_mode=mode, preconditioner=precs[f],
                                      far_symmetric=a.far_symmetric)
            for f in forms}
    # cold solve: handle creation (validation, Morton order, near-pair lists and
    # every device stage) plus the first solve, from host arrays
    handles, cold = {}, {}
    for f in forms:
        t0 = time.perf_counter()
        handles[f] = pbm.MeshHandle(mesh.xyz, mesh.tri, opts[f])
        t1 = time.perf_counter()
        pbm.pb_mesh_solve(handles[f], ch.xyz, ch.q)
        t2 = time.perf_counter()
        cold[f] = {"t_create_ms": round(1e3 * (t1 - t0), 1), "cold_solve_ms": round(1e3 * (t2 - t0), 1)}
    print("bench: handles created", file=sys.stderr, flush=True)

    # FP64 reference (the plain method's precision) for the accuracy gate, outside the timed region
    ref = {}
    if not a.no_reference:
        for f in forms:
            ref[f] = pbm.pb_solve(mesh.xyz, mesh.tri, ch.xyz, ch.q,
                                  pbm.pb_default_options(formulation=f, precision=pbm.PB_FP64,
                                                         operator_mode=pbm.PB_MATRIX_FREE, preconditioner=precs[f]))
        print("bench: FP64 reference solves done", file=sys.stderr, flush=True)

    lat = {f: [] for f in forms}
    res = {f: [] for f in forms}

    def step(k):
        f = forms[k % len(forms)]
        s0 = time.perf_counter()
        h = handles[f]
        pbm.pb_mesh_refresh(h)
        r = pbm.pb_mesh_solve(h, ch.xyz, ch.q)
        lat[f].append(time.perf_counter() - s0)
        res[f].append(r)

    for k in range(a.warmup):
        step(k)
    assembled = any(h.info()["assembled"] for h in handles.values())
    # the far-field product kernel (matrix-free) or the assembly (assembled), HIP events on its stream
    for h in handles.values():
        pbm.pb_mesh_profile(h, 2 if assembled else 1)
    for f in forms:
        lat[f].clear()
        res[f].clear()
    print("bench: timed steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for k in range(a.steps):
        step(k)
    for h in handles.values():
        pbm.pb_mesh_synchronize(h)
    elapsed = time.perf_counter() - t0
    print(f"bench: timed steps done, {elapsed:.1f} s", file=sys.stderr, flush=True)
    done = [f for f in forms if res[f]]
    phases_ms = {str(f): {k: round(1e3 * float(np.median([r[k] for r in res[f]])), 3)
                          for k in ("t_setup", "t_rhs", "t_prec", "t_gmres", "t_dG")} for f in done}
    for f in done:
        phases_ms[str(f)].update(cold[f])
    prof = {f: pbm.pb_mesh_profile_read(handles[f], 0) for f in forms}
    prof_asm = {f: pbm.pb_mesh_profile_read(handles[f], 1) for f in forms}
    info = {f: handles[f].info() for f in forms}
    dtype = "f64" if prec == pbm.PB_FP64 else "f32"
    peaks = measured_peaks()
    launches = sum(prof[f][0] for f in forms)
    kern_ms = sum(prof[f][1] for f in forms)
    pairs_timed = 0.0
    if assembled:
        asm_ms = sum(prof_asm[f][1] for f in forms)
        evals = sum(prof_asm[f][2] for f in forms)
        flops = sum(prof_asm[f][2] * ASM_FLOPS_PER_PP[f] for f in forms)
        achieved = flops / (asm_ms * 1e-3) / 1e12 if asm_ms > 0 else 0.0
        nasm = sum(prof_asm[f][0] for f in forms)
        tr = measured_traffic(key) if dtype == "f32" else None
        traffic = None
        if tr and nasm > 0:
            traffic = round(sum(tr["assembly_bytes"][str(f)] * prof_asm[f][0] for f in forms) / nasm, 1)
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[dtype], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_TFLOPS[dtype], 4), "traffic": traffic,
                "kernel": "far-field assembly (k_fill x2, k_assemble_tile, k_sym_finish x4 per assembly)",
                "launches": nasm, "avg_launch_ms": round(asm_ms / max(nasm, 1), 4),
                "point_pair_evals_per_s": round(evals / (asm_ms * 1e-3), 1) if asm_ms > 0 else None}
        if dtype == "f32" and asm_ms > 0:
            roof["valu_issue"] = valu_issue({f: prof_asm[f][2] for f in forms}, ASM_VALU_PER_PP, ASM_TRANS_PER_PP,
                                            asm_ms * 1e-3, peaks)
        # products stream the matrix: each solve's products counted from iterations
        for f in done:
            pairs_timed += sum((r["iterations"] + 1) * float(P) * P for r in res[f])
    else:
        pairs_timed = sum(prof[f][2] for f in forms)
        flops = sum(prof[f][2] * FLOPS_PER_PAIR[f] for f in forms)
        achieved = flops / (kern_ms * 1e-3) / 1e12 if kern_ms > 0 else 0.0
        # the counters and traffic on record are those of the symmetric kernel
        sym = all(info[f]["far_symmetric"] for f in forms)
        tr = measured_traffic(key, kernel="k_far") if (dtype == "f32" and sym) else None
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[dtype], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_TFLOPS[dtype], 4),
                "traffic": (round(sum(tr["bytes_per_launch"][str(f)] * prof[f][0] for f in forms)
                                  / max(launches, 1), 1) if tr else None),
                "kernel": ("k_far_sym (matrix-free far field, every unordered pair once" if sym else
                           "k_far (matrix-free far field, every ordered pair") +
                          "; the finish and the near field excluded)",
                "launches": launches, "avg_launch_ms": round(kern_ms / max(launches, 1), 4),
                "kernel_pairs_per_s": round(pairs_timed / (kern_ms * 1e-3), 1) if kern_ms > 0 else None}
        if dtype == "f32" and sym and kern_ms > 0:
            roof["valu_issue"] = valu_issue({f: prof[f][2] for f in forms}, FAR_VALU_PER_PAIR, FAR_TRANS_PER_PAIR,
                                            kern_ms * 1e-3, peaks)
        by_form = {}
        for f in forms:
            n, ms, w = prof[f]
            if n == 0 or ms <= 0:
                continue
            e = {"launches": n, "avg_launch_ms": round(ms / n, 3), "kernel_pairs_per_s": round(w / (ms * 1e-3), 1),
                 "tflops": round(w * FLOPS_PER_PAIR[f] / (ms * 1e-3) / 1e12, 3)}
            if dtype == "f32" and sym:
                e["valu_issue_frac"] = round(w * FAR_VALU_PER_PAIR[f] / (ms * 1e-3) / ISSUE_PEAK, 4)
            by_form[str(f)] = e
        roof["by_formulation"] = by_form

    solves = sum(len(res[f]) for f in forms)
    all_lat = [1e3 * x for f in forms for x in lat[f]]
    last = {f: res[f][-1] for f in done}
    rel_err = (max(abs(last[f]["dG"] - ref[f]["dG"]) / abs(ref[f]["dG"]) for f in done) if ref else None)
    rec = {
        "metric": METRIC,
        "value": round(pairs_timed / elapsed, 1),
        "unit": "kernel-pairs/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(1e3 * elapsed / a.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": workload, "precision": a.precision,
                   "operator_mode": "assembled" if assembled else "matrix-free",
                   "source_chunks": info[forms[0]]["source_chunks"],
                   "far_symmetric": a.far_symmetric,
                   "preconditioner": {"direct": "block-diagonal",
                                      "juffer": "scaled mass" if a.preconditioner == "scaled-mass"
                                      else "block-diagonal"}},
        "value_definition": ("operator-product kernel pairs (P^2 = (6T)^2 target x source quadrature-point pairs "
                             "per product, near pairs included) of every product in the timed complete solves, "
                             "divided by the timed region's wall time"),
        "solves_per_s": round(solves / elapsed, 4),
        "p50_ms": round(_pct(all_lat, 0.5), 3),
        "p99_ms": round(_pct(all_lat, 0.99), 3),
        "latency_ms_by_formulation": {str(f): {"p50": round(_pct([1e3 * x for x in lat[f]], 0.5), 3),
                                               "max": round(1e3 * max(lat[f]), 3)} for f in done},
        "phases_ms": phases_ms,
        "dG_kcal": {str(f): last[f]["dG"] for f in done},
        "dG_rel_err_vs_fp64": rel_err,
        "iterations": {str(f): last[f]["iterations"] for f in done},
        "fp64_reference_solve_s": ({str(f): round(ref[f]["t_setup"] + ref[f]["t_rhs"] + ref[f]["t_prec"]
                                                  + ref[f]["t_gmres"] + ref[f]["t_dG"], 4) for f in forms}
                                   if ref else None),
        "roofline": roof,
    }
    if rel_err is not None and rel_err > 1e-4:
        rec["accuracy_gate"] = "FAILED"
    for h in handles.values():
        h.close()
    if a.serving_requests > 0:
        rec["serving"] = serving_prefix(a.serving_requests)
    if not a.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(mesh, rec["iterations"], a.cpu_rows, P, key)
    print(json.dumps(rec), flush=True)


def serving_prefix(nreq, rate=20.0, slots=8):
    """The first nreq requests of the serving trace (seed 5: Poisson arrivals at
    20 req/s, star surfaces of 1280-81920 triangles log-uniform, 50-4000
    charges, direct or Juffer), replayed twice with their arrival times: on the
    continuous-batching server in mixed BF16 (assembled 16-bit far field, FP64
    refinement), and one after another in FIFO order with the plain FP64 solve
    (pb_solve, FP64, assembled when it fits), each request starting at its
    arrival or when the previous one ends.  Both measured; every served
    Delta G is checked against the FP64 one."""
    import threading
    import paper_2108_10481_amd as pbm
    trace = inputs.serving_trace(5, nreq, rate)
    reqs = []
    for k, r in enumerate(trace):
        reqs.append((r,) + inputs.build_request(r))
        if k % 64 == 63:
            print(f"bench: serving {k + 1}/{nreq} requests built", file=sys.stderr, flush=True)
    print(f"bench: serving {nreq} requests built", file=sys.stderr, flush=True)
    opt_mixed = {f: pbm.pb_default_options(formulation=f, precision=pbm.PB_MIXED_BF16,
                                           operator_mode=pbm.PB_ASSEMBLED) for f in (0, 1)}
    opt_fp64 = {f: pbm.pb_default_options(formulation=f, precision=pbm.PB_FP64, operator_mode=pbm.PB_AUTO)
                for f in (0, 1)}
    served = [None] * len(reqs)
    with pbm.Server(max_slots=slots) as srv:
        r0, m0, c0 = reqs[0]
        srv.wait(srv.submit(m0.xyz, m0.tri, c0.xyz, c0.q, opt_mixed[r0["formulation"]]))   # warm-up
        tickets = [None] * len(reqs)
        base = time.perf_counter()

        def submitter():
            for k, (r, m, c) in enumerate(reqs):
                delay = base + r["arrival_s"] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                tickets[k] = srv.submit(m.xyz, m.tri, c.xyz, c.q, opt_mixed[r["formulation"]])
        th = threading.Thread(target=submitter)
        th.start()
        for k in range(len(reqs)):
            while tickets[k] is None:
                time.sleep(0.001)
            served[k] = srv.wait(tickets[k])
            if k % 64 == 63:
                print(f"bench: served {k + 1}/{len(reqs)}", file=sys.stderr, flush=True)
        th.join()
        stats = srv.stats()
    lat = [x["t_end"] - x["t_submit"] for x in served]
    span = max(x["t_end"] for x in served) - min(x["t_submit"] for x in served)
    print("bench: served run done", file=sys.stderr, flush=True)
    # serial plain FP64, FIFO on the same arrival times
    ser_lat, worst = [], 0.0
    base = time.perf_counter()
    for k, (r, m, c) in enumerate(reqs):
        delay = base + r["arrival_s"] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        g = pbm.pb_solve(m.xyz, m.tri, c.xyz, c.q, opt_fp64[r["formulation"]])
        ser_lat.append(time.perf_counter() - (base + r["arrival_s"]))
        worst = max(worst, abs(served[k]["dG"] - g["dG"]) / abs(g["dG"]))
        if k % 16 == 15:
            print(f"bench: serial FP64 {k + 1}/{len(reqs)}", file=sys.stderr, flush=True)
    ser_span = time.perf_counter() - (base + reqs[0][0]["arrival_s"])
    sizes = sorted(r["n_triangles"] for r, _, _ in reqs)
    return {"workload": f"first {len(reqs)} requests of the serving trace (seed 5, Poisson arrivals at {rate} req/s, "
                        f"star surfaces of {sizes[0]}-{sizes[-1]} triangles, direct/Juffer mixed)",
            "served_mixed_bf16": {"slots": slots, "solves_per_s": round(len(reqs) / span, 4),
                                  "p50_s": round(_pct(lat, 0.5), 4), "p99_s": round(_pct(lat, 0.99), 4),
                                  "peak_running": stats["peak_running"],
                                  "peak_inflight_GB": round(stats["peak_inflight_bytes"] / 1e9, 2)},
            "serial_fp64_fifo": {"solves_per_s": round(len(reqs) / ser_span, 4),
                                 "p50_s": round(_pct(ser_lat, 0.5), 4), "p99_s": round(_pct(ser_lat, 0.99), 4),
                                 "how": "pb_solve FP64 (assembled when it fits), one request at a time in "
                                        "arrival order, measured"},
            "dG_rel_err_vs_fp64_max": worst}


def cpu_baseline(mesh, iterations, nrows, P, key):
    """The FP64 oracle timed on this host: operator rows of a bounded sample of
    vertices (both formulations), in kernel pairs per second, and the solves/s
    it implies when scaled to full products times the GPU run's iterations."""
    import oracle
    oracle.lib()
    rng = np.random.default_rng(7)
    rows = np.sort(rng.choice(mesh.n_vertices, nrows, replace=False))
    x = rng.standard_normal(2 * mesh.n_vertices)
    t_solve = 0.0
    pairs = 0.0
    t_all = 0.0
    for f in (0, 1):
        t0 = time.perf_counter()
        oracle.system_rows(mesh, 4.0, 80.0, 0.125, f, rows, x)
        dt = time.perf_counter() - t0
        t_all += dt
        t_solve += dt * mesh.n_vertices / nrows * (iterations.get(str(f), 0) + 1)
        pairs += float(P) * P * nrows / mesh.n_vertices
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    cores = min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))
    return {"value": round(pairs / t_all, 1), "unit": "kernel-pairs/s", "cores": cores, "kind": "oracle",
            "solves_per_s": round(2.0 / t_solve, 7) if t_solve > 0 else None,
            "sample": f"oracle operator rows (FP64, every ordered triangle pair of the sampled rows) for {nrows} "
                      f"sampled vertices per formulation (direct, Juffer) on the {key} workload, {t_all:.1f} s "
                      f"of CPU time: their share of the products' kernel pairs per second; solves/s scales "
                      f"the rows to full products times the GPU run's iterations + 1"}


def serving(argv=None):
    """The whole serving trace (512 requests by default): served on the
    continuous-batching server in mixed BF16 and replayed serially in FIFO
    order with the plain FP64 solve, both measured (serving_prefix)."""
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--slots", type=int, default=8)
    a, _ = ap.parse_known_args(argv)
    rec = serving_prefix(a.requests, a.rate, a.slots)
    rec["workload"] = rec["workload"].replace(f"first {a.requests} requests of the serving trace",
                                              f"serving trace, {a.requests} requests")
    print(json.dumps(rec), flush=True)


def multi(argv=None):
    """16 charge sets on the 40962-vertex sphere, solved together on one
    resident mesh (pb_solve_multi): the MFMA GEMM on the 16-bit far field."""
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--freq", type=int, default=64)
    a, _ = ap.parse_known_args(argv)
    import paper_2108_10481_amd as pbm
    mesh, sets = inputs.config_sphere_multi(freq=a.freq)
    args = [(c.xyz, c.q) for c in sets]
    out = {}
    ref = None
    for name, prec in (("fp64", pbm.PB_FP64), ("fp32", pbm.PB_FP32), ("mixed-bf16", pbm.PB_MIXED_BF16),
                       ("mixed-fp16", pbm.PB_MIXED_FP16)):
        with pbm.MeshHandle(mesh.xyz, mesh.tri, pbm.pb_default_options(precision=prec,
                                                                       operator_mode=pbm.PB_ASSEMBLED)) as h:
            t_setup = h.info()
            res = pbm.pb_solve_multi(h, args)
            if name == "fp64":
                ref = [r["dG"] for r in res]
            steps = 1 if name == "fp64" else a.steps
            for _ in range(0 if name == "fp64" else a.warmup):
                pbm.pb_solve_multi(h, args)
            pbm.pb_mesh_profile(h, True)
            t0 = time.perf_counter()
            for _ in range(steps):
                res = pbm.pb_solve_multi(h, args)
            dt = (time.perf_counter() - t0) / steps
            n, ms, work = pbm.pb_mesh_profile_read(h, 0)
            t_setup = h.info()   # after the batched products (the GEMM's tiled copy included)
            err = max(abs(r["dG"] - g) / abs(g) for r, g in zip(res, ref))
            out[name] = {"solves_per_s": round(len(sets) / dt, 3), "s_per_16_set_batch": round(dt, 4),
                         "inner_iterations_max": max(r["iterations"] for r in res),
                         "outer_iterations_max": max(r["outer_iterations"] for r in res),
                         "dG_rel_err_vs_fp64_max": err,
                         "operator_product": {"launches": n, "avg_ms": round(ms / max(n, 1), 4),
                                              "GB_per_s": round(work / (ms * 1e-3) / 1e9, 1) if ms > 0 else None,
                                              "hbm_frac": round(work / (ms * 1e-3) / 8e12, 4) if ms > 0 else None},
                         "device_GB": round(t_setup["device_bytes"] / 1e9, 2)}
    rec = {"workload": f"sphere R=10 A, {mesh.n_triangles} triangles / {mesh.n_vertices} vertices, 16 charge sets x "
                       "50 charges (seeds 40..55), direct formulation, assembled far field; resident mesh, "
                       "pb_solve_multi per batch (setup excluded)", "results": out}
    print(json.dumps(rec), flush=True)


def calderon(argv=None):
    """PMCHWT formulations on the 20480-triangle sphere with the mass matrix and
    every Calderon preconditioner (the paper's Cases 15-26, 20b, 23b): complete
    solves (every device stage redone per solve, as in the default workload),
    iterations, Krylov time per iteration, Delta G against the FP64 matrix-free
    mass-preconditioned solve."""
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "mixed-bf16"])
    a, _ = ap.parse_known_args(argv)
    import paper_2108_10481_amd as pbm
    prec = {"fp64": pbm.PB_FP64, "fp32": pbm.PB_FP32, "mixed-bf16": pbm.PB_MIXED_BF16}[a.precision]
    mesh, ch = inputs.config_sphere()
    cases = [("mass", pbm.PB_MASS, 0), ("calderon", pbm.PB_CALDERON, 0), ("calderon_int", pbm.PB_CALDERON_INT, 0),
             ("calderon_ext", pbm.PB_CALDERON_EXT, 0), ("scaled_calderon_int", pbm.PB_SCALED_CALDERON_INT, 0),
             ("scaled_calderon_ext", pbm.PB_SCALED_CALDERON_EXT, 0), ("fast_calderon", pbm.PB_CALDERON, 1),
             ("fast_scaled_calderon_int", pbm.PB_SCALED_CALDERON_INT, 1)]
    out = {}
    for form, fname in ((pbm.PB_PMCHWT_INT, "pmchwt_int"), (pbm.PB_PMCHWT_EXT, "pmchwt_ext")):
        ref = pbm.pb_solve(mesh.xyz, mesh.tri, ch.xyz, ch.q,
                           pbm.pb_default_options(formulation=form, preconditioner=pbm.PB_MASS))["dG"]
        for name, pc, fast in cases:
            opt = pbm.pb_default_options(formulation=form, precision=prec, operator_mode=pbm.PB_ASSEMBLED,
                                         preconditioner=pc, calderon_fast=fast)
            with pbm.MeshHandle(mesh.xyz, mesh.tri, opt) as h:
                for _ in range(a.warmup):
                    pbm.pb_mesh_refresh(h)
                    pbm.pb_mesh_solve(h, ch.xyz, ch.q)
                t_set, t_kry, res = [], [], None
                t0 = time.perf_counter()
                for _ in range(a.steps):
                    s0 = time.perf_counter()
                    pbm.pb_mesh_refresh(h)
                    t_set.append(time.perf_counter() - s0)
                    res = pbm.pb_mesh_solve(h, ch.xyz, ch.q)
                    t_kry.append(res["t_gmres"])
                dt = (time.perf_counter() - t0) / a.steps
                gb = h.info()["device_bytes"] / 1e9
            its = res["iterations"]
            out[f"{fname}/{name}"] = {
                "solves_per_s": round(1.0 / dt, 3), "ms_per_solve": round(1e3 * dt, 2),
                "setup_ms": round(1e3 * min(t_set), 2), "iterations": its,
                "krylov_ms": round(1e3 * min(t_kry), 3),
                "krylov_ms_per_iteration": round(1e3 * min(t_kry) / max(its, 1), 3),
                "status": res["status"], "rel_residual": res["rel_residual"],
                "dG_rel_err_vs_fp64_mass": abs(res["dG"] - ref) / abs(ref), "device_GB": round(gb, 2)}
            print(f"calderon: {fname}/{name} done", file=sys.stderr, flush=True)
    rec = {"workload": f"sphere R=10 A, {mesh.n_triangles} triangles / {mesh.n_vertices} vertices, 50 charges, "
                       f"PMCHWT int/ext, {a.precision} assembled, GMRES tol 1e-5; one solve = refresh (geometry, "
                       "near field, assembly of A and P) + solve", "steps": a.steps, "results": out}
    print(json.dumps(rec), flush=True)


def batch(argv=None):
    """Uneven requests solved together (pb_solve_batch) against the same
    requests solved one after the other (pb_mesh_solve, captured GMRES), on two
    mixes of the serving-trace generator's star surfaces (seed 5, FP32
    matrix-free, direct or Juffer, handles resident): 16 requests of
    1280-15680 triangles, and 64 small ones of 1280-5120 triangles, which
    alone leave most of the device idle.  One step = every request of the mix
    solved once; in the fused solve the far fields of all requests still
    iterating run in one persistent launch per kernel form and GMRES
    iteration.  The fused solve's handles evaluate every unordered triangle
    pair once (far_symmetric 1), which a batch of small meshes can fill the
    device with; the one-after-another baseline uses the single-solve default
    (per ordered pair below 3584 triangles).  The fused results are bitwise
    those of single solves on the same handles, which the run checks; the
    fused launches are timed with HIP events.  The first fused call plans
    the far-field work lists and captures the batch graph, which later calls
    with the same handles reuse; its time is reported beside the steps'."""
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    a, _ = ap.parse_known_args(argv)
    import paper_2108_10481_amd as pbm
    out = {}
    for name, nreq, fmax in (("mix16_1280_15680", 16, 32), ("small64_1280_5120", 64, 16)):
        trace = inputs.serving_trace(seed=5, n_requests=nreq, fmax=fmax)
        reqs = [inputs.build_request(r) + (r["formulation"],) for r in trace]
        def handles(sym):
            return [pbm.MeshHandle(m.xyz, m.tri, pbm.pb_default_options(formulation=f, precision=pbm.PB_FP32,
                                                                         operator_mode=pbm.PB_MATRIX_FREE,
                                                                         far_symmetric=sym))
                    for m, _, f in reqs]
        # the fused solve's handles evaluate every unordered triangle pair once
        # (far_symmetric 1: the batch fills the device whatever the mesh sizes);
        # the one-after-another baseline uses the single-solve default (0)
        hs = handles(1)
        ha = handles(0)
        sets = [(c.xyz, c.q) for _, c, _ in reqs]

        def singles(hh):
            return [pbm.pb_mesh_solve(h, *st) for h, st in zip(hh, sets)]

        def fused():
            return pbm.pb_solve_batch(hs, sets)

        t_first = None
        for _ in range(a.warmup):
            singles(ha)
            singles(hs)
            t0 = time.perf_counter()
            fused()
            if t_first is None:   # plans the work lists and captures the batch graph
                t_first = time.perf_counter() - t0
        t0 = time.perf_counter()
        for _ in range(a.steps):
            singles(ha)
        t_single = (time.perf_counter() - t0) / a.steps
        t0 = time.perf_counter()
        for _ in range(a.steps):
            rs = singles(hs)
        t_single_same = (time.perf_counter() - t0) / a.steps
        t0 = time.perf_counter()
        for _ in range(a.steps):
            rb = fused()
        t_fused = (time.perf_counter() - t0) / a.steps
        same = all(x["dG"] == y["dG"] and x["iterations"] == y["iterations"] and np.array_equal(x["phi"], y["phi"])
                   for x, y in zip(rb, rs))
        # one more fused step with the fused far-field launches timed (first handle's profile)
        pbm.pb_mesh_profile(hs[0], 1)
        rp = fused()
        pbm.pb_mesh_synchronize(hs[0])
        launches, ms, pairs = pbm.pb_mesh_profile_read(hs[0], 0)
        pbm.pb_mesh_profile(hs[0], 0)
        flops = sum(rp[k]["iterations"] * 36.0 * m.n_triangles ** 2 * FLOPS_PER_PAIR[f]
                    for k, (m, _, f) in enumerate(reqs))
        achieved = flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        for h in hs + ha:
            h.close()
        sizes = sorted(m.n_triangles for m, _, _ in reqs)
        out[name] = {
            "requests": len(reqs), "triangles_min_max": [sizes[0], sizes[-1]],
            "fused": {"solves_per_s": round(len(reqs) / t_fused, 3), "s_per_step": round(t_fused, 4),
                      "first_call_s": round(t_first, 4) if t_first is not None else None, "far_symmetric": 1},
            "one_after_another": {"solves_per_s": round(len(reqs) / t_single, 3), "s_per_step": round(t_single, 4),
                                  "far_symmetric": 0},
            "one_after_another_same_handles": {"solves_per_s": round(len(reqs) / t_single_same, 3),
                                               "far_symmetric": 1},
            "speedup": round(t_single / t_fused, 3), "bitwise_equal_to_same_handles": bool(same),
            "fused_far_field": {"kernel": "k_far_sym_batch (one launch per kernel form and GMRES iteration)",
                                "products": int(launches), "avg_product_ms": round(ms / max(launches, 1), 4),
                                "kernel_pairs_per_s": round(pairs / (ms * 1e-3), 1) if ms > 0 else None,
                                "bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS["f32"],
                                "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS["f32"], 4)}}
        print(f"batch: {name} done", file=sys.stderr, flush=True)
    rec = {"workload": "serving-trace star surfaces (seed 5), FP32 matrix-free, direct/Juffer mixed, resident "
                       "handles; one step = every request of the mix solved once", "steps": a.steps, "mixes": out}
    print(json.dumps(rec), flush=True)


def large(argv=None):
    """Treecode far field at the paper's largest size: a 450000-triangle /
    225002-vertex star surface (the paper's 1igt has 226312 vertices), 4000
    charges, direct + block-diagonal and Juffer + scaled mass (the paper's
    Cases 2 and 10), FP32 treecode, complete solves with every device stage
    redone; the direct O(N^2) matrix-free product timed once beside it."""
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload")
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--freq", type=int, default=150)
    ap.add_argument("--no-direct", action="store_true")
    a, _ = ap.parse_known_args(argv)
    import paper_2108_10481_amd as pbm
    mesh, ch = inputs.config_star_large(freq=a.freq)
    print(f"large: {mesh.n_triangles} triangles, {mesh.n_vertices} vertices", file=sys.stderr, flush=True)
    out = {}
    x = np.random.default_rng(0).standard_normal(2 * mesh.n_vertices)
    for fname, form, prec in (("direct", pbm.PB_DIRECT_INT, pbm.PB_BLOCK_DIAG),
                              ("juffer", pbm.PB_JUFFER, pbm.PB_SCALED_MASS)):
        opt = pbm.pb_default_options(formulation=form, precision=pbm.PB_FP32, operator_mode=pbm.PB_TREECODE,
                                     preconditioner=prec)
        t0 = time.perf_counter()
        with pbm.MeshHandle(mesh.xyz, mesh.tri, opt) as h:
            t_create = time.perf_counter() - t0
            for _ in range(a.warmup):
                pbm.pb_mesh_refresh(h)
                pbm.pb_mesh_solve(h, ch.xyz, ch.q)
            pbm.pb_mesh_profile(h, 1)
            t1 = time.perf_counter()
            for _ in range(a.steps):
                pbm.pb_mesh_refresh(h)
                r = pbm.pb_mesh_solve(h, ch.xyz, ch.q)
            dt = (time.perf_counter() - t1) / a.steps
            n, ms, w = pbm.pb_mesh_profile_read(h, 0)
            gb = h.info()["device_bytes"] / 1e9
        # treecode product (upward pass + evaluation), HIP events on the handle's stream;
        # algorithmic: every kernel evaluation (target point x source point or proxy)
        # at the direct kernel's flops per pair
        tf = w * FLOPS_PER_PAIR[form] / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        out[fname] = {"s_per_solve": round(dt, 3), "iterations": r["iterations"], "status": r["status"],
                      "dG_kcal": r["dG"], "t_setup_s": round(r["t_setup"], 3), "t_gmres_s": round(r["t_gmres"], 3),
                      "handle_create_s": round(t_create, 2), "device_GB": round(gb, 2),
                      "treecode_product": {"launches": n, "avg_ms": round(ms / max(n, 1), 2),
                                           "evals_per_product": w / max(n, 1),
                                           "evals_per_s": round(w / (ms * 1e-3), 1) if ms > 0 else None},
                      "roofline": {"bound": "alu", "achieved": round(tf, 3), "peak": PEAK_TFLOPS["f32"],
                                   "unit": "TFLOP/s", "frac": round(tf / PEAK_TFLOPS["f32"], 4), "traffic": None,
                                   "kernel": "treecode product (k_tree_charges, k_tree_proxies, k_tree_eval)"}}
        print(f"large: {fname} done", file=sys.stderr, flush=True)
    if not a.no_direct:
        with pbm.MeshHandle(mesh.xyz, mesh.tri, pbm.pb_default_options(formulation=pbm.PB_JUFFER,
                                                                       precision=pbm.PB_FP32)) as h:
            yd = pbm.pb_mesh_apply(h, x)
            pbm.pb_mesh_profile(h, 1)
            pbm.pb_mesh_apply(h, x)
            n, ms, w = pbm.pb_mesh_profile_read(h, 0)
        with pbm.MeshHandle(mesh.xyz, mesh.tri, pbm.pb_default_options(
                formulation=pbm.PB_JUFFER, precision=pbm.PB_FP32, operator_mode=pbm.PB_TREECODE)) as h:
            yt = pbm.pb_mesh_apply(h, x)
        out["direct_product_fp32"] = {"ms": round(ms / max(n, 1), 1), "kernel_pairs": w / max(n, 1),
                                      "treecode_rel_err": float(np.linalg.norm(yt - yd) / np.linalg.norm(yd))}
    rec = {"workload": f"star surface R=36 A (seed 7), {mesh.n_triangles} triangles / {mesh.n_vertices} vertices, "
                       f"{ch.n} charges, FP32 treecode (degree {opt.tree_degree}, theta {opt.tree_theta}), GMRES tol "
                       "1e-5; one solve = refresh + "
                       "solve", "steps": a.steps, "results": out}
    print(json.dumps(rec), flush=True)


def calibrate_copy(nbytes=1 << 30):
    """A plain device-to-device copy of known size (the runtime's copy kernel),
    used to scale the FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import ctypes
    import paper_2108_10481_amd as pbm
    pbm.load()
    hip = ctypes.CDLL("libamdhip64.so.7")
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(a), ctypes.c_size_t(nbytes)) == 0
    assert hip.hipMalloc(ctypes.byref(b), ctypes.c_size_t(nbytes)) == 0
    for _ in range(3):
        assert hip.hipMemcpy(b, a, ctypes.c_size_t(nbytes), 3) == 0   # hipMemcpyDeviceToDevice
    assert hip.hipDeviceSynchronize() == 0
    hip.hipFree(a)
    hip.hipFree(b)
    print(json.dumps({"calibration_copy_bytes": nbytes, "copies": 3}), flush=True)


def measure_peaks():
    """Peaks of this MI355X measured by the microbenchmarks of
    paper_2108_10481_amd/csrc/peaks.hip (libpbm_peaks.so): lane instructions
    per second of v_fma_f32, v_exp_f32, v_rsq_f32 and v_fma_f64 (8 independent
    chains per lane, 8 blocks of 256 lanes per CU), a 4-FMA + 1-exp mix, BF16
    MFMA flop/s (v_mfma_f32_16x16x32_bf16, 4 independent accumulators per
    wavefront) and HBM read / copy bandwidth (4 GiB buffers).  The
    transcendental issue cost is the FMA rate over the transcendental rate."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2108_10481_amd", "libpbm_peaks.so"))
    lib.pbk_compute.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_float),
                                ctypes.POINTER(ctypes.c_double)]
    lib.pbk_stream.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(ctypes.c_float)]
    cus = lib.pbk_cu_count()
    rates = {}
    for kind, name, iters in ((0, "fma32", 200000), (1, "exp32", 100000), (2, "rsq32", 100000),
                              (3, "fma4_exp1", 50000), (4, "fma64", 100000), (5, "mfma_bf16", 50000),
                              (6, "fma4_exp1_indep", 50000), (7, "fma1_exp1_indep", 100000)):
        ms = ctypes.c_float()
        ops = ctypes.c_double()
        if lib.pbk_compute(kind, 8, iters, ctypes.byref(ms), ctypes.byref(ops)) != 0:
            raise RuntimeError(f"peak kernel {name} failed")
        rates[name] = ops.value / (ms.value * 1e-3)
        print(f"peaks: {name} {rates[name]:.4e} /s ({ms.value:.2f} ms)", file=sys.stderr, flush=True)
    bw = {}
    for kind, name, factor in ((0, "hbm_read", 1.0), (1, "hbm_copy", 2.0)):
        ms = ctypes.c_float()
        nbytes = 4 << 30
        if lib.pbk_stream(kind, nbytes, ctypes.byref(ms)) != 0:
            raise RuntimeError(f"stream kernel {name} failed")
        bw[name] = factor * nbytes / (ms.value * 1e-3)
        print(f"peaks: {name} {bw[name] / 1e9:.1f} GB/s", file=sys.stderr, flush=True)
    trans = rates["fma32"] / min(rates["exp32"], rates["rsq32"])
    # the mixes: n FMA + 1 exp per iteration.  If issue slots add, the rate in
    # lane instructions is (n + 1) / (n + trans) of the FMA rate; if the
    # transcendental unit runs beside the FMA pipeline it is (n + 1) / max(n, trans).
    # The extra FMA-pipeline slots one transcendental takes when independent
    # FMAs are there to issue: (n + 1) fma / mix - n, from the 4 + 1 mix.
    mix_pred = rates["fma32"] * 5.0 / (4.0 + trans)
    beside = max(0.0, 5.0 * rates["fma32"] / rates["fma4_exp1_indep"] - 4.0)
    rec = {"device_cus": cus,
           "fma32_lane_ops_per_s": rates["fma32"], "fma32_tflops": 2.0 * rates["fma32"] / 1e12,
           "exp32_lane_ops_per_s": rates["exp32"], "rsq32_lane_ops_per_s": rates["rsq32"],
           "trans_slots": round(trans, 3),
           "mix_4fma_1exp_lane_ops_per_s": rates["fma4_exp1"], "mix_predicted_if_slots_add": mix_pred,
           "mix_4fma_1exp_indep_lane_ops_per_s": rates["fma4_exp1_indep"],
           "mix_4fma_1exp_indep_predicted": {"if_slots_add": mix_pred,
                                             "if_beside": rates["fma32"] * 5.0 / max(4.0, trans)},
           "mix_1fma_1exp_indep_lane_ops_per_s": rates["fma1_exp1_indep"],
           "mix_1fma_1exp_indep_predicted": {"if_slots_add": rates["fma32"] * 2.0 / (1.0 + trans),
                                             "if_beside": rates["fma32"] * 2.0 / max(1.0, trans)},
           "trans_slots_beside_fma": round(beside, 3),
           "fma64_lane_ops_per_s": rates["fma64"], "fma64_tflops": 2.0 * rates["fma64"] / 1e12,
           "mfma_bf16_tflops": 2.0 * rates["mfma_bf16"] / 1e12,
           "hbm_read_GBps": bw["hbm_read"] / 1e9, "hbm_copy_GBps": bw["hbm_copy"] / 1e9,
           "datasheet": {"fp32_vector_tflops": 157.3, "fp64_vector_tflops": 78.6, "bf16_mfma_tflops": 2500.0,
                         "hbm_GBps": 8000.0},
           "note": "packed FP32 (v_pk_fma_f32) is not used by the library; the FMA rate is the unpacked one"}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    if "--calibrate-copy" in sys.argv:
        calibrate_copy()
        sys.exit(0)
    if "--measure-peaks" in sys.argv:
        measure_peaks()
        sys.exit(0)
    wl = sys.argv[sys.argv.index("--workload") + 1] if "--workload" in sys.argv else "star"
    if wl == "serving":
        serving()
    elif wl == "multi":
        multi()
    elif wl == "calderon":
        calderon()
    elif wl == "large":
        large()
    elif wl == "batch":
        batch()
    else:
        main()
