#!/usr/bin/env python3
"""Write tests/golden/sphere20480_dG.txt: the FP64 oracle's solvation energy on
the 20480-triangle sphere workload (radius 10 A, frequency-32 icosphere, 50
charges uniform in r < 8 A with values U[-1, 1] e from seed 2, eps 4 / 80,
kappa 0.125 / A) for the internal direct (Eq. bie:dirichlet:int) and Juffer
(Eq. bie:juffer:int) formulations with the block-diagonal preconditioner,
GMRES without restart at the paper's tolerance 1e-5 and at 1e-10.

Calls only ``oracle`` and the seeded generators in ``inputs``.  The dense
operators take about 17 GB of host memory and several minutes on 8 cores.
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import inputs  # noqa: E402
import oracle  # noqa: E402

EPS_IN, EPS_OUT, KAPPA = 4.0, 80.0, 0.125


def main(out=os.path.join(HERE, "sphere20480_dG.txt")):
    mesh, ch = inputs.config_sphere()
    nv = mesh.n_vertices
    t0 = time.time()
    ops = {}
    for name, kap in (("L", 0.0), ("Y", KAPPA)):
        ops[name] = oracle.assemble(mesh, kap, ("V", "K", "D"))
        ops[name]["T"] = ops[name]["K"].T.copy()
        print(f"operators {name}: {time.time() - t0:.0f} s", flush=True)
    M = oracle.mass(mesh)
    bD, bN = oracle.rhs(mesh, ch, EPS_IN)
    lines = []
    for form, label in ((oracle.DIRECT, "direct"), (oracle.JUFFER, "juffer")):
        A = np.block([list(oracle.system_blocks(ops["L"], ops["Y"], M, EPS_IN, EPS_OUT, form)[:2]),
                      list(oracle.system_blocks(ops["L"], ops["Y"], M, EPS_IN, EPS_OUT, form)[2:])])
        b = oracle.system_rhs(bD, bN, form, EPS_IN, EPS_OUT)
        inv = oracle.block_diagonal_inverse(A, nv)
        P = lambda v: oracle.apply_block_diag(inv, v)
        pb = P(b)
        for tol in (1e-5, 1e-10):
            u, its, _ = oracle.gmres(lambda v: P(A @ v), pb, tol)
            res = float(np.linalg.norm(pb - P(A @ u)) / np.linalg.norm(pb))
            phi, dphi = oracle.interior_traces(u, nv, form, EPS_IN, EPS_OUT)
            dG = oracle.solvation_energy(mesh, ch, phi, dphi)
            lines.append(f"{label} {tol:.0e} {dG:.15e} {its} {res:.3e}")
            print(lines[-1], f"({time.time() - t0:.0f} s)", flush=True)
        del A
    with open(out, "w") as f:
        f.write("# FP64 oracle solvation energy on the 20480-triangle sphere workload: icosphere\n"
                "# frequency 32, radius 10 A (10242 vertices), 50 charges uniform in r < 8 A, values\n"
                "# U[-1, 1] e (seed 2); eps_in 4, eps_out 80, kappa 0.125 / A; block-diagonal\n"
                "# preconditioner; unrestarted GMRES from x0 = 0 (Results: solver setup).\n"
                "# Formulations: internal direct (Eq. bie:dirichlet:int), Juffer (Eq. bie:juffer:int);\n"
                "# energy: Eqs. phireac_bie and dG.  Written by make_sphere20480_golden.py, which\n"
                "# calls only oracle/ and inputs/.\n"
                "# columns: formulation gmres_tol dG_kcal_per_mol iterations rel_residual\n")
        f.write("\n".join(lines) + "\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
