"""FP64 CPU oracle for the boundary-integral Poisson-Boltzmann hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library never calls it and shares no code with it.

Plain and slow on purpose: the per-pair quadrature lives in ``pbm_oracle.c``
(plain C loops, FP64); this module composes the paper's block systems from
dense operator matrices with NumPy, applies the block-diagonal or the (scaled)
mass-matrix preconditioner, runs unrestarted GMRES (modified Gram-Schmidt, Givens
rotations) and evaluates the solvation energy.

Citations are to Search, Cooper & van 't Wout, arXiv 2108.10481:
  * internal / external direct ......... Eqs. bie:dirichlet:int, bie:dirichlet:ext
  * Juffer, Lu formulations ............. Eqs. bie:juffer:int, bie:lu:ext
  * Mueller, PMCHWT formulations ........ Eqs. bie:muller:int/ext, bie:pmchwt:int/ext
  * combined field (alpha, beta) ........ Eqs. bie:combined:int, bie:combined:ext
  * source projections .................. Eq. sources
  * reaction potential, energy .......... Eqs. phireac_bie and dG
  * block-diagonal preconditioner ....... Preconditioning / Algebraic preconditioners
  * (scaled) mass-matrix preconditioner . Eqs. prec:mass and prec:mass:scaled
  * Calderon preconditioners (PMCHWT) ... Eqs. prec:calderon:int, prec:calderon:ext,
                                          precond:calderon:eigenval(_semi)
  * GMRES, tol 1e-5, no restart ......... Results and Discussion (setup paragraph)
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "pbm_oracle.c")

#: e^2 / (4 pi eps0 * 1 angstrom) in kcal/mol.  Potentials here carry a
#: 1/(4 pi) without eps0, so energies are multiplied by 4 pi times this.
COULOMB_KCAL = 332.0637
ENERGY_C = 4.0 * math.pi * COULOMB_KCAL

DIRECT = 0            # internal direct, Eq. bie:dirichlet:int
JUFFER = 1            # Eq. bie:juffer:int
DIRECT_EXT = 2        # external direct, Eq. bie:dirichlet:ext
DIRECT_INT_PERM = 3   # Eq. bie:dirichlet:int with its two rows swapped ("permuted")
DIRECT_EXT_PERM = 4   # Eq. bie:dirichlet:ext with its two rows swapped
MULLER_INT = 5        # Eq. bie:muller:int
MULLER_EXT = 6        # Eq. bie:muller:ext
LU = 7                # Eq. bie:lu:ext
PMCHWT_INT = 8        # Eq. bie:pmchwt:int
PMCHWT_EXT = 9        # Eq. bie:pmchwt:ext
CFIE_INT = 10         # Eq. bie:combined:int (real alpha, beta)
CFIE_EXT = 11         # Eq. bie:combined:ext (real alpha, beta)
FORMULATIONS = tuple(range(12))
#: formulations whose unknowns are the exterior traces (gamma_D^+, gamma_N^+)
EXTERIOR = (DIRECT_EXT, DIRECT_EXT_PERM, MULLER_EXT, LU, PMCHWT_EXT, CFIE_EXT)
#: formulations with only single- and double-layer operators
DIRECT_FAMILY = (DIRECT, DIRECT_EXT, DIRECT_INT_PERM, DIRECT_EXT_PERM)


def build(force: bool = False) -> str:
    """Compile the C part of the oracle with gcc (FP64, no fast-math)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None
_dp = np.ctypeslib.ndpointer(np.float64, flags="C")
_ip = np.ctypeslib.ndpointer(np.int32, flags="C")
_c_int = ctypes.c_int
_c_dbl = ctypes.c_double


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_regular_rule.argtypes = [_dp, _dp]
        L.orc_gauss_legendre01.argtypes = [_c_int, _dp, _dp]
        L.orc_triangle_geometry.argtypes = [_dp, _ip, _c_int, _dp, _dp]
        L.orc_pair_block.argtypes = [_dp, _ip, _c_int, _c_int, _c_dbl, _c_int, _c_int, _c_int, _dp, _dp]
        L.orc_pair_block.restype = _c_int
        L.orc_operator_rows.argtypes = [_c_int, _c_int, _dp, _ip, _c_dbl, _c_int, _c_int, _ip, _c_int,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, _c_int]
        L.orc_mass_rows.argtypes = [_c_int, _c_int, _dp, _ip, _c_int, _ip, _dp]
        L.orc_rhs.argtypes = [_c_int, _c_int, _dp, _ip, _c_int, _dp, _dp, _c_dbl, _dp, _dp]
        L.orc_reaction_potential.argtypes = [_c_int, _c_int, _dp, _ip, _dp, _dp, _c_int, _dp, _dp]
        _lib = L
    return _lib


def _mesh_arrays(mesh):
    return (np.ascontiguousarray(mesh.xyz, dtype=np.float64),
            np.ascontiguousarray(mesh.tri, dtype=np.int32))


# ------------------------------------------------------------------ rules
def regular_rule():
    b = np.zeros(18)
    w = np.zeros(6)
    lib().orc_regular_rule(b, w)
    return b.reshape(6, 3), w


def gauss_legendre01(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    if lib().orc_gauss_legendre01(n, x, w) != 0:
        raise ValueError(n)
    return x, w


def triangle_geometry(mesh):
    xyz, tri = _mesh_arrays(mesh)
    a = np.zeros(len(tri))
    n = np.zeros((len(tri), 3))
    lib().orc_triangle_geometry(xyz, tri, len(tri), a, n)
    return a, n


def pair_block(mesh, t: int, s: int, kappa: float, nss: int = 4,
               kernel_mode: int = 0, quad_mode: int = 0):
    """Local 3x3 blocks (V, K) of the ordered pair (test t, trial s)."""
    xyz, tri = _mesh_arrays(mesh)
    V = np.zeros(9)
    K = np.zeros(9)
    ns = lib().orc_pair_block(xyz, tri, int(t), int(s), float(kappa), int(nss),
                              int(kernel_mode), int(quad_mode), V, K)
    return V.reshape(3, 3), K.reshape(3, 3), ns


# -------------------------------------------------------------- operators
def operator_rows(mesh, kappa: float, rows, mode: int = 0, want=("V", "K", "D"), nss: int = 4,
                  centroid: bool = False):
    """Rows (mode 0) or columns (mode 1) of V, K, D for the kernel exp(-kappa r)/(4 pi r).
    centroid: the one-point rule instead of the 6-point rule on pairs sharing no vertex."""
    xyz, tri = _mesh_arrays(mesh)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    nv = len(xyz)
    out = {k: np.zeros((len(rows), nv)) for k in want}
    ptr = lambda k: out[k].ctypes.data_as(ctypes.c_void_p) if k in out else None
    lib().orc_operator_rows(nv, len(tri), xyz, tri, float(kappa), int(nss), len(rows), rows,
                            int(mode), ptr("V"), ptr("K"), ptr("D"), 2 if centroid else 0)
    return out


def assemble(mesh, kappa: float, want=("V", "K", "D"), nss: int = 4, centroid: bool = False):
    """Dense V, K, D (rows = test vertex, columns = trial vertex)."""
    return operator_rows(mesh, kappa, np.arange(mesh.n_vertices), 0, want, nss, centroid)


def mass_rows(mesh, rows):
    xyz, tri = _mesh_arrays(mesh)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.zeros((len(rows), len(xyz)))
    lib().orc_mass_rows(len(xyz), len(tri), xyz, tri, len(rows), rows, out)
    return out


def mass(mesh):
    return mass_rows(mesh, np.arange(mesh.n_vertices))


# --------------------------------------------------------------- sources
def rhs(mesh, charges, eps_in: float):
    """Galerkin-tested source projections (b_D, b_N) of Eq. sources."""
    xyz, tri = _mesh_arrays(mesh)
    bD = np.zeros(len(xyz))
    bN = np.zeros(len(xyz))
    lib().orc_rhs(len(xyz), len(tri), xyz, tri, charges.n,
                  np.ascontiguousarray(charges.xyz, dtype=np.float64),
                  np.ascontiguousarray(charges.q, dtype=np.float64), float(eps_in), bD, bN)
    return bD, bN


def reaction_potential(mesh, phi, dphi, pts):
    """phi_reac at points (Eq. phireac_bie), Laplace potentials of the traces."""
    xyz, tri = _mesh_arrays(mesh)
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(len(pts))
    lib().orc_reaction_potential(len(xyz), len(tri), xyz, tri,
                                 np.ascontiguousarray(phi, dtype=np.float64),
                                 np.ascontiguousarray(dphi, dtype=np.float64), len(pts), pts, out)
    return out


def solvation_energy(mesh, charges, phi, dphi):
    """Delta G = 1/2 sum_j q_j phi_reac(x_j) (Eq. dG), in kcal/mol."""
    pr = reaction_potential(mesh, phi, dphi, charges.xyz)
    return 0.5 * ENERGY_C * float(np.dot(charges.q, pr))


# ------------------------------------------------------------ formulations
def system_blocks(ops_L, ops_Y, M, eps_in, eps_out, formulation, alpha=1.0, beta=1.0):
    """2x2 block system of the chosen formulation, Galerkin form, typed in as
    the paper prints it.

    ops_L / ops_Y hold V, K and (second-kind and PMCHWT formulations) D and T
    of the Laplace ("int") and Yukawa ("ext") kernels; the identity becomes
    the mass matrix M.  e = eps_in / eps_out; alpha, beta: the constants of
    the combined-field formulations.
    """
    e = eps_in / eps_out
    L, Y = ops_L, ops_Y
    if formulation == CFIE_INT:                     # Eq. bie:combined:int
        # interior trace equations + diag(alpha, beta) exterior trace equations
        A11 = (0.5 * M + L["K"]) + alpha * (0.5 * M - Y["K"])
        A12 = -L["V"] + alpha * (e * Y["V"])
        A21 = -L["D"] + beta * ((1.0 / e) * Y["D"])
        A22 = (0.5 * M - L["T"]) + beta * (0.5 * M + Y["T"])
        return A11, A12, A21, A22
    if formulation == CFIE_EXT:                     # Eq. bie:combined:ext
        # exterior trace equations + diag(alpha, beta) interior trace equations
        A11 = (0.5 * M - Y["K"]) + alpha * (0.5 * M + L["K"])
        A12 = Y["V"] + alpha * (-(1.0 / e) * L["V"])
        A21 = Y["D"] + beta * (-e * L["D"])
        A22 = (0.5 * M + Y["T"]) + beta * (0.5 * M - L["T"])
        return A11, A12, A21, A22
    if formulation == DIRECT:                       # Eq. bie:dirichlet:int
        A11 = 0.5 * M + L["K"]
        A12 = -L["V"]
        A21 = 0.5 * M - Y["K"]
        A22 = e * Y["V"]
    elif formulation == DIRECT_EXT:                 # Eq. bie:dirichlet:ext
        A11 = 0.5 * M - Y["K"]
        A12 = Y["V"]
        A21 = 0.5 * M + L["K"]
        A22 = -(1.0 / e) * L["V"]
    elif formulation == DIRECT_INT_PERM:            # rows of Eq. bie:dirichlet:int swapped
        A11 = 0.5 * M - Y["K"]
        A12 = e * Y["V"]
        A21 = 0.5 * M + L["K"]
        A22 = -L["V"]
    elif formulation == DIRECT_EXT_PERM:            # rows of Eq. bie:dirichlet:ext swapped
        A11 = 0.5 * M + L["K"]
        A12 = -(1.0 / e) * L["V"]
        A21 = 0.5 * M - Y["K"]
        A22 = Y["V"]
    elif formulation == JUFFER:                     # Eq. bie:juffer:int
        a = eps_out / eps_in
        b = eps_in / eps_out
        A11 = 0.5 * (1.0 + a) * M + L["K"] - a * Y["K"]
        A12 = -L["V"] + Y["V"]
        A21 = -L["D"] + Y["D"]
        A22 = 0.5 * (1.0 + b) * M - L["T"] + b * Y["T"]
    elif formulation == MULLER_INT:                 # Eq. bie:muller:int
        A11 = M + L["K"] - Y["K"]
        A12 = -L["V"] + e * Y["V"]
        A21 = -L["D"] + (1.0 / e) * Y["D"]
        A22 = M - L["T"] + Y["T"]
    elif formulation == MULLER_EXT:                 # Eq. bie:muller:ext
        A11 = M - Y["K"] + L["K"]
        A12 = Y["V"] - (1.0 / e) * L["V"]
        A21 = Y["D"] - e * L["D"]
        A22 = M + Y["T"] - L["T"]
    elif formulation == LU:                         # Eq. bie:lu:ext
        A11 = 0.5 * (1.0 + e) * M - Y["K"] + e * L["K"]
        A12 = Y["V"] - L["V"]
        A21 = e * Y["D"] - e * L["D"]
        A22 = 0.5 * (1.0 + e) * M + e * Y["T"] - L["T"]
    elif formulation == PMCHWT_INT:                 # Eq. bie:pmchwt:int
        A11 = -L["K"] - Y["K"]
        A12 = L["V"] + e * Y["V"]
        A21 = L["D"] + (1.0 / e) * Y["D"]
        A22 = L["T"] + Y["T"]
    elif formulation == PMCHWT_EXT:                 # Eq. bie:pmchwt:ext
        A11 = -Y["K"] - L["K"]
        A12 = Y["V"] + (1.0 / e) * L["V"]
        A21 = Y["D"] + e * L["D"]
        A22 = Y["T"] + L["T"]
    else:
        raise ValueError(formulation)
    return A11, A12, A21, A22


def _want(formulation):
    return ("V", "K") if formulation in DIRECT_FAMILY else ("V", "K", "D")


def system_matrix(mesh, eps_in, eps_out, kappa, formulation, nss: int = 4, alpha=1.0, beta=1.0,
                  centroid: bool = False):
    """Dense system; centroid: the one-point rule on pairs sharing no vertex
    (regular order 1) instead of the 6-point rule."""
    want = _want(formulation)
    oL = assemble(mesh, 0.0, want, nss, centroid)
    oY = assemble(mesh, kappa, want, nss, centroid)
    if "D" in want:
        oL["T"] = oL["K"].T.copy()                  # adjoint double layer as K^T
        oY["T"] = oY["K"].T.copy()
    M = mass(mesh)
    A11, A12, A21, A22 = system_blocks(oL, oY, M, eps_in, eps_out, formulation, alpha, beta)
    return np.block([[A11, A12], [A21, A22]])


def system_rhs(bD, bN, formulation, eps_in: float = 4.0, eps_out: float = 80.0, alpha=1.0, beta=1.0):
    """Right-hand side of the formulation from the source projections
    <phi_i, varphi_D>, <phi_i, varphi_N> (Eq. sources), as printed."""
    e = eps_in / eps_out
    z = np.zeros_like(bD)
    rhs = {DIRECT: (bD, z), DIRECT_EXT: (z, bD), DIRECT_INT_PERM: (z, bD), DIRECT_EXT_PERM: (bD, z),
           JUFFER: (bD, bN), MULLER_INT: (bD, bN), MULLER_EXT: (bD, e * bN), LU: (e * bD, e * bN),
           PMCHWT_INT: (-bD, -bN), PMCHWT_EXT: (-bD, -e * bN),
           CFIE_INT: (bD, bN), CFIE_EXT: (alpha * bD, beta * e * bN)}[formulation]
    return np.concatenate(rhs)


def interior_traces(u, nv, formulation, eps_in: float = 4.0, eps_out: float = 80.0):
    """(gamma_D^- phi, gamma_N^- phi) from a solution vector: exterior traces
    give the interior ones by the interface conditions (potential continuous,
    eps_in gamma_N^- = eps_out gamma_N^+)."""
    phi, dphi = u[:nv], u[nv:]
    if formulation in EXTERIOR:
        dphi = (eps_out / eps_in) * dphi
    return phi, dphi


def system_rows(mesh, eps_in, eps_out, kappa, formulation, rows, x, nss: int = 4, alpha=1.0, beta=1.0,
                centroid: bool = False):
    """Sampled rows of y = A x for large meshes: returns (y1[rows], y2[rows])."""
    rows = np.asarray(rows, dtype=np.int32)
    nv = mesh.n_vertices
    x1, x2 = x[:nv], x[nv:]
    want = _want(formulation)
    oL = operator_rows(mesh, 0.0, rows, 0, want, nss, centroid)
    oY = operator_rows(mesh, kappa, rows, 0, want, nss, centroid)
    if "D" in want:
        oL["T"] = operator_rows(mesh, 0.0, rows, 1, ("K",), nss, centroid)["K"]
        oY["T"] = operator_rows(mesh, kappa, rows, 1, ("K",), nss, centroid)["K"]
    M = mass_rows(mesh, rows)
    A11, A12, A21, A22 = system_blocks(oL, oY, M, eps_in, eps_out, formulation, alpha, beta)
    return A11 @ x1 + A12 @ x2, A21 @ x1 + A22 @ x2


def block_diagonal_inverse(A, nv):
    """Per-vertex 2x2 inverse of [[A11_ii, A12_ii], [A21_ii, A22_ii]]."""
    d = np.arange(nv)
    a = A[d, d]
    b = A[d, nv + d]
    c = A[nv + d, d]
    e = A[nv + d, nv + d]
    det = a * e - b * c
    inv = np.empty((nv, 2, 2))
    inv[:, 0, 0] = e / det
    inv[:, 0, 1] = -b / det
    inv[:, 1, 0] = -c / det
    inv[:, 1, 1] = a / det
    return inv


def apply_block_diag(inv, v):
    nv = inv.shape[0]
    v1, v2 = v[:nv], v[nv:]
    return np.concatenate([inv[:, 0, 0] * v1 + inv[:, 0, 1] * v2,
                           inv[:, 1, 0] * v1 + inv[:, 1, 1] * v2])


def mass_scales(eps_in, eps_out, formulation, scaled: bool):
    """(a, b) of blockdiag(aM, bM): 1, 1 for the plain mass matrix (Eq.
    prec:mass); for the Juffer formulation scaled as the Mass-matrix
    preconditioning paragraph states, a = 1 + eps_out/eps_in and
    b = 1 + eps_in/eps_out (Eq. prec:mass:scaled)."""
    if not scaled:
        return 1.0, 1.0
    if formulation != JUFFER:
        raise ValueError("the scaled mass preconditioner is defined for the Juffer formulation")
    return 1.0 + eps_out / eps_in, 1.0 + eps_in / eps_out


def mass_preconditioner(mesh, a: float = 1.0, b: float = 1.0):
    """v -> blockdiag(aM, bM)^-1 v with M the P1 mass matrix, through a dense
    Cholesky factorisation of M (M is symmetric positive definite)."""
    import scipy.linalg as sla
    nv = mesh.n_vertices
    F = sla.cho_factor(mass(mesh))

    def apply(v):
        return np.concatenate([sla.cho_solve(F, v[:nv]) / a, sla.cho_solve(F, v[nv:]) / b])
    return apply


# ------------------------------------------------------------- Calderon
#: preconditioner names of the Calderon-preconditioned PMCHWT systems: the
#: whole PMCHWT matrix, its interior-kernel or its exterior-kernel part as
#: the preconditioning operator, the halves optionally with the scaled mass
#: matrix on top (Calderon preconditioning paragraph)
CALDERON = ("calderon", "calderon_int", "calderon_ext", "scaled_calderon_int", "scaled_calderon_ext")


def calderon_part(preconditioner: str) -> str:
    return {"calderon": "full", "calderon_int": "int", "calderon_ext": "ext",
            "scaled_calderon_int": "int", "scaled_calderon_ext": "ext"}[preconditioner]


def calderon_blocks(ops_L, ops_Y, M, eps_in, eps_out, formulation, part):
    """Blocks of the preconditioning operator P of the Calderon-preconditioned
    PMCHWT systems, typed in as printed: the full PMCHWT matrix (Eqs.
    prec:calderon:int:full, prec:calderon:ext:full), its interior-kernel part
    (Eqs. prec:calderon:int:int, prec:calderon:ext:int) or its exterior-kernel
    part (Eqs. prec:calderon:int:ext, prec:calderon:ext:ext).  "Int" is the
    Laplace kernel, "ext" the Yukawa kernel; D is the hypersingular and T the
    adjoint double-layer operator.  e = eps_in / eps_out."""
    if formulation not in (PMCHWT_INT, PMCHWT_EXT):
        raise ValueError("Calderon preconditioning is defined for the PMCHWT formulations")
    e = eps_in / eps_out
    L, Y = ops_L, ops_Y
    if part == "full":
        return system_blocks(ops_L, ops_Y, M, eps_in, eps_out, formulation)
    if formulation == PMCHWT_INT:
        if part == "int":                           # Eq. prec:calderon:int:int
            return -L["K"], L["V"], L["D"], L["T"]
        if part == "ext":                           # Eq. prec:calderon:int:ext
            return -Y["K"], e * Y["V"], (1.0 / e) * Y["D"], Y["T"]
    else:
        if part == "ext":                           # Eq. prec:calderon:ext:ext
            return -Y["K"], Y["V"], Y["D"], Y["T"]
        if part == "int":                           # Eq. prec:calderon:ext:int
            return -L["K"], (1.0 / e) * L["V"], e * L["D"], L["T"]
    raise ValueError(part)


#: fast Calderon (Discussion): the preconditioner's operator with relaxed
#: quadrature, the one-point rule on pairs sharing no vertex and one Gauss
#: point fewer per dimension in the Sauter-Schwab rule
FAST_NSS = 3


def calderon_matrix(mesh, eps_in, eps_out, kappa, formulation, part, nss: int = 4, fast: bool = False):
    """Galerkin matrix of the preconditioning operator P (weak form, 2V x 2V);
    fast: assembled with the relaxed quadrature of the fast variant."""
    if fast:
        nss = FAST_NSS
    oL = assemble(mesh, 0.0, ("V", "K", "D"), nss, centroid=fast)
    oY = assemble(mesh, kappa, ("V", "K", "D"), nss, centroid=fast)
    oL["T"] = oL["K"].T.copy()
    oY["T"] = oY["K"].T.copy()
    P11, P12, P21, P22 = calderon_blocks(oL, oY, mass(mesh), eps_in, eps_out, formulation, part)
    return np.block([[P11, P12], [P21, P22]])


def calderon_rows(mesh, eps_in, eps_out, kappa, formulation, part, rows, x, nss: int = 4, fast: bool = False):
    """Sampled rows of y = P x for large meshes: returns (y1[rows], y2[rows])."""
    rows = np.asarray(rows, dtype=np.int32)
    nv = mesh.n_vertices
    if fast:
        nss = FAST_NSS
    oL = operator_rows(mesh, 0.0, rows, 0, ("V", "K", "D"), nss, fast)
    oY = operator_rows(mesh, kappa, rows, 0, ("V", "K", "D"), nss, fast)
    oL["T"] = operator_rows(mesh, 0.0, rows, 1, ("K",), nss, fast)["K"]
    oY["T"] = operator_rows(mesh, kappa, rows, 1, ("K",), nss, fast)["K"]
    P11, P12, P21, P22 = calderon_blocks(oL, oY, mass_rows(mesh, rows), eps_in, eps_out, formulation, part)
    return P11 @ x[:nv] + P12 @ x[nv:], P21 @ x[:nv] + P22 @ x[nv:]


def calderon_points(eps_in, eps_out):
    """Accumulation points of the Calderon-preconditioned PMCHWT spectra:
    full (Eq. precond:calderon:eigenval) and the two half points (Eq.
    precond:calderon:eigenval_semi)."""
    full = 0.5 + eps_out / (4.0 * eps_in) + eps_in / (4.0 * eps_out)
    return full, 0.25 + eps_out / (4.0 * eps_in), 0.25 + eps_in / (4.0 * eps_out)


def calderon_scales(eps_in, eps_out, formulation, part):
    """(a, b) of the scaled mass matrix on top of a half Calderon
    preconditioner.  The paper takes the two half points as a and b "or vice
    versa"; which point belongs to which block row follows from the leading
    (high-frequency) part of the product, where V D = D V = 1/4 for either
    kernel while K K, K V and V T vanish: with A = [[., alpha V], [beta D, .]]
    and P = [[., gamma V], [delta D, .]], P A becomes lower triangular with
    diagonal (gamma beta, delta alpha) / 4, its eigenvalues.
    Internal PMCHWT: alpha = 1 + e, beta = 1 + 1/e; its interior part has
    gamma = delta = 1 -> (half_1, half_2), its exterior part gamma = e,
    delta = 1/e -> (half_2, half_1).  External PMCHWT: alpha = 1 + 1/e,
    beta = 1 + e; exterior part gamma = delta = 1 -> (half_2, half_1),
    interior part gamma = 1/e, delta = e -> (half_1, half_2).  With P = A
    both rows give the full point."""
    _, h1, h2 = calderon_points(eps_in, eps_out)
    if formulation == PMCHWT_INT:
        return (h1, h2) if part == "int" else (h2, h1)
    if formulation == PMCHWT_EXT:
        return (h2, h1) if part == "ext" else (h1, h2)
    raise ValueError("Calderon preconditioning is defined for the PMCHWT formulations")


def calderon_preconditioner(mesh, P, a: float = 1.0, b: float = 1.0):
    """v -> blockdiag(aM, bM)^-1 P blockdiag(M, M)^-1 v: the Galerkin form of
    the operator product P A (the mass matrix maps the weak form of A back
    to coefficients before P acts, and after it for the strong form)."""
    M1 = mass_preconditioner(mesh)
    Ms = mass_preconditioner(mesh, a, b)

    def apply(v):
        return Ms(P @ M1(v))
    return apply


def gmres(apply, b, tol: float = 1e-5, max_iter: int = 1000):
    """Unrestarted GMRES from x0 = 0 with modified Gram-Schmidt and Givens
    rotations; stops when the residual estimate drops below tol * |b|.
    Returns (x, iterations, residual-estimate history)."""
    n = b.size
    beta = float(np.linalg.norm(b))
    if beta == 0.0:
        return np.zeros(n), 0, [0.0]
    m = min(max_iter, n)
    Q = np.zeros((m + 1, n))
    H = np.zeros((m + 1, m))
    cs = np.zeros(m)
    sn = np.zeros(m)
    g = np.zeros(m + 1)
    g[0] = beta
    Q[0] = b / beta
    hist = [beta]
    k = 0
    for j in range(m):
        w = apply(Q[j])
        for i in range(j + 1):
            H[i, j] = np.dot(w, Q[i])
            w = w - H[i, j] * Q[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] > 0:
            Q[j + 1] = w / H[j + 1, j]
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        den = math.hypot(H[j, j], H[j + 1, j])
        cs[j] = H[j, j] / den
        sn[j] = H[j + 1, j] / den
        H[j, j] = den
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        k = j + 1
        hist.append(abs(g[j + 1]))
        if abs(g[j + 1]) <= tol * beta:
            break
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
    return Q[:k].T @ y, k, hist


def solve(mesh, charges, eps_in=4.0, eps_out=80.0, kappa=0.125, formulation=DIRECT,
          preconditioner=True, tol=1e-5, max_iter=1000, nss: int = 4, A=None, fast: bool = False,
          alpha=1.0, beta=1.0, centroid: bool = False):
    """Dense FP64 solve: returns dict(phi, dphi, dG, iterations, rel_residual).
    preconditioner: True or "block_diag", False or None, "mass", "scaled_mass",
    or one of CALDERON (PMCHWT formulations); fast: the Calderon operator with
    the relaxed quadrature of the fast variant; alpha, beta: the constants of
    the combined-field formulations; centroid: the system with the one-point
    rule on pairs sharing no vertex (regular order 1; right-hand side and
    Delta G keep the 6-point rule)."""
    nv = mesh.n_vertices
    if A is None:
        A = system_matrix(mesh, eps_in, eps_out, kappa, formulation, nss, alpha, beta, centroid)
    bD, bN = rhs(mesh, charges, eps_in)
    b = system_rhs(bD, bN, formulation, eps_in, eps_out, alpha, beta)
    if preconditioner is True or preconditioner == "block_diag":
        inv = block_diagonal_inverse(A, nv)
        P = lambda v: apply_block_diag(inv, v)
    elif preconditioner in ("mass", "scaled_mass"):
        a, bb = mass_scales(eps_in, eps_out, formulation, preconditioner == "scaled_mass")
        P = mass_preconditioner(mesh, a, bb)
    elif preconditioner in CALDERON:
        part = calderon_part(preconditioner)
        Pm = (A if part == "full" and not fast
              else calderon_matrix(mesh, eps_in, eps_out, kappa, formulation, part, nss, fast))
        a, bb = (calderon_scales(eps_in, eps_out, formulation, part) if preconditioner.startswith("scaled")
                 else (1.0, 1.0))
        P = calderon_preconditioner(mesh, Pm, a, bb)
    elif preconditioner is False or preconditioner is None:
        P = lambda v: v
    else:
        raise ValueError(f"unknown preconditioner {preconditioner!r}")
    pb = P(b)
    u, its, hist = gmres(lambda v: P(A @ v), pb, tol, max_iter)
    res = float(np.linalg.norm(pb - P(A @ u)) / np.linalg.norm(pb))
    phi, dphi = interior_traces(u, nv, formulation, eps_in, eps_out)
    dG = solvation_energy(mesh, charges, phi, dphi)
    return {"phi": phi, "dphi": dphi, "dG": dG, "iterations": its, "rel_residual": res,
            "history": hist, "A": A, "b": b}
