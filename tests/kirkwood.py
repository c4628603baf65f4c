"""Closed-form references used to pin the oracle (textbook results, not the paper).

* Kirkwood's solvation energy of point charges inside a dielectric sphere in an
  ionic solvent (J. G. Kirkwood, J. Chem. Phys. 2, 351 (1934)), written for the
  linearised Poisson-Boltzmann interface problem of the paper's
  Eq. poissonboltzmann.
* Eigenvalues of the Laplace and Yukawa boundary operators on a sphere, from
  the addition theorem of the Green's function in spherical harmonics.

Both use SciPy's special functions only, so they share nothing with the oracle.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import eval_legendre, spherical_in, spherical_kn

COULOMB_KCAL = 332.0637


def _g(l: int, x: float) -> float:
    """x k_l'(x) / k_l(x) for the modified spherical Bessel function k_l."""
    return x * spherical_kn(l, x, derivative=True) / spherical_kn(l, x)


def kirkwood_energy(radius, qxyz, q, eps_in=4.0, eps_out=80.0, kappa=0.125, lmax=60):
    """Polar solvation energy (kcal/mol) of charges q at qxyz inside a sphere."""
    a = float(radius)
    qxyz = np.asarray(qxyz, dtype=float).reshape(-1, 3)
    q = np.asarray(q, dtype=float)
    r = np.linalg.norm(qxyz, axis=1)
    n = len(q)
    cosg = np.ones((n, n))
    for i in range(n):
        for k in range(n):
            if r[i] > 0 and r[k] > 0:
                cosg[i, k] = np.clip(np.dot(qxyz[i], qxyz[k]) / (r[i] * r[k]), -1, 1)
    x = kappa * a
    total = 0.0
    for l in range(lmax + 1):
        gl = _g(l, x) if kappa > 0 else -(l + 1.0)
        fac = (eps_in * (l + 1) + eps_out * gl) / (eps_in * l - eps_out * gl)
        rr = np.outer(r, r) / a ** 2
        with np.errstate(invalid="ignore"):
            pw = np.where(rr > 0, rr ** l, 1.0 if l == 0 else 0.0)
        total += fac * np.sum(np.outer(q, q) * pw * eval_legendre(l, cosg))
    return COULOMB_KCAL / 2.0 * total / (eps_in * a)


def kirkwood_central(radius, q=1.0, eps_in=4.0, eps_out=80.0, kappa=0.125):
    """Single charge at the centre: Born energy with ionic screening."""
    return COULOMB_KCAL / 2.0 * q * q / radius * (1.0 / (eps_out * (1.0 + kappa * radius)) - 1.0 / eps_in)


def sphere_eigenvalues(l: int, a: float, kappa: float):
    """Eigenvalues of V, K (= T) and D on the sphere of radius a for degree l."""
    if kappa == 0.0:
        return {"V": a / (2 * l + 1), "K": -1.0 / (2.0 * (2 * l + 1)),
                "D": l * (l + 1.0) / ((2 * l + 1) * a)}
    x = kappa * a
    i, k = spherical_in(l, x), spherical_kn(l, x)
    di, dk = spherical_in(l, x, derivative=True), spherical_kn(l, x, derivative=True)
    return {"V": 2.0 * kappa * a * a / math.pi * i * k,
            "K": kappa ** 2 * a * a / math.pi * (di * k + i * dk),
            "D": -2.0 * kappa ** 3 * a * a / math.pi * di * dk}
