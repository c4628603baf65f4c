"""Closed-form Laplace potentials of a flat triangle and a tanh-sinh outer
quadrature, for pinning the oracle's singular (Sauter-Schwab) quadrature
against integrals computed a different way.

For a flat triangle S with unit normal n and a point x with projection xp on
the plane of S, h = (x - xp).n, rho = y - xp, R = |x - y| (y in S):
  I0   = int_S 1/R dS          (uniform single layer)
  Irho = int_S rho/R dS        (linear single layer, in-plane vector)
  S3   = int_S h/R^3 dS        (uniform double layer: the signed solid angle)
  Jrho = int_S rho/R^3 dS      (in-plane vector)
from the edge integrals of the surface gradient theorem (D. R. Wilton et al.,
IEEE Trans. Antennas Propag. 32 (1984) 276; R. D. Graglia, ibid. 41 (1993)
1448) and the solid angle of a triangle (A. van Oosterom and J. Strackee,
IEEE Trans. Biomed. Eng. 30 (1983) 125).  A P1 hat is affine, so
lambda_l(y) = lambda_l(xp) + grad lambda_l . rho, and
  int_S lambda_l(y) / R dS            = lambda_l(xp) I0 + grad lambda_l . Irho,
  int_S lambda_l(y) (x - y).n / R^3 dS = lambda_l(xp) S3 + h grad lambda_l . Jrho.
The outer integral over the test triangle uses a tanh-sinh rule on the unit
square mapped onto the triangle, so the derivative singularities of the
inner potential at a shared edge or vertex sit on the square's boundary,
where that rule converges exponentially; no Sauter-Schwab map is involved.
"""
from __future__ import annotations

import numpy as np


def _edge_log(sp, sm, Rp, Rm, R0sq):
    """int_edge dl / R from the foot parameter sm to sp, stable for either sign."""
    def L(s, R):
        return np.where(s >= 0, R + s, R0sq / np.maximum(R - s, 1e-300))
    return np.log(L(sp, Rp) / L(sm, Rm))


def potentials(P, x):
    """I0, Irho (k x 3), S3, Jrho (k x 3), h, xp for points x (k x 3) and the
    triangle with vertices P (3 x 3, counter-clockwise about its normal)."""
    P = np.asarray(P, float)
    x = np.atleast_2d(np.asarray(x, float))
    cr = np.cross(P[1] - P[0], P[2] - P[0])
    n = cr / np.linalg.norm(cr)
    h = (x - P[0]) @ n
    xp = x - h[:, None] * n
    ah = np.abs(h)
    I0 = np.zeros(len(x))
    Irho = np.zeros((len(x), 3))
    Jrho = np.zeros((len(x), 3))
    for i in range(3):
        a, b = P[i], P[(i + 1) % 3]
        e = (b - a) / np.linalg.norm(b - a)
        u = np.cross(e, n)                   # outward in-plane normal of the edge
        t = (a - xp) @ u                     # signed distance of xp to the edge line
        sm = (a - xp) @ e
        sp = (b - xp) @ e
        R0sq = t * t + h * h
        Rm = np.linalg.norm(x - a, axis=1)
        Rp = np.linalg.norm(x - b, axis=1)
        f = _edge_log(sp, sm, Rp, Rm, R0sq)
        beta = (np.arctan2(t * sp, R0sq + ah * Rp) - np.arctan2(t * sm, R0sq + ah * Rm))
        I0 += t * f - ah * beta
        Irho += np.outer(0.5 * (R0sq * f + sp * Rp - sm * Rm), u)
        Jrho -= np.outer(f, u)
    A, B, C = P[0] - x, P[1] - x, P[2] - x
    la, lb, lc = (np.linalg.norm(v, axis=1) for v in (A, B, C))
    num = np.einsum("ij,ij->i", A, np.cross(B, C))
    den = (la * lb * lc + np.einsum("ij,ij->i", A, B) * lc + np.einsum("ij,ij->i", A, C) * lb
           + np.einsum("ij,ij->i", B, C) * la)
    S3 = -2.0 * np.arctan2(num, den)
    # a point in the plane of S: (x - y).n = 0 for every y, so the double
    # layer vanishes (arctan2 would return the one-sided limit +-2 pi inside S)
    S3 = np.where(ah <= 1e-14 * np.linalg.norm(P[1] - P[0]), 0.0, S3)
    return I0, Irho, S3, Jrho, h, xp


def hat_affine(P):
    """lambda_l(z) = c_l + g_l . z for the three hats of the triangle P."""
    P = np.asarray(P, float)
    cr = np.cross(P[1] - P[0], P[2] - P[0])
    two_area = np.linalg.norm(cr)
    n = cr / two_area
    g = np.array([np.cross(n, P[(l + 2) % 3] - P[(l + 1) % 3]) / two_area for l in range(3)])
    c = np.array([1.0 - g[l] @ P[l] for l in range(3)])
    return c, g


def inner_laplace(P, x):
    """(Vin, Kin), each k x 3: int_S lambda_l(y) G(x,y) dS and
    int_S lambda_l(y) dG/dn_y(x,y) dS with G = 1/(4 pi R)."""
    I0, Irho, S3, Jrho, h, xp = potentials(P, x)
    c, g = hat_affine(P)
    lam = c[None, :] + xp @ g.T
    Vin = lam * I0[:, None] + Irho @ g.T
    Kin = lam * S3[:, None] + h[:, None] * (Jrho @ g.T)
    return Vin / (4 * np.pi), Kin / (4 * np.pi)


def _tanh_sinh01(step):
    """Tanh-sinh (double exponential) rule on [0, 1]: points z, 1 - z and
    weights; exponentially convergent for integrands with endpoint
    singularities of log or power type (Takahasi and Mori 1974)."""
    k = np.arange(-int(3.4 / step), int(3.4 / step) + 1)
    t = k * step
    s = 0.5 * np.pi * np.sinh(t)
    z = 1.0 / (1.0 + np.exp(-2.0 * s))          # (1 + tanh s) / 2
    zc = 1.0 / (1.0 + np.exp(2.0 * s))          # 1 - z without cancellation
    w = step * 0.5 * np.pi * np.cosh(t) / (2.0 * np.cosh(s) ** 2)
    keep = (np.minimum(z, zc) > 1e-13)   # the dropped tails carry ~1e-13 of the mass
    return z[keep], zc[keep], w[keep]


def outer_integral(Q, f, step=1.0 / 24):
    """int_Q lambda_k(x) f(x) dx (3 x m) for the test triangle Q, with f
    mapping points (k x 3) to k x m values.  Q is mapped from the unit square
    by x = Q0 + u (Q1 - Q0) + u v (Q2 - Q1) (Jacobian 2|Q| u); every edge and
    vertex of Q lies on the square's boundary, where the tanh-sinh rule in
    both variables absorbs the derivative singularities of f."""
    Q = np.asarray(Q, float)
    z, zc, w = _tanh_sinh01(step)
    u, v = (a.ravel() for a in np.meshgrid(z, z, indexing="ij"))
    uc, vc = (a.ravel() for a in np.meshgrid(zc, zc, indexing="ij"))
    wt = np.outer(w, w).ravel()
    # hats of Q0, Q1, Q2 at the mapped point, complements from the rule (no 1 - z cancellation)
    lam = np.stack([uc, u * vc, u * v], axis=1)
    pts = lam @ Q
    area = 0.5 * np.linalg.norm(np.cross(Q[1] - Q[0], Q[2] - Q[0]))
    wt = wt * 2.0 * area * u
    return np.einsum("p,pk,pm->km", wt, lam, f(pts))


def laplace_blocks(Ptest, Ptrial, step=1.0 / 24):
    """3 x 3 Galerkin blocks V[k, l] = int int lambda_k G lambda_l and
    K[k, l] = int int lambda_k dG/dn_y lambda_l of the Laplace kernel for the
    test triangle Ptest and the trial triangle Ptrial (vertex rows in the
    triangles' stored order)."""
    def f(x):
        Vin, Kin = inner_laplace(Ptrial, x)
        return np.concatenate([Vin, Kin], axis=1)
    out = outer_integral(Ptest, f, step=step)
    return out[:, :3], out[:, 3:]
