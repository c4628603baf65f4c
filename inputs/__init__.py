"""Seeded synthetic workloads: closed triangle meshes and point-charge sets.

This module is shared by the FP64 oracle and by the GPU library's tests and
benchmark.  It only builds geometry and draws random numbers; it performs none
of the boundary-element arithmetic (no kernels, quadrature, operators or
solves), so that the oracle and the GPU path stay independent.

The paper's own workloads are solvent-excluded molecular surfaces meshed at
4-10 vertices per square angstrom with point charges at atom centres (Results
section).  Those meshes and charge files are not available, so every workload
here is synthetic with the same shape statistics:

* ``icosphere``      - frequency-n class-I geodesic sphere, T = 20 n^2 flat
                       triangles, V = 10 n^2 + 2 vertices, counter-clockwise
                       seen from outside (outward normals).
* ``star_surface``   - the icosphere's directions mapped radially to
                       r(theta, phi) = R (1 + 0.15 f), f a random sum of real
                       spherical harmonics of degree <= 6 with coefficients
                       N(0,1)/(l+1): a smooth, star-shaped, protein-like blob.
* ``bipyramid``      - two cones over a regular n-gon: two apexes of valence n
                       and 2n skinny triangles (apex angle 2 pi / n), a
                       stress case for vertex valence and aspect ratio.
* ``charges_*``      - charges strictly inside the surface.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Mesh", "Charges", "icosphere", "star_surface", "charges_ball",
    "charges_in_star", "config_kirkwood", "config_sphere", "config_star",
    "config_sphere_multi", "serving_trace", "bipyramid",
]


@dataclass
class Mesh:
    xyz: np.ndarray          # (V, 3) float64, angstrom
    tri: np.ndarray          # (T, 3) int32, 0-based, counter-clockwise from outside
    meta: dict = field(default_factory=dict)

    @property
    def n_vertices(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_triangles(self) -> int:
        return int(self.tri.shape[0])


@dataclass
class Charges:
    xyz: np.ndarray          # (N, 3) float64, angstrom
    q: np.ndarray            # (N,) float64, elementary charges
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.q.shape[0])


def _icosahedron():
    g = (1.0 + math.sqrt(5.0)) / 2.0
    v = []
    for a in (-1.0, 1.0):
        for b in (-g, g):
            v.append((0.0, a, b))
            v.append((a, b, 0.0))
            v.append((b, 0.0, a))
    v = np.array(v, dtype=np.float64)
    # faces = triples of mutually adjacent vertices (edge length 2)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    adj = np.abs(d - 2.0) < 1e-9
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            if not adj[i, j]:
                continue
            for k in range(j + 1, 12):
                if adj[i, k] and adj[j, k]:
                    a, b, c = v[i], v[j], v[k]
                    nrm = np.cross(b - a, c - a)
                    if np.dot(nrm, a + b + c) > 0:
                        faces.append((i, j, k))
                    else:
                        faces.append((i, k, j))
    assert len(faces) == 20
    return v, faces


def icosphere(freq: int, radius: float = 1.0) -> Mesh:
    """Frequency-``freq`` class-I geodesic icosphere of the given radius (cached per frequency)."""
    xyz, tri = _unit_icosphere(int(freq))
    return Mesh(xyz * radius, tri.copy(), {"kind": "icosphere", "freq": int(freq), "radius": float(radius)})


_ICO_CACHE: dict = {}


def _unit_icosphere(freq: int):
    if freq not in _ICO_CACHE:
        m = _build_icosphere(freq)
        m.xyz.setflags(write=False)
        _ICO_CACHE[freq] = (m.xyz, m.tri)
    return _ICO_CACHE[freq]


def _build_icosphere(freq: int, radius: float = 1.0) -> Mesh:
    """Frequency-``freq`` class-I geodesic icosphere of the given radius.

    Every icosahedron face (A, B, C) is split into freq^2 triangles on the
    barycentric lattice; lattice points are projected radially onto the
    sphere.  Points shared between faces are identified exactly by their
    integer barycentric weights on the icosahedron vertices.
    """
    if freq < 1:
        raise ValueError("freq must be >= 1")
    base, faces = _icosahedron()
    n = int(freq)
    key_to_id: dict = {}
    pts: list = []
    tris: list = []

    def vid(fa, i, j):
        a, b, c = fa
        w = {}
        for vtx, wt in ((a, n - i - j), (b, i), (c, j)):
            if wt:
                w[vtx] = w.get(vtx, 0) + wt
        key = tuple(sorted(w.items()))
        got = key_to_id.get(key)
        if got is None:
            p = sum(base[vtx] * wt for vtx, wt in key) / n
            got = len(pts)
            key_to_id[key] = got
            pts.append(p)
        return got

    for fa in faces:
        for i in range(n):
            for j in range(n - i):
                v0 = vid(fa, i, j)
                v1 = vid(fa, i + 1, j)
                v2 = vid(fa, i, j + 1)
                tris.append((v0, v1, v2))
                if i + j < n - 1:
                    v3 = vid(fa, i + 1, j + 1)
                    tris.append((v1, v3, v2))
    xyz = np.array(pts, dtype=np.float64)
    xyz *= radius / np.linalg.norm(xyz, axis=1, keepdims=True)
    tri = np.array(tris, dtype=np.int32)
    assert xyz.shape[0] == 10 * n * n + 2 and tri.shape[0] == 20 * n * n
    return Mesh(xyz, tri, {"kind": "icosphere", "freq": n, "radius": float(radius)})


class StarShape:
    """Radial function r(u) = R (1 + amp * sum_lm c_lm Y_lm(u)) for unit u."""

    def __init__(self, seed: int, base_radius: float = 18.0, amp: float = 0.15, lmax: int = 6):
        self.base_radius = float(base_radius)
        self.amp = float(amp)
        self.lmax = int(lmax)
        sub = 0
        while True:
            rng = np.random.default_rng([int(seed), sub])
            coef = []
            for l in range(self.lmax + 1):
                for m in range(-l, l + 1):
                    coef.append((l, m, rng.standard_normal() / (l + 1)))
            self.coef = coef
            # reject shapes whose radius drops below half the base radius
            probe = icosphere(16).xyz
            if np.min(1.0 + self.amp * self._f(probe)) >= 0.5:
                break
            sub += 1
        self.sub_seed = sub

    def _f(self, u: np.ndarray) -> np.ndarray:
        from scipy.special import sph_harm_y
        u = u / np.linalg.norm(u, axis=1, keepdims=True)
        polar = np.arccos(np.clip(u[:, 2], -1.0, 1.0))
        azim = np.arctan2(u[:, 1], u[:, 0])
        coef = {(l, m): c for l, m, c in self.coef}
        f = np.zeros(u.shape[0])
        for l in range(self.lmax + 1):
            for m in range(0, l + 1):
                y = sph_harm_y(l, m, polar, azim)   # one evaluation serves +m and -m
                if m == 0:
                    f += coef[(l, 0)] * np.real(y)
                else:
                    s = math.sqrt(2.0) * (-1) ** m
                    f += coef[(l, m)] * s * np.real(y) + coef[(l, -m)] * s * np.imag(y)
        return f

    def radius(self, u: np.ndarray) -> np.ndarray:
        return self.base_radius * (1.0 + self.amp * self._f(u))


def bipyramid(n: int, radius: float = 1.0, height: float = 1.0) -> Mesh:
    """Closed bipyramid over a regular n-gon of the given radius in the plane
    z = 0, apexes at z = +-height; counter-clockwise seen from outside."""
    ang = 2.0 * math.pi * np.arange(n) / n
    ring = np.stack([radius * np.cos(ang), radius * np.sin(ang), np.zeros(n)], axis=1)
    xyz = np.vstack([ring, [[0.0, 0.0, height], [0.0, 0.0, -height]]])
    tri = []
    for i in range(n):
        j = (i + 1) % n
        tri += [[i, j, n], [j, i, n + 1]]
    return Mesh(xyz, np.array(tri, dtype=np.int32), {"kind": "bipyramid", "n": int(n)})


def star_surface(seed: int, freq: int, base_radius: float = 18.0) -> tuple:
    """Star-shaped molecule-like surface; returns (Mesh, StarShape)."""
    shape = StarShape(seed, base_radius)
    m = icosphere(freq, 1.0)
    r = shape.radius(m.xyz)
    xyz = m.xyz * r[:, None]
    return Mesh(xyz, m.tri, {"kind": "star", "seed": int(seed), "freq": int(freq),
                             "base_radius": float(base_radius)}), shape


def charges_ball(seed: int, n: int, radius: float) -> Charges:
    """n charges uniform in the ball |x| < radius, values U[-1, 1] e."""
    rng = np.random.default_rng(int(seed))
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = radius * rng.random(n) ** (1.0 / 3.0)
    q = rng.uniform(-1.0, 1.0, n)
    return Charges(d * r[:, None], q, {"kind": "ball", "seed": int(seed), "radius": float(radius)})


def charges_in_star(seed: int, n: int, shape: StarShape, frac: float = 0.8,
                    values: str = "normal", sigma: float = 0.4) -> Charges:
    """n charges uniform in {|x| < frac * r(x/|x|)}; values N(0, sigma) or U[-1, 1]."""
    rng = np.random.default_rng(int(seed))
    rmax = 1.05 * frac * float(np.max(shape.radius(icosphere(16).xyz)))
    out = []
    while sum(len(o) for o in out) < n:
        d = rng.standard_normal((16 * n, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        r = rmax * rng.random(16 * n) ** (1.0 / 3.0)
        keep = r < frac * shape.radius(d)
        out.append(d[keep] * r[keep, None])
    xyz = np.concatenate(out)[:n]
    if values == "normal":
        q = rng.normal(0.0, sigma, n)
    else:
        q = rng.uniform(-1.0, 1.0, n)
    return Charges(xyz, q, {"kind": "star", "seed": int(seed)})


# ---------------------------------------------------------------- workloads
PHYS = {"eps_in": 4.0, "eps_out": 80.0, "kappa": 0.125}


def config_kirkwood(freq: int = 4, radius: float = 2.0):
    """Sphere with one +1 e charge at its centre (radius 2 A, 320 triangles at freq 4)."""
    mesh = icosphere(freq, radius)
    ch = Charges(np.zeros((1, 3)), np.ones(1), {"kind": "centre"})
    return mesh, ch


def config_sphere(freq: int = 32, radius: float = 10.0, n_charges: int = 50,
                  charge_radius: float = 8.0, seed: int = 2):
    """Sphere (radius 10 A, 20480 triangles at freq 32) with 50 charges in r < 8 A."""
    return icosphere(freq, radius), charges_ball(seed, n_charges, charge_radius)


def config_star(freq: int = 64, seed: int = 3, n_charges: int = 2000, base_radius: float = 18.0):
    """Star surface (81920 triangles at freq 64) with 2000 N(0, 0.4) charges inside 0.8 r."""
    mesh, shape = star_surface(seed, freq, base_radius)
    return mesh, charges_in_star(seed + 1000, n_charges, shape)


def config_star_large(freq: int = 150, seed: int = 7, n_charges: int = 4000, base_radius: float = 36.0):
    """Star surface at the size of the paper's largest molecule: 450000 triangles /
    225002 vertices at freq 150 (1igt has 226312 vertices), 4000 charges."""
    mesh, shape = star_surface(seed, freq, base_radius)
    return mesh, charges_in_star(seed + 1000, n_charges, shape)


def config_sphere_multi(freq: int = 64, radius: float = 10.0, n_sets: int = 16,
                        n_charges: int = 50, seed0: int = 40):
    """Sphere (40962 vertices at freq 64) with n_sets independent charge sets."""
    mesh = icosphere(freq, radius)
    return mesh, [charges_ball(seed0 + k, n_charges, 8.0) for k in range(n_sets)]


def serving_trace(seed: int = 5, n_requests: int = 512, rate_hz: float = 20.0,
                  fmin: int = 8, fmax: int = 64):
    """Poisson-arrival stream of star-surface solve requests.

    Frequency n = round(exp(U[ln fmin, ln fmax])) so T = 20 n^2 is log-uniform
    in [1280, 81920]; base radius scales with sqrt(T) so the vertex density is
    constant; charge count grows from 50 to 4000 with T; formulation is a fair
    coin between direct (0) and Juffer (1).  Returns a list of dicts; meshes
    are built lazily by ``build_request``.
    """
    rng = np.random.default_rng(int(seed))
    t = 0.0
    reqs = []
    for k in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        f = int(round(math.exp(rng.uniform(math.log(fmin), math.log(fmax)))))
        T = 20 * f * f
        nq = int(round(50.0 * (T / 1280.0) ** (math.log(80.0) / math.log(64.0))))
        reqs.append({"id": k, "arrival_s": t, "freq": f, "n_triangles": T,
                     "n_charges": nq, "formulation": int(rng.integers(0, 2)),
                     "seed": int(rng.integers(0, 2**31 - 1))})
    return reqs


def build_request(req: dict):
    base = 18.0 * math.sqrt(req["n_triangles"] / 81920.0)
    mesh, shape = star_surface(req["seed"], req["freq"], base)
    ch = charges_in_star(req["seed"] + 1, req["n_charges"], shape, values="uniform")
    return mesh, ch
