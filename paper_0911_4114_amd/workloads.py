"""Seeded synthetic inputs shaped like the paper's workloads (points in a cube, Section 3.5.3) and
like the surface scatterers the method targets (sphere, ellipsoid). Shared by the tests, the
benchmark and the CPU baseline; holds none of the method's arithmetic.

Generator: numpy PCG64 (``numpy.random.default_rng(seed)``); complex values are drawn re then
im, each ``standard_normal``.
"""
import numpy as np


def cube_points(n, seed=0):
    """n points uniform in [0, 1)^3."""
    return np.random.default_rng(seed).random((n, 3))


def sphere_points(n, seed=0):
    """n points uniform on the unit sphere: g ~ N(0, I_3), x = g / |g|."""
    g = np.random.default_rng(seed).standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def ellipsoid_points(n, axes=(1.0, 0.6, 0.3), seed=0):
    """n points uniform in area on the ellipsoid with the given semi-axes: u uniform on the unit
    sphere, accepted with probability proportional to the area element of the map
    u -> (a u1, b u2, c u3), i.e. sqrt((b c u1)^2 + (a c u2)^2 + (a b u3)^2) / (a b)."""
    a, b, c = axes
    rng = np.random.default_rng(seed)
    out = []
    have = 0
    pmax = max(a * b, b * c, a * c)
    while have < n:
        m = 2 * (n - have) + 1024
        g = rng.standard_normal((m, 3))
        u = g / np.linalg.norm(g, axis=1, keepdims=True)
        dens = np.sqrt((b * c * u[:, 0]) ** 2 + (a * c * u[:, 1]) ** 2 + (a * b * u[:, 2]) ** 2)
        keep = rng.random(m) < dens / pmax
        x = u[keep] * np.array([a, b, c])
        out.append(x)
        have += len(x)
    return np.concatenate(out)[:n]


def complex_normal(n, seed=1, nrhs=None):
    """Complex N(0, 1) per component: re then im, each standard_normal. Shape [n] or [nrhs, n]."""
    rng = np.random.default_rng(seed)
    shape = (n,) if nrhs is None else (nrhs, n)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return re + 1j * im


def plane_wave_charges(x, kappa, nrhs, seed=2):
    """q_j^(m) = e^{i kappa d_m . x_j} for nrhs random unit directions d_m (incident plane waves)."""
    g = np.random.default_rng(seed).standard_normal((nrhs, 3))
    d = g / np.linalg.norm(g, axis=1, keepdims=True)
    return np.exp(1j * kappa * (d @ np.asarray(x).T))


def subset(n, m, seed=7):
    """m distinct target indices out of n, sorted (for direct-sum checks at large n)."""
    if m >= n:
        return np.arange(n)
    return np.sort(np.random.default_rng(seed).choice(n, size=m, replace=False))
