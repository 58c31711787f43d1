"""Seeded initial spin textures (NumPy PCG64).

Every function returns a float64 array of shape (3, N) in the site order
``i = a + Na*(b + Nb*(c + Nc*beta))``; every vector has unit length.
Nothing here evaluates the Hamiltonian or advances dynamics.
"""

from __future__ import annotations

import math

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _normalise(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v, axis=0, keepdims=True)


def site_coords(geometry):
    """Integer cell coordinates (a, b, c, beta) of every site, each shape (N,)."""
    na, nb, nc = geometry.n_cells
    nbasis = geometry.n_basis
    idx = np.arange(na * nb * nc * nbasis)
    a = idx % na
    b = (idx // na) % nb
    c = (idx // (na * nb)) % nc
    beta = idx // (na * nb * nc)
    return a, b, c, beta


def site_positions(geometry) -> np.ndarray:
    """Cartesian positions (3, N) in units of the lattice constant."""
    a, b, c, beta = site_coords(geometry)
    br = np.asarray(geometry.bravais, dtype=np.float64)
    bs = np.asarray(geometry.basis, dtype=np.float64)
    return (a[None, :] * br[0][:, None] + b[None, :] * br[1][:, None]
            + c[None, :] * br[2][:, None] + bs[beta].T)


def uniform_sphere(n: int, seed: int) -> np.ndarray:
    """n spins uniform on the unit sphere: normalised 3D standard normals."""
    g = _rng(seed).standard_normal((3, n))
    return _normalise(g)


def ferromagnet(n: int, direction=(0.0, 0.0, 1.0)) -> np.ndarray:
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    return np.repeat(d[:, None], n, axis=1).copy()


def spin_spiral(geometry, q, e1=(1.0, 0.0, 0.0), e2=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Flat spiral n = cos(q.r) e1 + sin(q.r) e2 (r in lattice-constant units)."""
    r = site_positions(geometry)
    phase = np.asarray(q, dtype=np.float64) @ r
    e1 = np.asarray(e1, dtype=np.float64)[:, None]
    e2 = np.asarray(e2, dtype=np.float64)[:, None]
    return _normalise(np.cos(phase)[None, :] * e1 + np.sin(phase)[None, :] * e2)


def _tilt(n: np.ndarray, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """Rotate each spin by a N(0, sigma) angle about a uniform axis tangent to it."""
    if sigma <= 0.0:
        return n
    N = n.shape[1]
    ref = rng.standard_normal((3, N))
    t = ref - np.sum(ref * n, axis=0, keepdims=True) * n
    t = _normalise(t)
    ang = rng.normal(0.0, sigma, size=N)
    return _normalise(n * np.cos(ang)[None, :] + t * np.sin(ang)[None, :])


def conical_helix(geometry, periods: int = 2, polar_deg: float = 60.0,
                  noise_rad: float = 0.05, seed: int = 0) -> np.ndarray:
    """Conical helix with wave vector along z (commensurate: ``periods`` turns
    over the z extent), cone half-angle ``polar_deg``, plus Gaussian tilt noise."""
    a, b, c, beta = site_coords(geometry)
    nc = geometry.n_cells[2]
    q = 2.0 * math.pi * periods / nc
    th = math.radians(polar_deg)
    phase = q * c
    n = np.stack([math.sin(th) * np.cos(phase), math.sin(th) * np.sin(phase),
                  np.full(phase.shape, math.cos(th))])
    return _tilt(_normalise(n), noise_rad, _rng(seed))


def skyrmion_ansatz(geometry, radius: float = 5.0, center=None, helicity: float = 0.0,
                    width: float = 2.0, core_down: bool = True, noise_rad: float = 0.0,
                    seed: int = 0) -> np.ndarray:
    """Isolated skyrmion/bubble in a +z background: polar angle
    theta(rho) = pi - (2 arctan(exp((rho - R)/w))) ... mapped so the core points
    -z and the background +z; in-plane angle = azimuth + helicity."""
    r = site_positions(geometry)
    if center is None:
        center = (r[0].max() / 2.0, r[1].max() / 2.0)
    dx = r[0] - center[0]
    dy = r[1] - center[1]
    rho = np.hypot(dx, dy)
    theta = 2.0 * np.arctan(np.exp(-(rho - radius) / width))  # pi at core, 0 far away
    if not core_down:
        theta = math.pi - theta
    phi = np.arctan2(dy, dx) + helicity
    n = np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])
    return _tilt(_normalise(n), noise_rad, _rng(seed))


def geodesic_chain(a: np.ndarray, b: np.ndarray, n_images: int,
                   fallback_axis=(0.0, 1.0, 0.0)) -> np.ndarray:
    """Initial GNEB chain: per spin, great-circle interpolation from a to b at
    n_images equally spaced parameters (endpoints included).  Antiparallel
    spins rotate about fallback_axis (projected perpendicular to the spin).
    Returns (n_images, 3, N)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    ax = np.cross(a.T, b.T).T
    s = np.linalg.norm(ax, axis=0)
    c = np.sum(a * b, axis=0)
    theta = np.arctan2(s, c)
    fb = np.asarray(fallback_axis, dtype=np.float64)[:, None]
    fb = fb - np.sum(fb * a, axis=0, keepdims=True) * a
    small = s < 1e-12
    axis = np.where(small[None, :], fb, ax)
    axis = axis / np.linalg.norm(axis, axis=0, keepdims=True)
    perp = np.cross(axis.T, a.T).T   # unit vector in the rotation plane, 90 deg ahead of a
    out = np.empty((n_images,) + a.shape)
    for k in range(n_images):
        t = k / (n_images - 1)
        out[k] = np.cos(t * theta)[None, :] * a + np.sin(t * theta)[None, :] * perp
    out[-1] = b
    return _normalise_chain(out)


def _normalise_chain(c: np.ndarray) -> np.ndarray:
    return c / np.linalg.norm(c, axis=1, keepdims=True)


def domain_walls(geometry, n_walls: int = 1, seed: int = 0, bloch: bool = True,
                 width_range=(2.0, 8.0)) -> np.ndarray:
    """Parallel tanh domain walls at random positions/orientation/width."""
    rng = _rng(seed)
    r = site_positions(geometry)
    ang = rng.uniform(0.0, 2.0 * math.pi)
    ex = np.array([math.cos(ang), math.sin(ang)])
    s = ex[0] * r[0] + ex[1] * r[1]
    span = (s.min(), s.max())
    pos = np.sort(rng.uniform(span[0], span[1], size=n_walls))
    w = rng.uniform(*width_range)
    theta = np.zeros_like(s)
    for k, p in enumerate(pos):
        theta += 2.0 * np.arctan(np.exp((s - p) / w))  # each wall adds pi
    if bloch:
        inplane = np.stack([-ex[1] * np.ones_like(s), ex[0] * np.ones_like(s)])
    else:
        inplane = np.stack([ex[0] * np.ones_like(s), ex[1] * np.ones_like(s)])
    n = np.stack([np.sin(theta) * inplane[0], np.sin(theta) * inplane[1], np.cos(theta)])
    return _normalise(n)
