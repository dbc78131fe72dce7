"""The synthetic workloads (seeded), in voxel units.

Each ``config_*`` returns a dict with keys ``n`` (3 ints), ``length`` (3 floats,
cell edge in voxel units), ``L`` (flat float64 nodal level set), ``phase``
(flat int32 labels), ``lame`` (nphase x 2 float64), ``loads`` (nload x 6 Mandel
macro strains) and ``info`` (a small dict describing the draw).
"""

import numpy as np

from .materials import lame_from_E_nu
from .shapes import spheres_levelset, rsa_spheres, ellipsoids_levelset, rsa_ellipsoids


def mandel_unit_loads():
    """The six unit macro strains of the Mandel basis (11, 22, 33, 23, 13, 12)."""
    return np.eye(6, dtype=np.float64)


def _pack(n, L, phase, lame, loads, info):
    n = tuple(int(v) for v in n)
    return dict(n=n, length=tuple(float(v) for v in n), L=L, phase=phase,
                lame=np.ascontiguousarray(lame, dtype=np.float64),
                loads=np.ascontiguousarray(loads, dtype=np.float64), info=info)


def config_single_sphere(N=16, radius_frac=0.3, E=(1.0, 10.0), nu=(0.3, 0.25)):
    """One centred sphere of radius 0.3 L on a 16^3 grid, one load e1 (x) e1."""
    n = (N, N, N)
    c = np.array([N / 2.0] * 3)
    L, phase = spheres_levelset(n, [c], [radius_frac * N])
    lam, mu = lame_from_E_nu(np.array(E), np.array(nu))
    lame = np.stack([lam, mu], axis=1)
    loads = np.zeros((1, 6))
    loads[0, 0] = 1.0
    return _pack(n, L, phase, lame, loads, dict(kind="single_sphere", radius=radius_frac * N))


def _spheres(N, count, rmin, rmax, gap, seed, E, nu, target_vf=None, allow_short=False, max_tries=200000):
    rng = np.random.default_rng(seed)
    n = (N, N, N)
    if rmin == rmax:
        sampler = lambda g: rmin * N
    else:
        sampler = lambda g: g.uniform(rmin, rmax) * N
    centers, radii = rsa_spheres(n, count, sampler, gap, rng, target_vf=target_vf, allow_short=allow_short,
                                 max_tries=max_tries)
    L, phase = spheres_levelset(n, centers, radii)
    lam, mu = lame_from_E_nu(np.array(E), np.array(nu))
    lame = np.stack([np.full(len(radii) + 1, lam[1]), np.full(len(radii) + 1, mu[1])], axis=1)
    lame[0] = (lam[0], mu[0])
    vf = float(np.sum(4.0 / 3.0 * np.pi * radii ** 3) / N ** 3)
    return n, L, phase, lame, dict(centers=centers.tolist(), radii=radii.tolist(), vf=vf)


def config_spheres64(seed=2):
    """64^3, ten periodic spheres of radius 0.12 L by RSA with a 2-voxel gap, contrast 100."""
    n, L, phase, lame, info = _spheres(64, 10, 0.12, 0.12, 2.0, seed, (1.0, 100.0), (0.3, 0.2))
    info["kind"] = "spheres64"
    return _pack(n, L, phase, lame, mandel_unit_loads(), info)


def config_spheres128(seed=3, count=40):
    """128^3, forty periodic spheres with radii U[0.06, 0.1] L, 2-voxel gap, contrast 10."""
    n, L, phase, lame, info = _spheres(128, count, 0.06, 0.1, 2.0, seed, (1.0, 10.0), (0.3, 0.25))
    info["kind"] = "spheres128"
    return _pack(n, L, phase, lame, mandel_unit_loads(), info)


def config_uneven_batch(seed=4, count=16, sizes=(32, 48, 64, 96, 128)):
    """Sixteen RVEs of uneven size with 10-30 % sphere volume fraction, contrast 100.

    Random sequential addition with a 2-voxel gap jams below the target on the
    small grids; there the spheres placed within 20000 candidates are kept and
    the achieved volume fraction is recorded (``info["vf"]``).
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        N = int(rng.choice(sizes))
        vf = float(rng.uniform(0.10, 0.30))
        n, L, phase, lame, info = _spheres(N, 0, 0.06, 0.1, 2.0, 40 + i, (1.0, 100.0), (0.3, 0.2),
                                           target_vf=vf, allow_short=True, max_tries=20000)
        info.update(kind="uneven_member", target_vf=vf)
        out.append(_pack(n, L, phase, lame, mandel_unit_loads(), info))
    return out


def config_ellipsoids(N=256, count=200, seed=5, b_frac=0.04301, aspect=3.0, gap=2.0):
    """Randomly oriented prolate spheroids (aspect 3) with per-inclusion Lame pairs.

    Matrix E = 1, nu = 0.35.  Inclusion i: E_i = 20 exp(0.25 z), nu_i =
    clip(0.22 exp(0.1 z'), 0.05, 0.45) with standard normal z, z'.
    """
    rng = np.random.default_rng(seed)
    n = (N, N, N)
    b = b_frac * N
    axes = np.array([aspect * b, b, b])
    centers, rots = rsa_ellipsoids(n, count, axes, gap, rng)
    L, phase = ellipsoids_levelset(n, centers, [axes] * count, rots)
    z1 = rng.standard_normal(count)
    z2 = rng.standard_normal(count)
    E = np.concatenate([[1.0], 20.0 * np.exp(0.25 * z1)])
    nu = np.concatenate([[0.35], np.clip(0.22 * np.exp(0.1 * z2), 0.05, 0.45)])
    lam, mu = lame_from_E_nu(E, nu)
    lame = np.stack([lam, mu], axis=1)
    vf = float(count * 4.0 / 3.0 * np.pi * np.prod(axes) / N ** 3)
    info = dict(kind="ellipsoids", axes=axes.tolist(), vf=vf)
    return _pack(n, L, phase, lame, mandel_unit_loads(), info)
