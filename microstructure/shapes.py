"""Level sets (signed distance, voxel units) and phase labels of simple shapes.

Every function returns ``(L, phase)`` as flat float64 / int32 arrays over the
nodes, or helpers to build them.  Inclusions get L < 0 and label >= 1; the
matrix gets L > 0 and label 0.
"""

import numpy as np

from .grid import node_coords, periodic_delta


def spheres_levelset(n, centers, radii):
    """Signed distance to the nearest of several periodic spheres.

    L(x) = min_i(|x - c_i|_periodic - r_i); the label is 1 + argmin where L < 0.
    """
    x, y, z = node_coords(n)
    best = np.full(x.shape, np.inf)
    lab = np.zeros(x.shape, dtype=np.int32)
    for idx, (c, r) in enumerate(zip(centers, radii)):
        dx = periodic_delta(x, c[0], n[0])
        dy = periodic_delta(y, c[1], n[1])
        dz = periodic_delta(z, c[2], n[2])
        d = np.sqrt(dx * dx + dy * dy + dz * dz) - r
        better = d < best
        best = np.where(better, d, best)
        lab = np.where(better, idx + 1, lab)
    phase = np.where(best < 0.0, lab, 0).astype(np.int32)
    return best.astype(np.float64), phase


def rsa_spheres(n, count, radius_sampler, gap, rng, max_tries=200000, target_vf=None, allow_short=False):
    """Random sequential addition of non-overlapping periodic spheres.

    Centres are uniform in the cell; a candidate is accepted when its surface
    keeps at least ``gap`` voxels from every accepted sphere.  Stops after
    ``count`` spheres, or, when ``target_vf`` is given, once the analytic volume
    fraction reaches it.  With ``allow_short`` the spheres placed within
    ``max_tries`` candidates are returned when the target is out of reach
    (random sequential addition jams well below dense packing).
    """
    n = np.asarray(n, dtype=np.float64)
    vol = float(np.prod(n))
    centers, radii = [], []
    tries = 0
    vf = 0.0
    while True:
        if target_vf is None and len(centers) >= count:
            break
        if target_vf is not None and vf >= target_vf:
            break
        if tries >= max_tries:
            if allow_short:
                break
            raise RuntimeError("RSA did not place the requested inclusions")
        tries += 1
        r = float(radius_sampler(rng))
        c = rng.uniform(0.0, 1.0, 3) * n
        if centers:
            d = periodic_delta(c[None, :], np.asarray(centers), n[None, :])
            if np.any(np.sqrt(np.sum(d * d, axis=1)) < r + np.asarray(radii) + gap):
                continue
        centers.append(c)
        radii.append(r)
        vf += 4.0 / 3.0 * np.pi * r ** 3 / vol
    return np.array(centers), np.array(radii)


def laminate_levelset(n, m, s1, s2):
    """Periodic rank-one laminate with integer normal direction ``m``.

    The phase coordinate s = m . x (mod n0, n0 = n1 = n2 required) places layer
    1 at s in [s1, s2).  L is the exact signed distance to the nearest plane of
    the family (negative in layer 1); layer 1 gets label 1.
    """
    assert n[0] == n[1] == n[2]
    N = float(n[0])
    m = np.asarray(m, dtype=np.float64)
    norm = np.sqrt(np.sum(m * m))
    x, y, z = node_coords(n)
    s = m[0] * x + m[1] * y + m[2] * z
    w = float(s2 - s1)
    t = np.mod(s - s1, N)
    inside = t < w
    d_in = np.minimum(t, w - t)
    d_out = np.minimum(t - w, N - t)
    L = np.where(inside, -d_in, d_out) / norm
    phase = np.where(inside, 1, 0).astype(np.int32)
    return L, phase


def coated_sphere_levelset(n, center, r_inclusion, r_coating):
    """Coated sphere: matrix (label 0, L > 0), coating (1, L < 0), core (2, L > 0).

    The level set changes sign at both spherical interfaces and is the signed
    distance to the nearer one.
    """
    x, y, z = node_coords(n)
    dx = periodic_delta(x, center[0], n[0])
    dy = periodic_delta(y, center[1], n[1])
    dz = periodic_delta(z, center[2], n[2])
    r = np.sqrt(dx * dx + dy * dy + dz * dz)
    L = np.where(r >= r_coating, r - r_coating,
                 np.where(r >= r_inclusion, -np.minimum(r_coating - r, r - r_inclusion), r_inclusion - r))
    phase = np.where(r >= r_coating, 0, np.where(r >= r_inclusion, 1, 2)).astype(np.int32)
    return L.astype(np.float64), phase


def _ellipsoid_distance(p, axes):
    """Signed distance from points p (m x 3, local frame) to an ellipsoid.

    Closest-point root of F(t) = sum (a_i p_i / (t + a_i^2))^2 - 1 found by
    bisection on t in (-min a^2, inf) (Eberly's formulation); negative inside.
    """
    a = np.asarray(axes, dtype=np.float64)
    q = np.abs(p)
    a2 = a * a
    inside = np.sum((q / a) ** 2, axis=1) < 1.0
    lo = np.where(inside, -a2.min() * (1.0 - 1e-15), 0.0)
    hi = np.where(inside, 0.0, np.sqrt(np.sum(q * q, axis=1)) * a.max() + a2.max())
    for _ in range(80):          # the bracket shrinks below double resolution well before
        t = 0.5 * (lo + hi)
        F = np.sum((a[None, :] * q / (t[:, None] + a2[None, :])) ** 2, axis=1) - 1.0
        pos = F > 0.0
        lo = np.where(pos, t, lo)
        hi = np.where(pos, hi, t)
    t = 0.5 * (lo + hi)
    xc = a2[None, :] * q / (t[:, None] + a2[None, :])
    d = np.sqrt(np.sum((xc - q) ** 2, axis=1))
    return np.where(inside, -d, d)


def _periodic_box(n, c, reach):
    """Wrapped index ranges and periodic offsets of the box |x - c| <= reach (per axis)."""
    idx, off = [], []
    for a in range(3):
        lo = int(np.floor(c[a] - reach))
        hi = int(np.ceil(c[a] + reach))
        if hi - lo + 1 >= n[a]:
            lo, hi = 0, n[a] - 1
            pos = np.arange(n[a])
            d = periodic_delta(pos.astype(np.float64), c[a], n[a])
        else:
            pos = np.arange(lo, hi + 1)
            d = pos - c[a]
            pos = np.mod(pos, n[a])
        idx.append(pos)
        off.append(d.astype(np.float64))
    return idx, off


def _box_local(off, R):
    """Local (rotated) coordinates of all box points: array (nz, ny, nx, 3)."""
    dx, dy, dz = off
    g = np.stack(np.broadcast_arrays(dx[None, None, :], dy[None, :, None], dz[:, None, None]), axis=-1)
    return g @ np.asarray(R)


def ellipsoids_levelset(n, centers, axes, rotations, clamp=3.0):
    """Signed distance (clamped to +-clamp) to the nearest of several ellipsoids.

    ``rotations[i]`` maps local to global coordinates.  Only nodes within a
    shell of +-clamp around each surface need the exact distance (root find);
    deeper nodes get -clamp (inside) and farther ones stay at +clamp.
    """
    L3 = np.full((n[2], n[1], n[0]), clamp)
    P3 = np.zeros((n[2], n[1], n[0]), dtype=np.int32)
    for idx, (c, ax, R) in enumerate(zip(centers, axes, rotations)):
        ax = np.asarray(ax, dtype=np.float64)
        reach = float(np.max(ax)) + clamp + 1.0
        (ix, iy, iz), off = _periodic_box(n, c, reach)
        loc = _box_local(off, R)
        q_out = np.sum((loc / (ax + clamp)) ** 2, axis=-1)
        inner = np.maximum(ax - clamp, 1e-6)
        q_in = np.sum((loc / inner) ** 2, axis=-1)
        d = np.full(q_out.shape, clamp)
        deep = (q_in <= 1.0) & np.all(ax > clamp)
        d[deep] = -clamp
        shell = (q_out <= 1.0) & ~deep
        if np.any(shell):
            d[shell] = np.clip(_ellipsoid_distance(loc[shell], ax), -clamp, clamp)
        sub = np.ix_(iz, iy, ix)
        cur = L3[sub]
        better = d < cur
        L3[sub] = np.where(better, d, cur)
        ph = P3[sub]
        P3[sub] = np.where(better & (d < 0.0), idx + 1, np.where(better, 0, ph))
    return L3.ravel().astype(np.float64), P3.ravel().astype(np.int32)


def _random_rotation(rng):
    """Uniformly distributed rotation matrix (from a random unit quaternion)."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, a, b, c = q
    return np.array([
        [1 - 2 * (b * b + c * c), 2 * (a * b - c * w), 2 * (a * c + b * w)],
        [2 * (a * b + c * w), 1 - 2 * (a * a + c * c), 2 * (b * c - a * w)],
        [2 * (a * c - b * w), 2 * (b * c + a * w), 1 - 2 * (a * a + b * b)],
    ])


def rsa_ellipsoids(n, count, axes, gap, rng, max_tries=20000):
    """Random sequential addition of randomly oriented, equal ellipsoids.

    Overlap is tested on the node raster: every candidate's ellipsoid inflated
    by ``gap / 2`` must not cover a node already covered by an accepted one.
    """
    occupied = np.zeros((n[2], n[1], n[0]), dtype=bool)
    ax_inf = np.asarray(axes, dtype=np.float64) + 0.5 * gap
    reach = float(np.max(ax_inf)) + 1.0
    centers, rots = [], []
    tries = 0
    while len(centers) < count:
        if tries >= max_tries:
            raise RuntimeError("ellipsoid RSA did not place the requested inclusions")
        tries += 1
        c = rng.uniform(0.0, 1.0, 3) * np.asarray(n, dtype=np.float64)
        R = _random_rotation(rng)
        if centers:
            # both inflated ellipsoids contain the ball of their smallest axis:
            # closer centres certainly overlap (cheap rejection before the raster test)
            dc = periodic_delta(np.asarray(centers), c[None, :], np.asarray(n, dtype=np.float64)[None, :])
            if np.min(np.sum(dc * dc, axis=1)) < (2.0 * float(np.min(ax_inf))) ** 2:
                continue
        (ix, iy, iz), off = _periodic_box(n, c, reach)
        loc = _box_local(off, R)
        cover = np.sum((loc / ax_inf) ** 2, axis=-1) <= 1.0
        sub = np.ix_(iz, iy, ix)
        occ = occupied[sub]
        if np.any(occ & cover):
            continue
        occupied[sub] = occ | cover
        centers.append(c)
        rots.append(R)
    return np.array(centers), np.array(rots)


def rotation_xyz(deg):
    """Rotation by ``deg`` degrees about x, then about y, then about z (R = Rz Ry Rx)."""
    a = np.deg2rad(deg)
    c, s = np.cos(a), np.sin(a)
    Rx = np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    Ry = np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    Rz = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def cube_levelset(n, center, edge, R=None):
    """Signed distance to one cube (edge length ``edge``, voxel units) centred at
    ``center``, its axes rotated by R (columns: the cube's axes in the cell frame).

    Exact Euclidean distance to the box outside, minus the distance to the
    nearest face inside; periodic images are taken by the nearest-image offset,
    which is exact while the cube and its distance band fit in the cell.
    """
    x, y, z = node_coords(n)
    off = np.stack([periodic_delta(x, center[0], n[0]), periodic_delta(y, center[1], n[1]),
                    periodic_delta(z, center[2], n[2])], axis=-1)
    p = off if R is None else off @ np.asarray(R, dtype=np.float64)      # coordinates in the cube frame
    q = np.abs(p) - 0.5 * edge
    outside = np.sqrt(np.sum(np.maximum(q, 0.0) ** 2, axis=-1))
    inside = np.minimum(np.max(q, axis=-1), 0.0)
    L = (outside + inside).reshape(-1)
    phase = np.where(L < 0.0, 1, 0).astype(np.int32)
    return L.astype(np.float64), phase
