"""Grid helpers: node coordinates and periodic differences (voxel units)."""

import numpy as np


def flat_shape(n):
    """numpy shape (n2, n1, n0) whose C-order flattening gives i + n0*(j + n1*k)."""
    return (int(n[2]), int(n[1]), int(n[0]))


def node_coords(n, h=1.0):
    """Coordinates of every node as three flat arrays (x fastest)."""
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    return (i.ravel() * h).astype(np.float64), (j.ravel() * h).astype(np.float64), (k.ravel() * h).astype(np.float64)


def periodic_delta(a, b, period):
    """Signed difference a - b wrapped into [-period/2, period/2)."""
    d = a - b
    return d - period * np.floor(d / period + 0.5)
