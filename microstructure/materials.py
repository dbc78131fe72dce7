"""Isotropic elastic constants."""

import numpy as np


def lame_from_E_nu(E, nu):
    """(lambda, mu) from Young's modulus and Poisson's ratio (textbook relations)."""
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def isotropic_bulk_shear(lam, mu):
    """(K, G) of an isotropic material given its Lame pair."""
    return lam + 2.0 * mu / 3.0, mu
