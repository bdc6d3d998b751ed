"""Isotropic kernels k(r; l) and their derivatives (oracle, test infrastructure).

The paper's experiments (Sec. 4.1, the Fig. 3 paragraph) use the Cauchy kernel,
a Gaussian and the Matern kernels with nu = 1.5 and nu = 2.5.  The Gaussian is
taken here as exp(-r^2 / (2 l^2)) (the lengthscale convention of the synthetic
workloads; the paper writes exp(-(r/sigma)^2), i.e. sigma = sqrt(2) l).  Every function accepts real or complex ``r`` / ``l`` so that the
complex-step derivative can be used on it.
"""
import numpy as np

KERNELS = ("gaussian", "cauchy", "matern32", "matern52")
KERNEL_ID = {"gaussian": 0, "cauchy": 1, "matern32": 2, "matern52": 3}


def kappa(name, r, l):
    """k(r; l) for r >= 0 (Sec. 4.1)."""
    r = np.asarray(r)
    if name == "gaussian":
        return np.exp(-(r * r) / (2.0 * l * l))
    if name == "cauchy":
        return 1.0 / (1.0 + (r * r) / (l * l))
    if name == "matern32":
        z = np.sqrt(3.0) * r / l
        return (1.0 + z) * np.exp(-z)
    if name == "matern52":
        z = np.sqrt(5.0) * r / l
        return (1.0 + z + z * z / 3.0) * np.exp(-z)
    raise ValueError(name)


def dkappa_dr(name, r, l):
    """d k / d r, closed form."""
    r = np.asarray(r)
    k = kappa(name, r, l)
    if name == "gaussian":
        return -k * r / (l * l)
    if name == "cauchy":
        return -2.0 * r * k * k / (l * l)
    if name == "matern32":
        c = np.sqrt(3.0) / l
        z = c * r
        return -z * np.exp(-z) * c
    if name == "matern52":
        c = np.sqrt(5.0) / l
        z = c * r
        return -(z / 3.0) * (1.0 + z) * np.exp(-z) * c
    raise ValueError(name)


def dkappa_dl(name, r, l):
    """d k / d l, closed form (z = c r / l gives dz/dl = -z/l)."""
    r = np.asarray(r)
    k = kappa(name, r, l)
    if name == "gaussian":
        return k * r * r / (l * l * l)
    if name == "cauchy":
        return 2.0 * r * r * k * k / (l * l * l)
    if name == "matern32":
        z = np.sqrt(3.0) * r / l
        return z * np.exp(-z) * z / l
    if name == "matern52":
        z = np.sqrt(5.0) * r / l
        return (z / 3.0) * (1.0 + z) * np.exp(-z) * z / l
    raise ValueError(name)
