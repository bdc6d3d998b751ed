"""Domain normalisation (oracle, test infrastructure).

Sec. 3.3 (footnote 1) assumes every pairwise distance lies in [0, 1] and
absorbs the diameter of the point set into the kernel's lengthscale.  The
reading used here: centre c = midpoint of the bounding box, radius
R = max_i ||x_i - c||, diameter bound D = 2R, so that z = (x - c)/D has
||z_i - z_j|| <= 1.  The normalised radius rho_i = ||x_i - c|| / R lies in
[0, 1] and ||z_i|| = rho_i / 2.

Every step is written so that its rounding is fixed: min/max are exact,
(min + max)/2 is exact in binary64 for binary32 inputs, the squared norms are
summed in coordinate order with no fused multiply-add, and sqrt is correctly
rounded.
"""
import numpy as np


def geometry(X):
    """Return dict(c, R, D, xt, rho2, u0, u1) for points X (N x d, float64).

    xt = (X - c) / R_eff (R_eff = R, or 1 when all points coincide),
    rho2_i = sum_j xt_ij^2 (coordinate order), u0/u1 = the interval of rho^2
    on which the radial Chebyshev basis is defined.
    """
    X = np.asarray(X, dtype=np.float64)
    N, d = X.shape
    c = (X.min(axis=0) + X.max(axis=0)) / 2.0
    s = np.zeros(N)
    for j in range(d):
        t = X[:, j] - c[j]
        s = s + t * t
    R2 = s.max()
    R = float(np.sqrt(R2))
    Reff = R if R > 0.0 else 1.0
    xt = (X - c[None, :]) / Reff
    rho2 = np.zeros(N)
    for j in range(d):
        rho2 = rho2 + xt[:, j] * xt[:, j]
    u0, u1 = radial_interval(rho2.min(), rho2.max())
    return dict(c=c, R=R, Reff=Reff, D=2.0 * R, xt=xt, rho2=rho2, u0=u0, u1=u1)


def radial_interval(rmin2, rmax2):
    """Interval [u0, u1] of rho^2 carrying the radial basis.

    Reading (the paper is silent): the data range [min rho^2, max rho^2]; when
    it has zero width the interval is widened to [0, max rho^2], and to [0, 1]
    when every rho is zero.
    """
    u0, u1 = float(rmin2), float(rmax2)
    if not (u1 > u0):
        u0 = 0.0
        if not (u1 > 0.0):
            u1 = 1.0
    return u0, u1
