"""Real hyperspherical harmonics (oracle, test infrastructure).

Eq. additiontheorem: C_k^alpha(cos g) / Z_k = sum_{h in H_k} Y_k^h(x) Y_k^h(y),
with H_k = {(mu_1..mu_{d-2}) : k >= mu_1 >= ... >= |mu_{d-2}| >= 0} (Sec. 3.3)
and |H_k| = C(k+d-1, k) - C(k+d-3, k-2) (App. B).  The paper leaves the
definition of the real basis to the literature; the one used here is the
standard polar-chain construction:

* coordinates x_1..x_d, polar axis x_1, azimuthal plane (x_{d-1}, x_d),
  partial radii r_j^2 = x_j^2 + ... + x_d^2;
* with mu_0 = k, n_j = |mu_{j-1}| - |mu_j| and lambda_j = |mu_j| + (d-j-1)/2,
  the solid harmonic (homogeneous harmonic polynomial of degree k) is

    S_mu(x) = N_mu * prod_{j=1}^{d-2} r_j^{n_j} C^{lambda_j}_{n_j}(x_j / r_j)
                   * (Re if mu_{d-2} >= 0 else Im) (x_{d-1} + i x_d)^{|mu_{d-2}|}

  where each bracket is a polynomial in (x_j, r_j^2) (no square roots);
* N_mu^{-2} = (2 pi if mu_{d-2} = 0 else pi) * prod_j h^{lambda_j}_{n_j},
  h_n^lam = pi 2^{1-2 lam} Gamma(n + 2 lam) / (n! (n + lam) Gamma(lam)^2), so
  that Y = S / ||x||^k is orthonormal on the unit sphere;
* Z_k = alpha |S^{d-1}| / (k + alpha), |S^{d-1}| = 2 pi^{d/2} / Gamma(d/2).

Enumeration order (fixed, shared by construction with the device path only
through this written rule): k ascending, then lexicographic ascending in
(mu_1, ..., mu_{d-2}), the last entry running from -mu_{d-3} to +mu_{d-3}.
"""
from functools import lru_cache
from math import comb

import mpmath
import numpy as np


def index_set(d, k):
    """H_k as a list of tuples in the fixed enumeration order."""
    out = []

    def rec(prefix, upper, depth):
        if depth == d - 2:            # last (signed) index
            for m in range(-upper, upper + 1):
                out.append(tuple(prefix) + (m,))
            return
        for mu in range(0, upper + 1):
            rec(prefix + [mu], mu, depth + 1)

    rec([], k, 1)
    return out


def count(d, k):
    """|H_k| (App. B)."""
    if k < 0:
        return 0
    return comb(k + d - 1, k) - (comb(k + d - 3, k - 2) if k >= 2 else 0)


def count_upto(d, K):
    """sum_{k<=K} |H_k| = C(K+d-1, d-1) + C(K+d-2, d-1) (App. B)."""
    return comb(K + d - 1, d - 1) + comb(K + d - 2, d - 1)


def sphere_area_mp(d):
    return 2 * mpmath.pi ** (mpmath.mpf(d) / 2) / mpmath.gamma(mpmath.mpf(d) / 2)


def Z_mp(k, d):
    alpha = mpmath.mpf(d) / 2 - 1
    return alpha * sphere_area_mp(d) / (k + alpha)


def Z(k, d):
    return float(Z_mp(k, d))


def sphere_area(d):
    return float(sphere_area_mp(d))


@lru_cache(maxsize=None)
def _h(n, lam2):
    """h_n^lambda for lambda = lam2/2 (exact half-integers), via mpmath."""
    with mpmath.workdps(40):
        lam = mpmath.mpf(lam2) / 2
        v = (mpmath.pi * mpmath.power(2, 1 - 2 * lam) * mpmath.gamma(n + 2 * lam)
             / (mpmath.factorial(n) * (n + lam) * mpmath.gamma(lam) ** 2))
        return v


@lru_cache(maxsize=None)
def norm_const(d, k, mu):
    """N_mu (binary64)."""
    with mpmath.workdps(40):
        prev = k
        inv2 = 2 * mpmath.pi if mu[-1] == 0 else mpmath.pi
        for j in range(1, d - 1):
            cur = abs(mu[j - 1])
            n = prev - cur
            lam2 = 2 * cur + (d - j - 1)
            inv2 *= _h(n, lam2)
            prev = cur
        return float(1 / mpmath.sqrt(inv2))


def gegen_solid(n_max, lam, x, r2):
    """[r^n C_n^lam(x/r) for n = 0..n_max] as polynomials in (x, r^2)."""
    P = [np.ones_like(x)]
    if n_max >= 1:
        P.append(2.0 * lam * x)
    for n in range(1, n_max):
        P.append((2.0 * (n + lam) * x * P[n] - (n + 2.0 * lam - 1.0) * r2 * P[n - 1]) / (n + 1))
    return P


def solid_harmonics(X, K, degrees=None):
    """Dict k -> array (N, |H_k|) of S_mu(X) for the unit-ball points X.

    X may be complex (complex-step differentiation); r_j^2 is the analytic
    sum of squares.
    """
    X = np.asarray(X)
    N, d = X.shape
    if degrees is None:
        degrees = range(K + 1)
    r2 = [None] * d                  # r2[j] for 0-based coordinate j
    acc = np.zeros(N, dtype=X.dtype)
    for j in range(d - 1, -1, -1):
        acc = acc + X[:, j] * X[:, j]
        r2[j] = acc
    cache = {}

    def factor(level, n, b):
        # level j (1-based) -> coordinate j-1; lambda = b + (d-j-1)/2
        key = (level, b)
        if key not in cache:
            lam = b + (d - level - 1) / 2.0
            cache[key] = gegen_solid(K - b, lam, X[:, level - 1], r2[level - 1])
        return cache[key][n]

    out = {}
    for k in degrees:
        H = index_set(d, k)
        S = np.empty((N, len(H)), dtype=X.dtype)
        for h, mu in enumerate(H):
            v = np.full(N, norm_const(d, k, mu), dtype=X.dtype)
            prev = k
            for j in range(1, d - 1):
                cur = abs(mu[j - 1])
                v = v * factor(j, prev - cur, cur)
                prev = cur
            m = mu[-1]
            v = v * _azimuthal(X, abs(m), m >= 0)
            S[:, h] = v
        out[k] = S
    return out


def _azimuthal(X, m, real_part):
    """Re / Im of (x_{d-1} + i x_d)^m as polynomials in (x_{d-1}, x_d).

    C_{q+1} = a C_q - b S_q, S_{q+1} = b C_q + a S_q (complex multiplication
    written on the real and imaginary parts), so complex X (complex-step) is
    handled without mixing the two imaginary units.
    """
    d = X.shape[1]
    a = X[:, d - 2]
    b = X[:, d - 1]
    C = np.ones_like(a)
    S = np.zeros_like(a)
    for _ in range(m):
        C, S = a * C - b * S, b * C + a * S
    return C if real_part else S
