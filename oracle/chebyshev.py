"""Truncated Chebyshev expansion of the kernel (oracle, test infrastructure).

Sec. 3.3 (Eq. chebtrunc): the kernel, with the diameter D absorbed
(f(s) = k(D |s|; l) on [-1, 1]), is even, so its Chebyshev coefficients of odd
index vanish and the truncation degree p is even.  The coefficients are
obtained from the discrete cosine transform (Clenshaw-Curtis, Sec. 3.3) at
N_F first-kind nodes; at N_F >> p this interpolant equals the truncated series
to rounding level (reading of the unweighted integral written in Sec. 3.3: the
standard Chebyshev projection is meant).

Degree selection (ChebDegreeNeeded of Algorithm 1, left unspecified by the
paper, Sec. 3.5 Remark 3): the smallest even p whose tail sum_{i>p} |a_i| is
at most eps * nu / 2, where nu ~ ||K||_F / N.  Since |T_i| <= 1 on [-1, 1] the
tail bounds every entry of the truncation error, so its Frobenius norm is at
most eps * nu * N / 2.
"""
from fractions import Fraction

import numpy as np
import scipy.fft

from .kernels import kappa, dkappa_dl

N_F = 8192          # number of Chebyshev nodes of the transform
P_MAX = 256         # largest degree the method is allowed to choose


def cheb_nodes(n=N_F):
    theta = np.pi * (np.arange(n) + 0.5) / n
    return np.cos(theta)


def cheb_coeffs_values(fvals):
    """Chebyshev coefficients of the interpolant through first-kind nodes.

    a_i = (2/n) sum_j f(s_j) cos(i theta_j), a_0 halved; odd a_i set to zero
    (Sec. 3.3: the even extension has no odd coefficients).
    """
    n = len(fvals)
    a = scipy.fft.dct(np.asarray(fvals), type=2) / n
    a[0] *= 0.5
    a[1::2] = 0.0
    return a


def cheb_coeffs(name, D, l, n=N_F):
    """Coefficients of f(s) = k(D |s|; l) (Eq. chebtrunc)."""
    s = cheb_nodes(n)
    return cheb_coeffs_values(kappa(name, D * np.abs(s), l))


def cheb_coeffs_dl(name, D, l, n=N_F):
    """Coefficients of d f / d l, used by the lengthscale derivative."""
    s = cheb_nodes(n)
    return cheb_coeffs_values(dkappa_dl(name, D * np.abs(s), l))


def tail_sums(a):
    """tail[p] = sum_{i>p} |a_i|, accumulated from the highest index down."""
    n = len(a)
    tail = np.zeros(n)
    acc = 0.0
    for i in range(n - 1, 0, -1):
        acc = acc + abs(a[i])
        tail[i - 1] = acc
    return tail


def choose_degree(a, eps, nu, p_max=P_MAX):
    """Smallest even p with sum_{i>p}|a_i| <= eps*nu/2; None if p > p_max."""
    tail = tail_sums(a)
    thr = eps * nu / 2.0
    for p in range(0, min(p_max, len(a) - 1) + 1, 2):
        if tail[p] <= thr:
            return p, tail[p], thr
    return None, None, thr


def cheb_monomial_table(p):
    """t[i][j]: T_i(s) = sum_j t[i][j] s^j (Eq. chebdef), exact integers.

    The three-term recurrence T_i = 2 s T_{i-1} - T_{i-2} gives
    t_{i,j} = 2 t_{i-1,j-1} - t_{i-2,j} with t_{0,0} = t_{1,1} = 1.  (Sec. 3.3
    states t_{i,i} = 1 for every i, which holds only for i <= 1: the leading
    coefficient of T_i is 2^{i-1}.)
    """
    t = [[0] * (p + 1) for _ in range(p + 1)]
    t[0][0] = 1
    if p >= 1:
        t[1][1] = 1
    for i in range(2, p + 1):
        for j in range(0, i + 1):
            v = -t[i - 2][j]
            if j >= 1:
                v += 2 * t[i - 1][j - 1]
            t[i][j] = v
    return t


def exact(a):
    """Exact rational value of each binary64 coefficient."""
    return [Fraction(float(v)) for v in a]
