"""Analytic expansion into Gegenbauer degrees (oracle, test infrastructure).

App. A re-expands sum_i a_i T_i(||x - y||) by the multinomial theorem, swaps
the sums, and turns powers of cos(gamma) into Gegenbauer polynomials
C_j^alpha (alpha = d/2 - 1), giving (Eq. preharm)

    k(||x - y||) ~ sum_j C_j^alpha(cos gamma) sum_{m,n} ||y||^m ||x||^n T'_{j,m,n}

with (end of App. A)

    T'_{j,m,n} = sum_{k3} A_{j,k3} (-2)^{k3} multinom((n+m)/2; (n-k3)/2, (m-k3)/2, k3)
                 * sum_{i >= n+m} t_{i,n+m} a_i .

Everything here is exact rational arithmetic.  Readings of garbled passages:

* A_{j,i}, the coefficient of C_j^alpha in cos^i (App. A), is
  i! (alpha + j) / (2^i ((i-j)/2)! (alpha)_{(i+j)/2+1}) for i = j mod 2; the
  printed formula lacks the factorial on (i-j)/2.
* the multinomial sum bound written k_2 <= j - k_3 in App. A is j/2 - k_3.
* T'_{j,m,n} is non-zero only for m = n = j (mod 2); for degree j the radial
  exponents are n = j + 2a, m = j + 2b with a + b <= (p - 2j)/2, so r^{(j)}
  (Eq. rdef) has rank L_j = (p - 2j)/2 + 1 (Sec. 3.4 states (p - 2j)/2).

Radial basis.  With ||x|| = rho/2 (see geometry.py) the degree-j part is
(rho_x rho_y)^j times a polynomial in (rho_x^2, rho_y^2).  Sec. 3.7 notes that
powers of the norm make ill-conditioned Vandermonde matrices and suggests an
orthogonal-polynomial basis instead; the core is therefore re-expressed
exactly in Chebyshev polynomials phi_a(rho^2) = T_a(t),
t = (2 rho^2 - u0 - u1) / (u1 - u0), before a single rounding to binary64.
The addition-theorem factor Z_j (Eq. additiontheorem, T'' = Z T' in
Eq. preeigen) is folded into the core, so that

    k ~ sum_j sum_h S_j^h(xt) S_j^h(yt) sum_{a,b} M_j[a,b] phi_a(rho_x^2) phi_b(rho_y^2)

with S_j^h the solid harmonics of the unit-ball points xt = (x - c)/R.
"""
from fractions import Fraction
from math import comb, factorial

import mpmath

from .chebyshev import cheb_monomial_table, exact
from .harmonics import sphere_area_mp, Z_mp


def rising(x, n):
    """Pochhammer (x)_n for a Fraction x."""
    r = Fraction(1)
    for i in range(n):
        r *= x + i
    return r


def gegenbauer_power_coeff(j, i, alpha):
    """A_{j,i}: cos^i(g) = sum_j A_{j,i} C_j^alpha(cos g) (App. A)."""
    if j > i or (i - j) % 2:
        return Fraction(0)
    return Fraction(factorial(i)) * (alpha + j) / (
        Fraction(2) ** i * factorial((i - j) // 2) * rising(alpha, (i + j) // 2 + 1))


def multinomial(n, ks):
    r = factorial(n)
    for k in ks:
        r //= factorial(k)
    return r


def power_coeffs(a_exact, p):
    """c_J = sum_{i >= J} t_{i,J} a_i: monomial coefficients of sum_i a_i T_i."""
    t = cheb_monomial_table(p)
    return [sum((t[i][J] * a_exact[i] for i in range(J, p + 1)), Fraction(0))
            for J in range(p + 1)]


def T_prime(a_exact, p, d):
    """Dict (j, m, n) -> exact T'_{j,m,n} (end of App. A)."""
    alpha = Fraction(d - 2, 2)
    c = power_coeffs(a_exact, p)
    out = {}
    for j in range(p // 2 + 1):
        for m in range(j, p - j + 1, 2):
            for n in range(j, p - m + 1, 2):
                acc = Fraction(0)
                for k3 in range(j, min(m, n) + 1, 2):
                    acc += (gegenbauer_power_coeff(j, k3, alpha) * (-2) ** k3
                            * multinomial((n + m) // 2, ((n - k3) // 2, (m - k3) // 2, k3)))
                out[(j, m, n)] = acc * c[n + m]
    return out


def power_core(Tp, p, j):
    """P_j[a][b]: coefficient of (rho_x^2)^a (rho_y^2)^b, without Z_j.

    ||x||^n ||y||^m with ||x|| = rho_x / 2, n = j + 2a, m = j + 2b.
    """
    L = (p - 2 * j) // 2 + 1
    P = [[Fraction(0)] * L for _ in range(L)]
    for a in range(L):
        for b in range(L - a):
            P[a][b] = Tp[(j, j + 2 * b, j + 2 * a)] / Fraction(4) ** (j + a + b)
    return P


def monomial_to_cheb(L, u0, u1):
    """B[a][c]: (rho^2)^a = sum_c B[a][c] T_c(t), rho^2 = (u0+u1)/2 + t (u1-u0)/2."""
    a0 = (Fraction(u0) + Fraction(u1)) / 2
    a1 = (Fraction(u1) - Fraction(u0)) / 2
    # t^e in Chebyshev polynomials: 2^{1-e} sum_{c=e,e-2,..} C(e,(e-c)/2) T_c, T_0 term halved
    tpow = []
    for e in range(L):
        row = [Fraction(0)] * L
        for cc in range(e % 2, e + 1, 2):
            v = Fraction(comb(e, (e - cc) // 2)) / Fraction(2) ** (e - 1) if e > 0 else Fraction(2)
            if cc == 0:
                v /= 2
            row[cc] = v
        tpow.append(row)
    B = []
    for a in range(L):
        row = [Fraction(0)] * L
        for e in range(a + 1):
            coef = comb(a, e) * a0 ** (a - e) * a1 ** e
            if coef == 0:
                continue
            for cc in range(L):
                if tpow[e][cc]:
                    row[cc] += coef * tpow[e][cc]
        B.append(row)
    return B


def radial_cores(a, p, d, u0, u1, dps=60):
    """Binary64 cores M_j (j = 0..p/2), each L_j x L_j, in the T_a(t) basis.

    Exact: M_j = Z_j * B^T P_j B, rounded once (Z_j evaluated at ``dps``
    digits).
    """
    a_ex = exact(list(a[: p + 1]))
    Tp = T_prime(a_ex, p, d)
    mpmath.mp.dps = dps
    cores = []
    for j in range(p // 2 + 1):
        L = (p - 2 * j) // 2 + 1
        P = power_core(Tp, p, j)
        B = monomial_to_cheb(L, u0, u1)
        # PB = P B ; M = B^T P B
        PB = [[sum((P[a][b] * B[b][cc] for b in range(L) if P[a][b]), Fraction(0))
               for cc in range(L)] for a in range(L)]
        Mx = [[sum((B[a][r] * PB[a][cc] for a in range(L)), Fraction(0))
               for cc in range(L)] for r in range(L)]
        Z = Z_mp(j, d)
        cores.append([[float(mpmath.mpf(v.numerator) / v.denominator * Z) for v in row]
                      for row in Mx])
    return cores
