"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks one oracle step against something other than itself: a
closed form, a library special case, an identity, a brute-force sum or a
hand-written fixture.  None of them needs a GPU.
"""
import os
from math import comb

import numpy as np
import pytest
import scipy.special as ss
from numpy.polynomial import chebyshev as npcheb

from oracle import chebyshev, cross, dense, expansion, geometry, harmonics, hdf, kernels, splitmix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def unit_ball(rng, N, d):
    g = rng.normal(size=(N, d))
    return g / np.linalg.norm(g, axis=1)[:, None] * rng.random(N)[:, None] ** (1.0 / d)


# ---------------------------------------------------------------- Q1 kernels
@pytest.mark.parametrize("name", kernels.KERNELS)
def test_kernel_derivatives_complex_step(name):
    r = np.linspace(0.01, 3.0, 50)
    l = 0.8
    h = 1e-30
    dr = kernels.kappa(name, r + 1j * h, l).imag / h
    dl = kernels.kappa(name, r, l + 1j * h).imag / h
    np.testing.assert_allclose(kernels.dkappa_dr(name, r, l), dr, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(kernels.dkappa_dl(name, r, l), dl, rtol=1e-13, atol=1e-15)


def test_kernel_values():
    # k(0) = 1 for all four; spot values from the definitions of Sec. 4.1
    for name in kernels.KERNELS:
        assert kernels.kappa(name, 0.0, 1.3) == 1.0
    assert np.isclose(kernels.kappa("cauchy", 2.0, 1.0), 0.2)
    assert np.isclose(kernels.kappa("gaussian", 1.0, 1.0), np.exp(-0.5))
    z = np.sqrt(3.0)
    assert np.isclose(kernels.kappa("matern32", 1.0, 1.0), (1 + z) * np.exp(-z))
    z = np.sqrt(5.0)
    assert np.isclose(kernels.kappa("matern52", 1.0, 1.0), (1 + z + z * z / 3) * np.exp(-z))


# ------------------------------------------------------ Q2 Chebyshev transform
@pytest.mark.parametrize("D,l", [(2.0, 1.0), (3.9, 0.7), (1.0, 0.3)])
def test_cheb_gaussian_closed_form(D, l):
    # exp(-A s^2), A = D^2/(2 l^2): a_2n = (2 - delta_n0) (-1)^n e^{-A/2} I_n(A/2)
    A = D * D / (2 * l * l)
    a = chebyshev.cheb_coeffs("gaussian", D, l)
    n = np.arange(40)
    ref = (2.0 - (n == 0)) * (-1.0) ** n * ss.ive(n, A / 2)
    np.testing.assert_allclose(a[0:80:2], ref, atol=5e-16 * max(1, A))
    assert np.all(a[1::2] == 0.0)


@pytest.mark.parametrize("D,l", [(2.0, 1.0), (1.9, 1.0), (7.5, 1.0)])
def test_cheb_cauchy_closed_form(D, l):
    # 1/(1 + b^2 s^2): a_2n = (2 - delta_n0)(-1)^n q^{2n} / sqrt(1+b^2), q = (sqrt(1+b^2)-1)/b
    b = D / l
    q = (np.sqrt(1 + b * b) - 1) / b
    a = chebyshev.cheb_coeffs("cauchy", D, l)
    n = np.arange(60)
    ref = (2.0 - (n == 0)) * (-1.0) ** n * q ** (2 * n) / np.sqrt(1 + b * b)
    np.testing.assert_allclose(a[0:120:2], ref, atol=1e-15)


@pytest.mark.parametrize("name", ["matern32", "matern52"])
def test_cheb_matern_node_doubling(name):
    a1 = chebyshev.cheb_coeffs(name, 2.0, 0.5, n=8192)
    a2 = chebyshev.cheb_coeffs(name, 2.0, 0.5, n=16384)
    # aliasing error ~ |a_{2n_f - i}|: the algebraic tail (i^-4 / i^-6) is tiny here
    np.testing.assert_allclose(a1[:400], a2[:400], atol=1e-12)


def test_degree_selection_rule():
    a = chebyshev.cheb_coeffs("cauchy", 2.0, 1.0)
    p, tail, thr = chebyshev.choose_degree(a, 1e-4, 0.5)
    assert p % 2 == 0
    assert np.sum(np.abs(a[p + 1:])) <= thr * (1 + 1e-12)
    assert np.sum(np.abs(a[p - 1:])) > thr         # p - 2 would not do
    # truncation error is bounded entrywise by the tail (|T_i| <= 1)
    s = np.linspace(-1, 1, 2001)
    f = kernels.kappa("cauchy", 2.0 * np.abs(s), 1.0)
    assert np.max(np.abs(npcheb.chebval(s, a[: p + 1]) - f)) <= tail + 1e-15


# ------------------------------------------------------------- Q3 t_{i,j}
def test_cheb_monomial_table_matches_numpy():
    p = 24
    t = chebyshev.cheb_monomial_table(p)
    for i in range(p + 1):
        e = np.zeros(i + 1)
        e[i] = 1
        ref = npcheb.cheb2poly(e)
        assert [int(round(v)) for v in ref] == t[i][: i + 1]


def test_cheb_monomial_table_leading_coefficient():
    # the corrected recurrence: leading coefficient of T_i is 2^{i-1} for i >= 1
    t = chebyshev.cheb_monomial_table(12)
    assert t[0][0] == 1 and t[1][1] == 1
    for i in range(2, 13):
        assert t[i][i] == 2 ** (i - 1)


# ---------------------------------------------------------------- Q4 A_{j,i}
@pytest.mark.parametrize("d", [3, 4, 5, 6, 7])
def test_gegenbauer_power_coeffs(d):
    from fractions import Fraction
    alpha = Fraction(d - 2, 2)
    tt = np.linspace(-1, 1, 21)
    for i in range(0, 13):
        acc = np.zeros_like(tt)
        for j in range(i + 1):
            acc += float(expansion.gegenbauer_power_coeff(j, i, alpha)) * ss.eval_gegenbauer(j, float(alpha), tt)
        np.testing.assert_allclose(acc, tt ** i, atol=1e-13)


# ------------------------------------------------------------------ Q5 T'
@pytest.mark.parametrize("d", [3, 4, 5, 6])
@pytest.mark.parametrize("name,D,l,p", [("gaussian", 2.0, 1.0, 12), ("cauchy", 1.9, 1.0, 16),
                                        ("matern52", 1.0, 0.7, 10)])
def test_Tprime_brute_force_identity(d, name, D, l, p):
    """sum_i a_i T_i(||x-y||) = sum_j C_j(cos g) sum_{m,n} ||y||^m ||x||^n T'_{j,m,n}."""
    rng = np.random.default_rng(5 + d + p)
    a = chebyshev.cheb_coeffs(name, D, l)[: p + 1]
    Tp = expansion.T_prime(chebyshev.exact(a), p, d)
    alpha = (d - 2) / 2
    for _ in range(6):
        x = unit_ball(rng, 1, d)[0] * 0.5
        y = unit_ball(rng, 1, d)[0] * 0.5
        s = np.linalg.norm(x - y)
        lhs = npcheb.chebval(s, a)
        nx, ny = np.linalg.norm(x), np.linalg.norm(y)
        cg = x @ y / (nx * ny)
        rhs = 0.0
        for (j, m, n), v in Tp.items():
            rhs += ss.eval_gegenbauer(j, alpha, cg) * ny ** m * nx ** n * float(v)
        assert abs(lhs - rhs) < 2e-14 * max(1.0, np.sum(np.abs(a)))


def test_Tprime_symmetry_and_parity():
    a = chebyshev.cheb_coeffs("cauchy", 2.0, 1.0)[:15]
    Tp = expansion.T_prime(chebyshev.exact(a), 14, 5)
    for (j, m, n), v in Tp.items():
        assert (j - m) % 2 == 0 and (j - n) % 2 == 0
        assert Tp.get((j, n, m)) == v


# -------------------------------------------------------------- Q6 counts
@pytest.mark.parametrize("d", [3, 4, 5, 6, 7])
def test_harmonic_counts(d):
    tot = 0
    for k in range(0, 12):
        n = len(harmonics.index_set(d, k))
        assert n == harmonics.count(d, k)
        # dimension of degree-k harmonics: (2k+d-2)(k+d-3)!/(k!(d-2)!)
        assert n == (2 * k + d - 2) * comb(k + d - 3, k) // (d - 2)
        tot += n
        assert tot == harmonics.count_upto(d, k)


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append(tuple(int(v) for v in line.split()))
    return rows


def test_index_set_golden():
    assert harmonics.index_set(4, 2) == _read_golden("index_set_d4_k2.txt")
    assert harmonics.index_set(5, 2) == _read_golden("index_set_d5_k2.txt")


# ------------------------------------------------------------ Q7 harmonics
@pytest.mark.parametrize("d", [3, 4, 5, 6])
def test_addition_theorem(d):
    rng = np.random.default_rng(d)
    K = 7
    x = rng.normal(size=(20, d))
    y = rng.normal(size=(20, d))
    x /= np.linalg.norm(x, axis=1)[:, None]
    y /= np.linalg.norm(y, axis=1)[:, None]
    Sx = harmonics.solid_harmonics(x, K)
    Sy = harmonics.solid_harmonics(y, K)
    cg = np.sum(x * y, axis=1)
    for k in range(K + 1):
        lhs = np.sum(Sx[k] * Sy[k], axis=1)
        rhs = ss.eval_gegenbauer(k, (d - 2) / 2, cg) / harmonics.Z(k, d)
        np.testing.assert_allclose(lhs, rhs, atol=1e-13)


@pytest.mark.parametrize("d", [3, 4, 5])
def test_solid_harmonics_are_harmonic_and_homogeneous(d):
    rng = np.random.default_rng(40 + d)
    K = 5
    x = rng.normal(size=(4, d)) * 0.4
    S = harmonics.solid_harmonics(x, K)
    S2 = harmonics.solid_harmonics(1.7 * x, K)
    for k in range(K + 1):
        np.testing.assert_allclose(S2[k], 1.7 ** k * S[k], rtol=1e-12, atol=1e-14)
    # mean-value property: the average over any sphere equals the centre value
    Xq, w = _sphere_quadrature(d, n_theta=16, n_phi=24)
    area = w.sum()
    for i in range(x.shape[0]):
        Sq = harmonics.solid_harmonics(x[i] + 0.35 * Xq, K)
        for k in range(K + 1):
            np.testing.assert_allclose(w @ Sq[k] / area, S[k][i], atol=1e-13)


def _sphere_quadrature(d, n_theta=40, n_phi=64):
    """Product rule on S^{d-1}: Gauss-Legendre in each polar angle, trapezoid in phi."""
    xg, wg = np.polynomial.legendre.leggauss(n_theta)
    th = (xg + 1) * np.pi / 2
    wth = wg * np.pi / 2
    phis = 2 * np.pi * np.arange(n_phi) / n_phi
    grids = np.meshgrid(*([th] * (d - 2) + [phis]), indexing="ij")
    wgrids = np.meshgrid(*([wth] * (d - 2) + [np.full(n_phi, 2 * np.pi / n_phi)]), indexing="ij")
    angles = [g.ravel() for g in grids]
    w = np.ones_like(angles[0])
    for j in range(d - 2):
        w = w * wgrids[j].ravel() * np.sin(angles[j]) ** (d - j - 2)
    w = w * wgrids[d - 2].ravel()
    X = np.empty((len(w), d))
    sprod = np.ones_like(w)
    for j in range(d - 2):
        X[:, j] = sprod * np.cos(angles[j])
        sprod = sprod * np.sin(angles[j])
    X[:, d - 2] = sprod * np.cos(angles[d - 2])
    X[:, d - 1] = sprod * np.sin(angles[d - 2])
    return X, w


@pytest.mark.parametrize("d,K,nt", [(3, 6, 40), (4, 4, 30), (5, 3, 20)])
def test_harmonics_orthonormal_quadrature(d, K, nt):
    X, w = _sphere_quadrature(d, n_theta=nt, n_phi=4 * K + 8)
    assert abs(w.sum() - harmonics.sphere_area(d)) < 1e-12
    S = harmonics.solid_harmonics(X, K)
    A = np.concatenate([S[k] for k in range(K + 1)], axis=1)
    G = A.T @ (w[:, None] * A)
    np.testing.assert_allclose(G, np.eye(G.shape[0]), atol=1e-13)


def test_d3_matches_scipy_spherical_harmonics():
    rng = np.random.default_rng(7)
    x = rng.normal(size=(30, 3))
    x /= np.linalg.norm(x, axis=1)[:, None]
    theta = np.arccos(x[:, 0])            # polar axis x_1
    phi = np.arctan2(x[:, 2], x[:, 1])    # azimuth in (x_2, x_3)
    K = 6
    S = harmonics.solid_harmonics(x, K)
    for k in range(K + 1):
        for h, (m,) in enumerate(harmonics.index_set(3, k)):
            Y = ss.sph_harm_y(k, abs(m), theta, phi)
            ref = Y.real if m == 0 else np.sqrt(2) * (Y.real if m > 0 else Y.imag)
            ratio = S[k][:, h] / ref
            # same function up to the Condon-Shortley sign (-1)^m
            np.testing.assert_allclose(ratio, (-1.0) ** abs(m), rtol=1e-11)


# ------------------------------------------------------------------ Q8 M_k
def test_change_of_basis():
    u0, u1 = 0.037, 0.91
    B = expansion.monomial_to_cheb(9, u0, u1)
    rr = np.linspace(u0, u1, 13)
    t = (2 * rr - u0 - u1) / (u1 - u0)
    T = hdf.cheb_basis(t, 9)
    for a in range(9):
        np.testing.assert_allclose(T @ np.array([float(v) for v in B[a]]), rr ** a, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("d", [3, 4, 5, 6])
@pytest.mark.parametrize("name,D,l,p", [("gaussian", 2.0, 1.0, 14), ("cauchy", 1.9, 1.0, 12),
                                        ("matern32", 1.5, 1.0, 10)])
def test_cores_equal_gegenbauer_projection(d, name, D, l, p):
    """(rho_x rho_y)^k / Z_k * sum M_k phi phi = Gegenbauer coefficient of f_p(s(t))."""
    a = chebyshev.cheb_coeffs(name, D, l)[: p + 1]
    u0, u1 = 0.05, 0.97
    cores = expansion.radial_cores(a, p, d, u0, u1)
    alpha = (d - 2) / 2
    nodes, wts = ss.roots_gegenbauer(p // 2 + 2, alpha)
    rng = np.random.default_rng(d * 100 + p)
    for _ in range(4):
        rx2, ry2 = rng.uniform(u0, u1, 2)
        rx, ry = np.sqrt(rx2), np.sqrt(ry2)
        s = 0.5 * np.sqrt(rx2 + ry2 - 2 * rx * ry * nodes)
        f = npcheb.chebval(s, a)
        tx = (2 * rx2 - u0 - u1) / (u1 - u0)
        ty = (2 * ry2 - u0 - u1) / (u1 - u0)
        for k in range(p // 2 + 1):
            hk = np.pi * 2 ** (1 - 2 * alpha) * ss.gamma(k + 2 * alpha) / (
                ss.factorial(k) * (k + alpha) * ss.gamma(alpha) ** 2)
            proj = np.sum(wts * f * ss.eval_gegenbauer(k, alpha, nodes)) / hk
            L = p // 2 - k + 1
            M = np.array(cores[k])
            val = (rx * ry) ** k / harmonics.Z(k, d) * (hdf.cheb_basis(tx, L) @ M @ hdf.cheb_basis(ty, L))
            assert abs(val - proj) < 1e-13 * max(1.0, np.sum(np.abs(a)))


def test_cores_symmetric():
    a = chebyshev.cheb_coeffs("cauchy", 2.0, 1.0)
    cores = expansion.radial_cores(a, 18, 5, 0.0, 1.0)
    for M in cores:
        M = np.array(M)
        np.testing.assert_allclose(M, M.T, rtol=1e-15, atol=0)


# ------------------------------------------------- Q9 uncompressed factor
@pytest.mark.parametrize("d,name", [(3, "gaussian"), (4, "cauchy"), (5, "matern52"), (6, "gaussian")])
def test_uncompressed_factor_reproduces_chebyshev_kernel(d, name):
    rng = np.random.default_rng(11 * d)
    X = unit_ball(rng, 120, d) * 1.7 + 0.3
    p = 10
    st = hdf.build(X, name, 1.0, 1e-6, p=p, tau=0.0)
    U, Dv = hdf.factor(st)
    Kt = (U * Dv) @ U.T
    from scipy.spatial.distance import cdist
    s = cdist(X, X) / st["D"]
    Kp = npcheb.chebval(s, st["a"][: p + 1])
    assert np.max(np.abs(Kt - Kp)) < 1e-12
    # the rank with tau = 0 is sum_k |H_k| L_k (Sec. 3.6 bound with L_k = (p-2k)/2 + 1)
    assert st["r"] == sum(harmonics.count(d, k) * (p // 2 - k + 1) for k in range(p // 2 + 1))


# ------------------------------------------------------- Q10 compression
def test_compression_eigs_two_routes():
    rng = np.random.default_rng(3)
    X = unit_ball(rng, 500, 4)
    st = hdf.build(X, "cauchy", 1.0, 1e-5)
    geo = st["geo"]
    rho = np.sqrt(geo["rho2"])
    t = hdf.cheb_arg(geo["rho2"], st["u0"], st["u1"])
    for dd in st["deg"]:
        k, L = dd["k"], dd["L"]
        Y = (rho ** k)[:, None] * hdf.cheb_basis(t, L)
        ev = np.linalg.eigvals(np.array(st["cores"][k]) @ (Y.T @ Y))
        ev = ev[np.argsort(-np.abs(ev))].real
        np.testing.assert_allclose(np.sort(dd["lam_all"]), np.sort(ev), atol=1e-12 * np.max(np.abs(ev)))
        Xb = dd["Xbar"]
        np.testing.assert_allclose(Xb.T @ Xb, np.eye(dd["s"]), atol=1e-12)
        # Xbar = Y E (the radial functions reproduce the orthonormal columns)
        np.testing.assert_allclose(Y @ dd["E"], Xb, atol=1e-10)


def test_dropped_degree_and_rank_formula():
    rng = np.random.default_rng(4)
    X = unit_ball(rng, 800, 3)
    st = hdf.build(X, "gaussian", 1.0, 1e-3)
    assert st["r"] == sum(harmonics.count(3, dd["k"]) * dd["s"] for dd in st["deg"])
    for dd in st["deg"]:
        assert np.all(np.abs(dd["lam"]) > st["tau"])
        assert np.all(np.abs(dd["lam_all"][dd["s"]:]) <= st["tau"])


# --------------------------------------------------------- Q11 guarantee
@pytest.mark.parametrize("d,name,l,tol,N", [
    (3, "gaussian", 1.0, 1e-6, 2000),
    (3, "matern32", 2.0, 1e-4, 800),
    (4, "cauchy", 1.0, 1e-5, 800),
    (5, "matern52", 1.0, 1e-3, 600),
    (5, "cauchy", 1.0, 1e-4, 600),
    (6, "gaussian", 2.0, 1e-6, 400),
])
def test_guarantee_against_dense(d, name, l, tol, N):
    rng = np.random.default_rng(100 + d)
    X = unit_ball(rng, N, d)
    st = hdf.build(X, name, l, tol)
    U, Dv = hdf.factor(st)
    K = dense.dense_K(X, name, l)
    err = dense.rel_fro_error(K, (U * Dv) @ U.T)
    assert err <= tol
    # nu estimates ||K||_F / N
    assert abs(st["nu"] * N / np.linalg.norm(K) - 1) < 0.05
    # matvec equals the explicit product
    V = rng.normal(size=(N, 3))
    np.testing.assert_allclose(hdf.matvec(st, V, U, Dv), ((U * Dv) @ U.T) @ V, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("N,chunk", [(1001, 128), (1001, 97), (37, 1), (600, 600), (600, 10_000)])
def test_chunked_matvec_and_passes(N, chunk):
    """The point-chunked, matrix-free product (U re-evaluated per chunk from the radial
    coefficients E) against the product of the assembled factor (columns Q W_s from the QR):
    element by element, every row, for ragged last chunks, one-point chunks, one chunk and a
    chunk longer than N.  A chunk boundary that drops, repeats or shifts rows fails here."""
    rng = np.random.default_rng(31)
    X = unit_ball(rng, N, 4)
    st = hdf.build(X, "gaussian", 0.7, 1e-5)
    U, Dv = hdf.factor(st)
    V = rng.normal(size=(N, 3))
    ref = hdf.matvec(st, V, U, Dv)
    got = hdf.matvec_chunked(st, V, chunk=chunk)
    assert got.shape == ref.shape
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.max(np.abs(ref)))
    P = hdf.passes(st, V, chunk=chunk)
    PU = U.T @ V
    np.testing.assert_allclose(P, PU, rtol=0, atol=1e-12 * np.max(np.abs(PU)))


def test_rank_vs_optimal_reported(capsys):
    rng = np.random.default_rng(8)
    X = unit_ball(rng, 1000, 3)
    st = hdf.build(X, "gaussian", 1.0, 1e-6)
    K = dense.dense_K(X, "gaussian", 1.0)
    ropt = dense.optimal_rank(K, 1e-6)
    print(f"HDF rank {st['r']} vs optimal {ropt}")
    assert st["r"] >= ropt


# --------------------------------------------------------- geometry / nu
def test_geometry_and_norm_scale():
    rng = np.random.default_rng(9)
    X = rng.normal(size=(300, 4)) * 3 + 1
    g = geometry.geometry(X)
    assert np.all(g["c"] == (X.min(0) + X.max(0)) / 2)
    assert np.isclose(g["R"], np.max(np.linalg.norm(X - g["c"], axis=1)), rtol=1e-15)
    assert np.isclose(g["rho2"].max(), 1.0, rtol=1e-14)
    from scipy.spatial.distance import pdist
    assert np.max(pdist(X)) <= g["D"] * (1 + 1e-15)
    # single point / coincident points: R = 0, rho = 0
    g1 = geometry.geometry(np.ones((5, 3)))
    assert g1["R"] == 0.0 and g1["u0"] == 0.0 and g1["u1"] == 1.0


def test_splitmix_reference_vectors():
    for row in _read_golden("splitmix64.txt"):
        gen = splitmix.SplitMix64(row[0])
        assert [gen.next() for _ in range(3)] == list(row[1:])


def test_norm_scale_constant_kernel():
    X = np.zeros((10, 3))
    assert splitmix.norm_scale(X, "gaussian", 1.0) == 1.0


# --------------------------------------------------------- Q14 gradients
@pytest.mark.parametrize("d,name", [(3, "gaussian"), (4, "gaussian"), (5, "matern52")])
def test_frozen_structure_gradients_fd(d, name):
    rng = np.random.default_rng(20 + d)
    X = unit_ball(rng, 200, d) * 1.2 - 0.3
    l = 1.5
    st = hdf.build(X, name, l, 1e-5)
    m = 2
    Wm = rng.normal(size=(200, m))
    Vm = rng.normal(size=(200, m))
    # lengthscale: analytic (coefficients of dk/dl) vs central differences
    h = 1e-4
    Cp = hdf.core_blocks(st, chebyshev.cheb_coeffs(name, st["D"], l + h))
    Cm = hdf.core_blocks(st, chebyshev.cheb_coeffs(name, st["D"], l - h))
    fd = (hdf.objective(st, X, Wm, Vm, Cp) - hdf.objective(st, X, Wm, Vm, Cm)) / (2 * h)
    g = hdf.grad_l(st, Wm, Vm)
    assert abs(g - fd) <= 1e-7 * max(1.0, abs(g))
    # at the build point C_k = diag(lambda_k)
    C0 = hdf.core_blocks(st, st["a"])
    for dd in hdf.kept_degrees(st):
        np.testing.assert_allclose(C0[dd["k"]], np.diag(dd["lam"]), atol=1e-9 * np.max(np.abs(dd["lam"])))
    # points: complex-step gradient vs central differences along a direction
    G = hdf.grad_x(st, Wm, Vm)
    dX = rng.normal(size=X.shape)
    fd = (hdf.objective(st, X + h * dX, Wm, Vm) - hdf.objective(st, X - h * dX, Wm, Vm)) / (2 * h)
    assert abs(np.sum(G * dX) - fd) <= 1e-7 * max(1.0, np.sum(np.abs(G * dX)))
    for _ in range(8):
        i, j = rng.integers(0, 200), rng.integers(0, d)
        e = np.zeros_like(X)
        e[i, j] = h
        fd = (hdf.objective(st, X + e, Wm, Vm) - hdf.objective(st, X - e, Wm, Vm)) / (2 * h)
        assert abs(G[i, j] - fd) <= 1e-6 * max(1.0, abs(G[i, j]))


def test_gradients_vs_dense_closed_form():
    rng = np.random.default_rng(31)
    N, d = 600, 4
    X = rng.uniform(-1, 1, size=(N, d))
    l = 0.7
    st = hdf.build(X, "gaussian", l, 1e-7)
    w = rng.normal(size=N)
    v = rng.normal(size=N)
    gl = hdf.grad_l(st, w[:, None], v[:, None])
    gl_dense = dense.dense_grad_l(X, "gaussian", l, w, v)
    assert abs(gl - gl_dense) <= 1e-4 * abs(gl_dense)
    G = hdf.grad_x(st, w[:, None], v[:, None])
    Gd = dense.dense_grad_x(X, "gaussian", l, w, v)
    assert np.linalg.norm(G - Gd) <= 1e-3 * np.linalg.norm(Gd)


# ----------------------------------------------- Q17 general case X != Y
@pytest.mark.parametrize("d,name,l,tol", [(3, "gaussian", 1.0, 1e-6), (4, "cauchy", 1.0, 1e-4),
                                          (5, "matern52", 2.0, 1e-5)])
def test_cross_with_y_equal_x_is_the_symmetric_factor(d, name, l, tol):
    # R_x M R_y^T is then symmetric, its singular values are |lambda| and
    # U V^T = U D U^T: same degree, threshold, ranks and approximation
    rng = np.random.default_rng(40 + d)
    X = unit_ball(rng, 300, d)
    st = hdf.build(X, name, l, tol)
    sc = cross.build_cross(X, X, name, l, tol)
    assert sc["p"] == st["p"] and sc["nu"] == st["nu"]
    assert abs(sc["tau"] / st["tau"] - 1) < 1e-15
    for dc, ds in zip(sc["deg"], st["deg"]):
        np.testing.assert_allclose(dc["sig_all"], np.sort(np.abs(ds["lam_all"]))[::-1],
                                   atol=1e-12 * np.max(np.abs(ds["lam_all"])))
        assert dc["s"] == ds["s"]
    U, Dv = hdf.factor(st)
    Ux, Vy = cross.factor_cross(sc)
    Ks = (U * Dv) @ U.T
    assert np.max(np.abs(Ux @ Vy.T - Ks)) <= 1e-12 * np.max(np.abs(Ks))


@pytest.mark.parametrize("d,name", [(3, "gaussian"), (4, "matern32"), (6, "cauchy")])
def test_cross_uncompressed_reproduces_chebyshev_kernel(d, name):
    # tau = 0 keeps every singular value: U V^T is the degree-p Chebyshev
    # kernel between the two sets (different sizes and distributions)
    rng = np.random.default_rng(50 + d)
    X = unit_ball(rng, 90, d) * 1.3 + 0.2
    Y = rng.uniform(-1.0, 1.0, size=(70, d))
    p = 10
    sc = cross.build_cross(X, Y, name, 1.0, 1e-6, p=p, tau=0.0)
    Ux, Vy = cross.factor_cross(sc)
    from scipy.spatial.distance import cdist
    Kp = npcheb.chebval(cdist(X, Y) / sc["D"], sc["a"][: p + 1])
    assert np.max(np.abs(Ux @ Vy.T - Kp)) < 1e-12
    assert sc["r"] == sum(harmonics.count(d, k) * (p // 2 - k + 1) for k in range(p // 2 + 1))


@pytest.mark.parametrize("d,name,l,tol,nx,ny", [
    (3, "gaussian", 1.0, 1e-6, 900, 500),
    (4, "cauchy", 1.0, 1e-5, 700, 400),
    (5, "matern52", 1.0, 1e-3, 500, 600),
])
def test_cross_guarantee_against_dense(d, name, l, tol, nx, ny, capsys):
    rng = np.random.default_rng(60 + d)
    X = unit_ball(rng, nx, d)                               # training-like set
    Y = unit_ball(rng, ny, d) * 0.8 + 0.1                   # shifted query set
    sc = cross.build_cross(X, Y, name, l, tol)
    Ux, Vy = cross.factor_cross(sc)
    K = dense.dense_K_cross(X, Y, name, l)
    assert dense.rel_fro_error(K, Ux @ Vy.T) <= tol
    # nu estimates ||K(X, Y)||_F / sqrt(N_x N_y)
    assert abs(sc["nu"] * np.sqrt(nx * ny) / np.linalg.norm(K) - 1) < 0.05
    W = rng.normal(size=(ny, 2))
    np.testing.assert_allclose(cross.matvec_cross(sc, W, Ux, Vy), (Ux @ Vy.T) @ W, rtol=1e-11, atol=1e-11)
    # every kept singular value is above tau, every dropped one at or below
    for dd in sc["deg"]:
        assert np.all(dd["sig"] > sc["tau"]) and np.all(dd["sig_all"][dd["s"]:] <= sc["tau"])
    ropt = dense.optimal_rank_cross(K, tol)
    print(f"cross rank {sc['r']} vs optimal {ropt}")
    assert sc["r"] >= ropt


def test_norm_scale_cross_reduces_to_symmetric():
    rng = np.random.default_rng(70)
    X = rng.normal(size=(250, 4))
    assert splitmix.norm_scale_cross(X, X, "cauchy", 1.3) == splitmix.norm_scale(X, "cauchy", 1.3)
