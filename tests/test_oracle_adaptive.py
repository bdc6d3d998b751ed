"""Pins of the sampled degree and rank rules (oracle/adaptive.py).

- With every one of the N^2 pairs, the sampled error is the exact relative
  Frobenius error of the factor (dense K and dense U D U^T) and of the
  degree-p Chebyshev truncation (dense K_p built entry by entry).
- The addition theorem used for per-pair harmonic sums matches explicit sums
  of the orthonormal solid harmonics for d = 3..8.
- The tuned factor meets the tolerance against the dense K, keeps a subset of
  the budget factor's eigenpairs and does not raise the degree.
"""
import numpy as np
import pytest

from oracle import adaptive, chebyshev, dense, harmonics, hdf
from oracle.kernels import kappa
from paper_2202_03655_amd import workloads as wl


def all_pairs(N):
    return np.repeat(np.arange(N), N), np.tile(np.arange(N), N)


def test_sampled_error_over_all_pairs_is_the_frobenius_error():
    X = wl.unit_ball(40, 3, 7)
    N = 40
    st = hdf.build(X, "gaussian", 1.0, 1e-3)
    a, b = all_pairs(N)
    c, pairs = adaptive.pair_contributions(st, a, b)
    U, Dv = hdf.features(st, X)
    Kt = (U * Dv) @ U.T
    np.testing.assert_allclose(c.sum(axis=1).reshape(N, N), Kt, rtol=0, atol=1e-13 * np.abs(Kt).max())
    K = dense.dense_K(X, "gaussian", 1.0)
    exact = np.linalg.norm(K - Kt) / np.linalg.norm(K)
    e = adaptive.sampled_error(K.reshape(-1), c.sum(axis=1))
    assert abs(e - exact) <= 1e-12 * e
    # stratified: every off-diagonal pair and every diagonal point
    off = a != b
    cd, _ = adaptive.pair_contributions(st, np.arange(N), np.arange(N))
    es = adaptive.stratified_error(N, K.reshape(-1)[off], c.sum(axis=1)[off], np.diag(K), cd.sum(axis=1))
    assert abs(es - exact) <= 1e-12 * exact
    assert len(pairs) == c.shape[1] == sum(dd["s"] for dd in st["deg"])


@pytest.mark.parametrize("kernel,l", [("gaussian", 0.7), ("cauchy", 1.0), ("matern52", 2.0)])
def test_sampled_truncation_error_over_all_pairs(kernel, l):
    X = wl.uniform_cube(30, 4, 3)
    N = len(X)
    D = 2.0 * np.max(np.linalg.norm(X - 0.5 * (X.max(0) + X.min(0)), axis=1))
    a_coef = chebyshev.cheb_coeffs(kernel, D, l)
    r = np.linalg.norm(X[:, None, :] - X[None, :, :], axis=2)
    K = kappa(kernel, r, l)
    for p in (2, 6, 12):
        Kp = np.zeros_like(K)
        for i in range(N):
            for j in range(N):
                s = r[i, j] / D
                Tm, T = 1.0, s
                acc = a_coef[0] + (a_coef[1] * s if p >= 1 else 0.0)
                for q in range(2, p + 1):
                    Tm, T = T, 2 * s * T - Tm
                    acc += a_coef[q] * T
                Kp[i, j] = acc
        e = adaptive.sampled_error(K.reshape(-1), adaptive.cheb_partial(a_coef, r.reshape(-1) / D, p))
        assert abs(e - np.linalg.norm(K - Kp) / np.linalg.norm(K)) <= 1e-10 * max(e, 1e-300)


@pytest.mark.parametrize("d", [3, 4, 5, 6, 7, 8])
def test_addition_theorem_matches_explicit_harmonics(d):
    rng = np.random.default_rng(d)
    x = rng.normal(size=(5, d)) * 0.4
    y = rng.normal(size=(5, d)) * 0.4
    K = 6
    Sx = harmonics.solid_harmonics(x, K)
    Sy = harmonics.solid_harmonics(y, K)
    ra, rb = np.linalg.norm(x, axis=1), np.linalg.norm(y, axis=1)
    cosg = np.sum(x * y, axis=1) / (ra * rb)
    for k in range(K + 1):
        explicit = np.sum(Sx[k] * Sy[k], axis=1)
        formula = adaptive.addition_sum(d, k, ra, rb, cosg)
        np.testing.assert_allclose(explicit, formula, rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("case", [
    ("ball3_gauss", lambda: wl.unit_ball(1500, 3, 101), "gaussian", 1.0, 1e-5),
    ("cube4_gauss", lambda: wl.uniform_cube(1200, 4, 104), "gaussian", 0.7, 1e-4),
    ("gmm5_cauchy", lambda: wl.max_norm_one(wl.gaussian_mixture(1500, 5, 103)), "cauchy", 1.0, 1e-3),
], ids=lambda c: c[0])
def test_tuned_factor_meets_tolerance_with_smaller_rank(case):
    name, gen, kernel, l, tol = case
    X = gen()
    st = adaptive.build_sampled(X, kernel, l, tol)
    base = hdf.build(X, kernel, l, tol)
    K = dense.dense_K(X, kernel, l)
    U, Dv = hdf.features(st, X)
    err = np.linalg.norm(K - (U * Dv) @ U.T) / np.linalg.norm(K)
    print(f"{name}: p {st['p']} (bound {base['p']}), rank {st['r']} (bound {base['r']}), "
          f"tau {st['tau']:.3e} (tau0 {st['tau0']:.3e}), est {st['est_error']:.2e}, true {err:.2e}")
    assert err <= tol
    assert st["p"] <= base["p"] and st["p_bound"] == base["p"]
    assert st["tau"] >= st["tau0"]
    if st["p"] == base["p"]:
        for dd, db in zip(st["deg"], base["deg"]):
            assert dd["s"] <= db["s"]
    assert abs(st["est_error"] - err) <= 0.15 * err + 1e-3 * tol
