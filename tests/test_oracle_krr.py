"""Pins of the KRR consumer oracle (oracle/krr.py, Sec. 4.2).

- k-means: from the same initial centres, scikit-learn's Lloyd iteration
  reaches the same labels and centres; the result is a Lloyd fixed point
  (every point at its nearest centre by scipy's cdist, every centre the mean
  of its members); the objective never rises; well-separated blobs are
  recovered exactly; the initial indices are distinct and follow SplitMix64.
- PCG: its k-th iterate equals scipy's CG iterate after k steps (the Krylov
  minimiser is unique); an exact preconditioner converges in one iteration;
  with M = I, a matrix with three distinct eigenvalues converges in three;
  the stopping rule and the true residual agree with the recursive one.
- System operator: against the dense (lambda I + K) v the difference is
  bounded by the HDF blocks' Frobenius guarantee, and the off-diagonal part
  is exact (checked against the dense matrix with the blocks cut out).
- Preconditioner: multiplying its output by the dense blocks gives back r.
- Solve and predictions: with blocks at a tiny tolerance, w matches
  numpy.linalg.solve of the dense system, and predictions match K(x*, x) w.
"""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import dense, krr, splitmix
from paper_2202_03655_amd import workloads as wl


def test_init_centres_follow_splitmix_and_are_distinct():
    idx = krr.init_centres(np.zeros((7, 3)), 7, seed=5)
    assert sorted(idx.tolist()) == list(range(7))
    g = splitmix.SplitMix64(5)
    first = (g.next() >> 11) % 7
    assert idx[0] == first
    with pytest.raises(ValueError):
        krr.init_centres(np.zeros((3, 3)), 4)


def test_kmeans_matches_sklearn_lloyd_from_the_same_start():
    from sklearn.cluster import KMeans
    X, _, _, _ = wl.housing_split(3000)
    k = 12
    labels, C, its, hist = krr.kmeans(X, k, max_iter=300)
    init = X[krr.init_centres(X, k)]
    ref = KMeans(k, init=init, n_init=1, max_iter=300, tol=0.0, algorithm="lloyd").fit(X)
    assert np.array_equal(labels, ref.labels_)
    np.testing.assert_allclose(C, ref.cluster_centers_, rtol=0, atol=1e-12)


def test_kmeans_result_is_a_lloyd_fixed_point_and_objective_decreases():
    X = wl.unit_ball(1500, 4, 3)
    labels, C, its, hist = krr.kmeans(X, 9, max_iter=500)
    assert its < 500
    D = cdist(X, C, "sqeuclidean")
    best = D.min(axis=1)
    assert np.all(D[np.arange(len(X)), labels] <= best * (1 + 1e-12) + 1e-300)
    for c in range(9):
        np.testing.assert_allclose(C[c], X[labels == c].mean(axis=0), rtol=0, atol=1e-14)
    assert all(b <= a * (1 + 1e-14) for a, b in zip(hist, hist[1:]))


def test_kmeans_recovers_separated_blobs():
    rng = np.random.default_rng(4)
    centres = np.array([[0, 0, 0], [10, 0, 0], [0, 10, 0], [0, 0, 10]], dtype=float)
    truth = np.repeat(np.arange(4), 50)
    X = centres[truth] + 0.3 * rng.normal(size=(200, 3))
    # a start with one seed in each blob
    labels, C, its, _ = krr.kmeans(X, 4, seed=next(s for s in range(1000)
                                                   if len(set(truth[krr.init_centres(X, 4, s)])) == 4))
    for t in range(4):
        assert len(set(labels[truth == t])) == 1
    assert len(set(labels)) == 4


def test_cluster_order_is_stable():
    labels = np.array([2, 0, 2, 1, 0, 2])
    perm, off = krr.cluster_order(labels, 4)
    assert perm.tolist() == [1, 4, 3, 0, 2, 5] and off.tolist() == [0, 2, 3, 6, 6]


def _spd(n, seed, cond=1e3):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    return (Q * np.geomspace(1.0, cond, n)) @ Q.T


def test_pcg_iterates_equal_scipy_cg():
    from scipy.sparse.linalg import cg
    A = _spd(60, 1)
    Minv = np.diag(1.0 / np.diag(A))
    b = np.random.default_rng(2).normal(size=60)
    for k in (1, 4, 9):
        x, it, _ = krr.pcg(lambda v: A @ v, lambda r: Minv @ r, b, 0.0, k)
        assert it == k
        xs, _ = cg(A, b, x0=np.zeros(60), rtol=1e-300, atol=0.0, maxiter=k, M=Minv)
        np.testing.assert_allclose(x, xs, rtol=0, atol=1e-10 * np.linalg.norm(xs))


def test_pcg_special_cases():
    A = _spd(40, 3)
    b = np.random.default_rng(5).normal(size=40)
    x, it, hist = krr.pcg(lambda v: A @ v, lambda r: np.linalg.solve(A, r), b, 1e-10, 50)
    assert it == 1 and hist[0] <= 1e-10
    rng = np.random.default_rng(6)
    Q, _ = np.linalg.qr(rng.normal(size=(40, 40)))
    A3 = (Q * np.repeat([1.0, 3.0, 7.0], [10, 15, 15])) @ Q.T
    x, it, hist = krr.pcg(lambda v: A3 @ v, lambda r: r, b, 1e-10, 50)
    assert it <= 3 and hist[-1] <= 1e-10
    np.testing.assert_allclose(A3 @ x, b, rtol=0, atol=1e-9 * np.linalg.norm(b))
    x, it, hist = krr.pcg(lambda v: A @ v, lambda r: r, np.zeros(40), 1e-6, 10)
    assert it == 0 and not np.any(x)


def test_pcg_stops_at_the_first_small_residual():
    A = _spd(80, 7, cond=1e4)
    b = np.random.default_rng(8).normal(size=80)
    x, it, hist = krr.pcg(lambda v: A @ v, lambda r: r, b, 1e-6, 500)
    assert hist[-1] <= 1e-6 and all(h > 1e-6 for h in hist[:-1]) and len(hist) == it
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-5


def _small_system(tol, d=3, n=900, k=6, lam=0.1, kernel="gaussian", l=0.8):
    X = wl.unit_ball(n, d, 12) if d == 3 else wl.housing_split(n)[0]
    labels, _, _, _ = krr.kmeans(X, k)
    return X, labels, krr.create(X, labels, k, kernel, l, tol, lam)


def test_operator_within_the_block_guarantee_and_offdiag_exact():
    tol = 1e-6
    X, labels, S = _small_system(tol)
    K = dense.dense_K(X, "gaussian", 0.8)
    v = np.random.default_rng(9).normal(size=len(X))
    same = labels[:, None] == labels[None, :]
    np.testing.assert_allclose(krr.offdiag_apply(S, v), np.where(same, 0.0, K) @ v,
                               rtol=0, atol=1e-13 * np.abs(K).sum(axis=1).max() * np.abs(v).max())
    diff = krr.apply(S, v) - (0.1 * v + K @ v)
    bound = sum(tol * np.linalg.norm(K[np.ix_(labels == c, labels == c)]) * np.linalg.norm(v[labels == c])
                for c in range(6))
    assert np.linalg.norm(diff) <= bound
    assert np.linalg.norm(diff) > 0


def test_preconditioner_inverts_the_dense_blocks():
    X, labels, S = _small_system(1e-4)
    K = dense.dense_K(X, "gaussian", 0.8)
    r = np.random.default_rng(10).normal(size=len(X))
    z = krr.precond(S, r)
    back = np.zeros_like(r)
    for c in range(6):
        m = labels == c
        back[m] = (K[np.ix_(m, m)] + 0.1 * np.eye(m.sum())) @ z[m]
    np.testing.assert_allclose(back, r, rtol=0, atol=1e-11 * np.abs(r).max())


def test_solve_and_predict_match_dense_krr():
    X, labels, S = _small_system(1e-10)
    y = np.sin(3 * X[:, 0]) + X[:, 1] * X[:, 2]
    w, it, hist = krr.solve(S, y, 1e-10, 500)
    K = dense.dense_K(X, "gaussian", 0.8)
    w_ref = np.linalg.solve(K + 0.1 * np.eye(len(X)), y)
    assert hist[-1] <= 1e-10
    assert np.linalg.norm(w - w_ref) <= 1e-6 * np.linalg.norm(w_ref)
    Xq = wl.unit_ball(200, 3, 13)
    np.testing.assert_allclose(krr.predict(X, Xq, w, "gaussian", 0.8),
                               dense.dense_K_cross(Xq, X, "gaussian", 0.8) @ w, rtol=0, atol=1e-12 * np.abs(w).sum())


def test_housing_blocks_in_d8():
    """The d = 8 housing-shaped cloud: each block meets its tolerance against the dense block."""
    X, labels, S = _small_system(1e-4, d=8, n=1500, k=5, l=0.5)
    K = dense.dense_K(X, "gaussian", 0.5)
    for b in S["blocks"]:
        Kb = K[np.ix_(b["idx"], b["idx"])]
        E = np.eye(len(b["idx"]))
        from oracle import hdf
        Kt = hdf.matvec(b["st"], E)
        assert np.linalg.norm(Kt - Kb) <= 1e-4 * np.linalg.norm(Kb)
