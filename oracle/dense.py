"""Dense references (oracle, test infrastructure).

The kernel matrix K_ij = k(||x_i - x_j||) (Sec. 1) formed explicitly, the
relative Frobenius error of an approximation, and the optimal rank from the
eigendecomposition of K (the SVD reference of Sec. 2 and Fig. 3: by
Eckart-Young the best rank-r approximation of a symmetric matrix keeps the r
eigenvalues of largest magnitude).  Also the closed-form gradients of
w^T K v with respect to the lengthscale and the points.
"""
import numpy as np
from scipy.spatial.distance import cdist

from .kernels import kappa, dkappa_dl, dkappa_dr


def dense_K(X, name, l):
    X = np.asarray(X, dtype=np.float64)
    return kappa(name, cdist(X, X), l)


def dense_K_cross(X, Y, name, l):
    """K(X, Y)_ij = k(||x_i - y_j||)."""
    return kappa(name, cdist(np.asarray(X, dtype=np.float64), np.asarray(Y, dtype=np.float64)), l)


def optimal_rank_cross(K, eps):
    """Smallest r with ||K - K_r||_F <= eps ||K||_F (Eckart-Young, SVD)."""
    sv = np.sort(np.linalg.svd(K, compute_uv=False))      # ascending
    tail = np.sqrt(np.cumsum(sv ** 2))
    budget = eps * np.linalg.norm(sv)
    dropped = int(np.searchsorted(tail, budget, side="right"))
    return len(sv) - dropped


def rel_fro_error(K, Kt):
    return float(np.linalg.norm(K - Kt) / np.linalg.norm(K))


def optimal_rank(K, eps):
    """Smallest r with ||K - K_r||_F <= eps ||K||_F (Eckart-Young, eigh)."""
    lam = np.linalg.eigvalsh(K)
    mags = np.sort(np.abs(lam))            # ascending
    total = np.sum(mags ** 2)
    tail = np.cumsum(mags ** 2)            # tail[i] = energy of the i+1 smallest
    budget = (eps ** 2) * total
    # drop the largest number of smallest eigenvalues within budget
    n_drop = int(np.searchsorted(tail, budget, side="right"))
    return len(lam) - n_drop


def dense_grad_l(X, name, l, w, v):
    """d/dl of w^T K v = sum_ij w_i v_j dk/dl(r_ij)."""
    X = np.asarray(X, dtype=np.float64)
    return float(w @ dkappa_dl(name, cdist(X, X), l) @ v)


def dense_grad_x(X, name, l, w, v):
    """d/dx_i of w^T K v = sum_{j != i} (w_i v_j + w_j v_i) k'(r_ij) (x_i - x_j) / r_ij."""
    X = np.asarray(X, dtype=np.float64)
    r = cdist(X, X)
    with np.errstate(divide="ignore", invalid="ignore"):
        g = dkappa_dr(name, r, l) / r
    np.fill_diagonal(g, 0.0)
    Wt = np.outer(w, v) + np.outer(v, w)
    G = Wt * g
    return G.sum(axis=1)[:, None] * X - G @ X
