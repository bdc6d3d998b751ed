"""Kernel ridge regression with HDF diagonal blocks (oracle, test infrastructure).

Sec. 4.2: the weights solve (lambda I + K) w = y (Eq. opt) by conjugate
gradients.  The training points are split into k-means clusters C_i; each
diagonal block K_{C_i C_i} is replaced by its HDF factor, the off-diagonal
blocks stay exact, and the preconditioner is block diagonal with the inverses
of the exact blocks.  Predictions are K(x*, x) w.

Readings taken where the paper is silent:
- k-means is Lloyd's iteration.  The k initial centres are distinct training
  points drawn with SplitMix64 (seed KMEANS_SEED unless given): index
  (u >> 11) mod n, a repeated index skipped.  A point goes to the centre of
  smallest squared distance sum_j (x_j - c_j)^2, ties to the lower index; a
  centre becomes the mean of its members, an empty cluster keeps its centre.
  The iteration stops at the first assignment that changes no label, or after
  max_iter assignments.
- The preconditioner blocks are those of the system matrix, lambda I +
  K_{C_i C_i}, inverted exactly.
- Preconditioned CG from w_0 = 0 in its textbook form (Saad, Iterative Methods
  for Sparse Linear Systems, Alg. 9.1), stopped at the first iteration whose
  recursive residual has ||r|| <= rtol ||y||, or after max_iter iterations.
- Vectors passed in and out are in the caller's point order.

Every value here comes from plain definitions: explicit cluster means, the
oracle's HDF factors (hdf.py) applied block by block, the dense kernel for the
off-diagonal blocks, Cholesky solves for the preconditioner.
"""
import numpy as np
from scipy.linalg import cho_factor, cho_solve
from scipy.spatial.distance import cdist

from . import hdf, splitmix
from .kernels import kappa

KMEANS_SEED = 0x48444602


def init_centres(X, k, seed=KMEANS_SEED):
    """Indices of the k distinct initial centres."""
    n = X.shape[0]
    if k > n:
        raise ValueError("more clusters than points")
    g = splitmix.SplitMix64(seed)
    idx, seen = [], set()
    while len(idx) < k:
        i = (g.next() >> 11) % n
        if i not in seen:
            seen.add(i)
            idx.append(i)
    return np.array(idx, dtype=np.int64)


def assign(X, C):
    """Nearest centre of every point (squared distance summed over coordinates in order, ties to the
    lower index) and the squared distances to all centres."""
    n, d = X.shape
    D2 = np.zeros((n, C.shape[0]))
    for j in range(d):
        t = X[:, j][:, None] - C[:, j][None, :]
        D2 = D2 + t * t
    return np.argmin(D2, axis=1), D2


def kmeans(X, k, max_iter=100, seed=KMEANS_SEED):
    """Lloyd's iteration.  Returns labels, centres, the number of assignments made and the objective
    (sum of squared distances to the assigned centre) after each assignment."""
    X = np.asarray(X, dtype=np.float64)
    C = X[init_centres(X, k, seed)].copy()
    labels, history, its = None, [], 0
    for _ in range(max_iter):
        new, D2 = assign(X, C)
        its += 1
        history.append(float(D2[np.arange(len(X)), new].sum()))
        if labels is not None and np.array_equal(new, labels):
            break
        labels = new
        for c in range(k):
            members = labels == c
            if members.any():
                C[c] = X[members].mean(axis=0)
    return labels, C, its, history


def cluster_order(labels, k):
    """Stable order of the points by cluster: perm[p] is the caller index at position p, and cluster c
    occupies positions offsets[c] .. offsets[c+1]-1."""
    perm = np.argsort(labels, kind="stable")
    offsets = np.concatenate([[0], np.cumsum(np.bincount(labels, minlength=k))])
    return perm, offsets


def create(X, labels, k, kernel, l, tol, lam):
    """System state: the HDF factor of every non-empty diagonal block and the Cholesky factor of every
    preconditioner block lambda I + K_{C_i C_i}."""
    X = np.asarray(X, dtype=np.float64)
    perm, offsets = cluster_order(labels, k)
    blocks = []
    for c in range(k):
        idx = perm[offsets[c]:offsets[c + 1]]
        if len(idx) == 0:
            blocks.append(None)
            continue
        Xc = X[idx]
        st = hdf.build(Xc, kernel, l, tol)
        B = kappa(kernel, cdist(Xc, Xc), l) + lam * np.eye(len(idx))
        blocks.append(dict(idx=idx, st=st, chol=cho_factor(B, lower=True)))
    return dict(X=X, labels=np.asarray(labels), k=k, kernel=kernel, l=l, tol=tol, lam=lam,
                perm=perm, offsets=offsets, blocks=blocks)


def offdiag_apply(S, v, rows=None, chunk=1024):
    """sum over j outside the cluster of i of k(||x_i - x_j||) v_j, for the given rows (all if None)."""
    X, lab = S["X"], S["labels"]
    rows = np.arange(len(X)) if rows is None else np.asarray(rows)
    out = np.zeros(len(rows))
    for s in range(0, len(rows), chunk):
        r = rows[s:s + chunk]
        Kr = kappa(S["kernel"], cdist(X[r], X), S["l"])
        Kr[lab[r][:, None] == lab[None, :]] = 0.0
        out[s:s + chunk] = Kr @ v
    return out


def apply(S, v):
    """(lambda I + blockdiag(K~_{C_i C_i}) + offdiag(K)) v."""
    v = np.asarray(v, dtype=np.float64)
    out = S["lam"] * v + offdiag_apply(S, v)
    for b in S["blocks"]:
        if b is not None:
            out[b["idx"]] += hdf.matvec(b["st"], v[b["idx"]][:, None])[:, 0]
    return out


def precond(S, r):
    """blockdiag((lambda I + K_{C_i C_i})^{-1}) r."""
    z = np.zeros_like(np.asarray(r, dtype=np.float64))
    for b in S["blocks"]:
        if b is not None:
            z[b["idx"]] = cho_solve(b["chol"], r[b["idx"]])
    return z


def pcg(A, M, b, rtol, max_iter):
    """Preconditioned CG from x0 = 0.  A and M are callables.  Returns x, the number of iterations and
    the relative recursive residual after each iteration."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0, []
    r = b.copy()
    z = M(r)
    p = z.copy()
    rz = r @ z
    hist = []
    it = 0
    while it < max_iter:
        q = A(p)
        alpha = rz / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        hist.append(float(np.linalg.norm(r) / bn))
        if hist[-1] <= rtol:
            break
        z = M(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, hist


def solve(S, y, rtol, max_iter):
    return pcg(lambda v: apply(S, v), lambda r: precond(S, r), y, rtol, max_iter)


def predict(X, Xq, w, kernel, l, chunk=1024):
    """K(x*, x) w with the exact kernel."""
    X, Xq = np.asarray(X, dtype=np.float64), np.asarray(Xq, dtype=np.float64)
    out = np.zeros(len(Xq))
    for s in range(0, len(Xq), chunk):
        out[s:s + chunk] = kappa(kernel, cdist(Xq[s:s + chunk], X), l) @ w
    return out
