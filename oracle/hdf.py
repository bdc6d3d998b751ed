"""Algorithm 1 (HDF), symmetric case (oracle, test infrastructure).

Steps, in the paper's order:

1. p <- ChebDegreeNeeded, a <- ChebyshevTransform (Algorithm 1; chebyshev.py)
   after the diameter normalisation (geometry.py) and the ||K||_F estimate
   (splitmix.py).
2. Per degree k = 0..p/2 (Sec. 3.4): the radial matrix R^{(k)} = Y_k M_k Y_k^T
   with Y_k[i, a] = rho_i^k phi_a(rho_i^2) (Eq. vandermonde, in the
   Chebyshev radial basis of expansion.py), QR of Y_k, and for X = Y (Remark 1)
   the eigendecomposition of R_Y M_k R_Y^T in place of the SVD (Eq. svd).
   Eigenvalues with |lambda| <= tau are dropped (Eq. rapprox); a degree whose
   every eigenvalue is dropped disappears (Remark 2).
3. Factor assembly (Algorithm 1, inner loops): column (k, h, l) of U is
   Y_k^h(x_i) * Xbar_k[i, l] with Xbar_k = Q_k W_s (Algorithm 1 writes
   Xbar^{(k)} without the column index l); D = diag(lambda).  K ~ U D U^T.
4. Matvec in O(N r) (Sec. 3.6): K V ~ U (D (U^T V)).

Threshold tau (reading of Sec. 3.5): the paper's entrywise bound
sqrt(N) C_{p/2} tau is restated in Frobenius form.  |sum_h Y_k^h(x)Y_k^h(y)|
<= |H_k| / |S^{d-1}| (addition theorem at cos g = 1), dropping eigenvalues
below tau leaves ||dR_k||_F <= sqrt(L_k) tau, so with
tau = (eps nu N / 2) / sum_k (|H_k| / |S^{d-1}|) sqrt(L_k) the compression
error is at most eps nu N / 2, and the Chebyshev tail adds at most another
eps nu N / 2 (chebyshev.py).

Eigenvector conventions (a reading: the paper does not fix them): order by
|lambda| descending, ties to lambda > 0 first, then lower index; the sign of
each kept radial function is chosen so that its largest-magnitude coefficient
in the phi basis (lowest index on ties) is positive.

Derivatives (the paper does not differentiate): F(X, l) = sum_c w_c^T
Kt(X, l) v_c with the structure frozen at the build (c, R, p, [u0, u1], s_k,
the radial coefficients).  l enters through C_k(l) = E'_k^T M_k(a(l)) E'_k,
which equals diag(lambda_k) at the build; X enters through U(X).
"""
import numpy as np

from . import chebyshev, expansion, geometry, harmonics, splitmix


class Infeasible(Exception):
    pass


def cheb_basis(t, L):
    """[T_0(t), ..., T_{L-1}(t)] as columns (three-term recurrence)."""
    t = np.asarray(t)
    out = np.empty(t.shape + (L,), dtype=t.dtype)
    if L > 0:
        out[..., 0] = 1.0
    if L > 1:
        out[..., 1] = t
    for a in range(2, L):
        out[..., a] = 2.0 * t * out[..., a - 1] - out[..., a - 2]
    return out


def cheb_arg(rho2, u0, u1):
    return (2.0 * rho2 - u0 - u1) / (u1 - u0)


def tau_threshold(tol, nu, N, d, p):
    K = p // 2
    area = harmonics.sphere_area(d)
    denom = 0.0
    for k in range(K + 1):
        denom += harmonics.count(d, k) / area * np.sqrt(K - k + 1)
    return (tol * nu * N / 2.0) / denom


def _order(lam):
    idx = np.arange(len(lam))
    return np.lexsort((idx, (lam < 0).astype(int), -np.abs(lam)))


def _sign_pivot(e):
    mags = np.abs(e)
    j = int(np.argmax(mags))
    return j


def build(X, kernel, l, tol, p=None, tau=None):
    """Run the HDF on points X (N x d) and return a dict describing the factor.

    ``p`` / ``tau`` override the automatic choices (testing aids).
    """
    X = np.asarray(X, dtype=np.float64)
    N, d = X.shape
    if d < 3:
        raise ValueError("d >= 3 required")
    geo = geometry.geometry(X)
    nu = splitmix.norm_scale(X, kernel, l)
    a = chebyshev.cheb_coeffs(kernel, geo["D"], l)
    tail_at_p = None
    if p is None:
        p, tail_at_p, thr = chebyshev.choose_degree(a, tol, nu)
        if p is None:
            raise Infeasible("Chebyshev degree above the maximum")
    K = p // 2
    u0, u1 = geo["u0"], geo["u1"]
    cores = [np.array(M) for M in expansion.radial_cores(a, p, d, u0, u1)]
    if tau is None:
        tau = tau_threshold(tol, nu, N, d, p)
    rho2 = geo["rho2"]
    rho = np.sqrt(rho2)
    t = cheb_arg(rho2, u0, u1)
    deg = []
    for k in range(K + 1):
        L = K - k + 1
        Y = (rho ** k)[:, None] * cheb_basis(t, L)
        Q, Rr = np.linalg.qr(Y)                 # Householder QR (LAPACK)
        A = Rr @ cores[k] @ Rr.T
        A = (A + A.T) / 2.0
        lam, W = np.linalg.eigh(A)
        order = _order(lam)
        lam, W = lam[order], W[:, order]
        keep = np.abs(lam) > tau
        lam_s, W_s = lam[keep], W[:, keep]
        E = np.linalg.pinv(Rr, rcond=1e-15) @ W_s
        Ep = Rr.T @ W_s
        for c in range(E.shape[1]):
            j = _sign_pivot(E[:, c])
            if E[j, c] < 0:
                E[:, c] *= -1.0
                Ep[:, c] *= -1.0
                W_s[:, c] *= -1.0
        deg.append(dict(k=k, L=L, lam_all=lam, lam=lam_s, s=int(keep.sum()),
                        E=E, Ep=Ep, Xbar=Q @ W_s))
    st = dict(X=X, N=N, d=d, kernel=kernel, l=l, tol=tol, nu=nu, a=a, p=p, K=K,
              tail_at_p=tail_at_p, tau=tau, geo=geo, c=geo["c"], R=geo["R"],
              Reff=geo["Reff"], D=geo["D"], u0=u0, u1=u1, cores=cores, deg=deg)
    st["r"] = sum(harmonics.count(d, dd["k"]) * dd["s"] for dd in deg)
    st["H"] = sum(harmonics.count(d, dd["k"]) for dd in deg if dd["s"] > 0)
    st["S"] = sum(dd["s"] for dd in deg)
    return st


def kept_degrees(st):
    return [dd for dd in st["deg"] if dd["s"] > 0]


def enumeration(st):
    """List of (k, mu) for the kept harmonics in the fixed order."""
    out = []
    for dd in kept_degrees(st):
        for mu in harmonics.index_set(st["d"], dd["k"]):
            out.append((dd["k"], mu))
    return out


def factor(st):
    """U (N x r) exactly as Algorithm 1 assembles it, and D (r,).

    U[:, (k,h,l)] = Y_k^h(x_i) * Xbar_k[i, l], Y = S / rho^k (taken as 0 where
    rho = 0 and k > 0, where Xbar_k vanishes).
    """
    geo = st["geo"]
    xt = geo["xt"]
    rho = np.sqrt(geo["rho2"])
    kd = kept_degrees(st)
    if not kd:
        return np.zeros((st["N"], 0)), np.zeros(0)
    Sh = harmonics.solid_harmonics(xt, st["K"], degrees=[dd["k"] for dd in kd])
    cols, dv = [], []
    for dd in kd:
        k = dd["k"]
        with np.errstate(divide="ignore", invalid="ignore"):
            Yk = Sh[k] / (rho ** k)[:, None]
        Yk[~np.isfinite(Yk)] = 0.0
        for h in range(Yk.shape[1]):
            for l in range(dd["s"]):
                cols.append(Yk[:, h] * dd["Xbar"][:, l])
                dv.append(dd["lam"][l])
    return np.stack(cols, axis=1), np.array(dv)


def phi_psi(st, X):
    """Khatri-Rao parts at arbitrary points X (frozen structure).

    Returns (Sh, q): Sh[k] = solid harmonics S_k^h((x - c)/R) (N x |H_k|) and
    q[k] = radial functions sum_a E_k[a, l] phi_a(rho^2) (N x s_k), so that
    U[:, (k,h,l)] = Sh[k][:, h] * q[k][:, l].  X may be complex.
    """
    X = np.asarray(X)
    xt = (X - st["c"][None, :]) / st["Reff"]
    rho2 = np.zeros(X.shape[0], dtype=xt.dtype)
    for j in range(X.shape[1]):
        rho2 = rho2 + xt[:, j] * xt[:, j]
    t = cheb_arg(rho2, st["u0"], st["u1"])
    kd = kept_degrees(st)
    Sh = harmonics.solid_harmonics(xt, st["K"], degrees=[dd["k"] for dd in kd])
    q = {}
    for dd in kd:
        q[dd["k"]] = cheb_basis(t, dd["L"]) @ dd["E"]
    return Sh, q


def features(st, X):
    """U(X) (N x r) from the frozen structure, and D."""
    Sh, q = phi_psi(st, X)
    cols, dv = [], []
    for dd in kept_degrees(st):
        k = dd["k"]
        for h in range(Sh[k].shape[1]):
            for l in range(dd["s"]):
                cols.append(Sh[k][:, h] * q[k][:, l])
                dv.append(dd["lam"][l])
    if not cols:
        return np.zeros((X.shape[0], 0)), np.zeros(0)
    return np.stack(cols, axis=1), np.array(dv)


def matvec(st, V, U=None, Dv=None):
    """K V ~ U (D (U^T V)) (Sec. 3.6); V is (N,) or (N, m)."""
    if U is None:
        U, Dv = factor(st)
    V = np.asarray(V, dtype=np.float64)
    V2 = V.reshape(V.shape[0], -1)
    out = U @ (Dv[:, None] * (U.T @ V2))
    return out.reshape(V.shape)


def matvec_chunked(st, V, chunk=16384):
    """Matrix-free K V for large N: U never held whole (two passes over chunks)."""
    X = st.get("X")
    if X is None:
        raise ValueError("st['X'] needed")
    V = np.asarray(V, dtype=np.float64).reshape(X.shape[0], -1)
    W = None
    Dv = None
    for s in range(0, X.shape[0], chunk):
        U, Dv = features(st, X[s:s + chunk])
        part = U.T @ V[s:s + chunk]
        W = part if W is None else W + part
    W = Dv[:, None] * W
    out = np.empty_like(V)
    for s in range(0, X.shape[0], chunk):
        U, _ = features(st, X[s:s + chunk])
        out[s:s + chunk] = U @ W
    return out


# --------------------------------------------------------------------------
# Frozen-structure objective and its derivatives
# --------------------------------------------------------------------------

def core_blocks(st, a_coef):
    """C_k = E'_k^T M_k(a) E'_k for a coefficient vector a (linear in a)."""
    cores = expansion.radial_cores(a_coef, st["p"], st["d"], st["u0"], st["u1"])
    out = {}
    for dd in kept_degrees(st):
        M = np.array(cores[dd["k"]])
        out[dd["k"]] = dd["Ep"].T @ M @ dd["Ep"]
    return out


def _apply_core(st, C, G):
    """Multiply the (r x m) array G by the block-diagonal core C."""
    out = np.empty_like(G)
    o = 0
    for dd in kept_degrees(st):
        k, s = dd["k"], dd["s"]
        nh = harmonics.count(st["d"], k)
        blk = G[o:o + nh * s].reshape(nh, s, -1)
        out[o:o + nh * s] = np.einsum("ab,hbc->hac", C[k], blk).reshape(nh * s, -1)
        o += nh * s
    return out


def objective(st, X, Wm, Vm, C=None):
    """F = sum_c w_c^T U C U^T v_c (frozen structure)."""
    U, Dv = features(st, X)
    if C is None:
        C = {dd["k"]: np.diag(dd["lam"]) for dd in kept_degrees(st)}
    gw = U.T @ Wm
    gv = U.T @ Vm
    return np.sum(gw * _apply_core(st, C, gv))


def passes(st, M, chunk=16384):
    """U^T M over all points of st["X"], point chunk by point chunk."""
    X = st["X"]
    M = np.asarray(M, dtype=np.float64).reshape(X.shape[0], -1)
    out = None
    for s in range(0, X.shape[0], chunk):
        U, _ = features(st, X[s:s + chunk])
        part = U.T @ M[s:s + chunk]
        out = part if out is None else out + part
    return out


def grad_l_from_passes(st, gw, gv):
    """dF/dl = sum_c g_w^T (dC/dl) g_v from g_w = U^T W, g_v = U^T V, with
    dM/dl from the Chebyshev coefficients of dk/dl (structure frozen)."""
    da = chebyshev.cheb_coeffs_dl(st["kernel"], st["D"], st["l"])
    dC = core_blocks(st, da)
    return float(np.sum(gw * _apply_core(st, dC, gv)))


def grad_l(st, Wm, Vm):
    """dF/dl for F = sum_c w_c^T U C(l) U^T v_c (structure frozen)."""
    U, _ = features(st, st["X"])
    return grad_l_from_passes(st, U.T @ Wm, U.T @ Vm)


def grad_x(st, Wm, Vm, h=1e-30):
    """dF/dX (N x d): complex-step derivative of each feature row."""
    X = st["X"]
    U, Dv = features(st, X)
    C = {dd["k"]: np.diag(dd["lam"]) for dd in kept_degrees(st)}
    gw = U.T @ Wm
    gv = U.T @ Vm
    Cgv = _apply_core(st, C, gv)
    Cgw = _apply_core(st, C, gw)
    N, d = X.shape
    out = np.zeros((N, d))
    for j in range(d):
        Xc = X.astype(complex)
        Xc[:, j] += 1j * h
        Uc, _ = features(st, Xc)
        dU = Uc.imag / h
        out[:, j] = np.sum(Wm * (dU @ Cgv), axis=1) + np.sum(Vm * (dU @ Cgw), axis=1)
    return out
