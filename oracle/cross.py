"""Algorithm 1, general case X != Y: K(X, Y) ~ U V^T (oracle, test infrastructure).

Steps, in the paper's order (Algorithm 1; Sec. 3.4):

1. One normalisation for both sets: centre and radius of X u Y (geometry.py
   on the stacked points), so the degree-k expansion (Eq. preharm) holds for
   every pair (x, y).  The radial basis interval covers rho^2 of both sets.
2. ||K(X, Y)||_F ~ nu sqrt(N_x N_y) with nu^2 the mean of k(||x_a - y_b||)^2
   over SplitMix64 pairs a < N_x, b < N_y (splitmix.py); the degree rule and
   the Frobenius budget of the symmetric case then hold with N replaced by
   sqrt(N_x N_y).
3. Per degree k: R^{(k)} = X^{(k)} (Y^{(k)})^T with both radial matrices in the
   Chebyshev radial basis, X^{(k)} = Y_x M_k and Y^{(k)} = Y_y (Eq. vandermonde,
   the core folded into the x side); QR of Y_x and Y_y, the SVD of
   R_x M_k R_y^T (Eq. svd), and the singular values above tau kept
   (Eq. rapprox): Xbar = Q_x U_s sqrt(S_s), Ybar = Q_y V_s sqrt(S_s).
4. Assembly: column (k, h, l) of U is S_k^h(x_t) * Xbar[:, l], of V is
   S_k^h(y_t) * Ybar[:, l]; K(X, Y) ~ U V^T, and K(X, Y) W ~ U (V^T W).

Conventions (readings; the paper does not fix them): singular values in
descending order, ties to the lower index; each kept pair (u, v) is signed so
that the largest-magnitude coefficient of the x-side radial function in the
phi basis (lowest index on ties) is positive.
"""
import numpy as np

from . import chebyshev, expansion, geometry, harmonics, splitmix
from .hdf import Infeasible, cheb_arg, cheb_basis, tau_threshold


def build_cross(X, Y, kernel, l, tol, p=None, tau=None):
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    Nx, d = X.shape
    Ny, dy = Y.shape
    if d != dy:
        raise ValueError("X and Y must have the same dimension")
    if d < 3:
        raise ValueError("d >= 3 required")
    geo = geometry.geometry(np.vstack([X, Y]))
    nu = splitmix.norm_scale_cross(X, Y, kernel, l)
    a = chebyshev.cheb_coeffs(kernel, geo["D"], l)
    tail_at_p = None
    if p is None:
        p, tail_at_p, _ = chebyshev.choose_degree(a, tol, nu)
        if p is None:
            raise Infeasible("Chebyshev degree above the maximum")
    K = p // 2
    u0, u1 = geo["u0"], geo["u1"]
    cores = [np.array(M) for M in expansion.radial_cores(a, p, d, u0, u1)]
    if tau is None:
        tau = tau_threshold(tol, nu, np.sqrt(float(Nx) * float(Ny)), d, p)
    rho2x, rho2y = geo["rho2"][:Nx], geo["rho2"][Nx:]
    rhox, rhoy = np.sqrt(rho2x), np.sqrt(rho2y)
    tx, ty = cheb_arg(rho2x, u0, u1), cheb_arg(rho2y, u0, u1)
    deg = []
    for k in range(K + 1):
        L = K - k + 1
        Yx = (rhox ** k)[:, None] * cheb_basis(tx, L)
        Yy = (rhoy ** k)[:, None] * cheb_basis(ty, L)
        Qx, Rx = np.linalg.qr(Yx)
        Qy, Ry = np.linalg.qr(Yy)
        Us, sig, Vt = np.linalg.svd(Rx @ cores[k] @ Ry.T)
        keep = sig > tau
        s = int(keep.sum())
        Us, Vs, sg = Us[:, :s], Vt[:s, :].T, sig[:s]
        Ex = np.linalg.pinv(Rx, rcond=1e-15) @ Us * np.sqrt(sg)
        Ey = np.linalg.pinv(Ry, rcond=1e-15) @ Vs * np.sqrt(sg)
        for c in range(s):
            j = int(np.argmax(np.abs(Ex[:, c])))
            if Ex[j, c] < 0:
                Ex[:, c] *= -1.0
                Ey[:, c] *= -1.0
                Us[:, c] *= -1.0
                Vs[:, c] *= -1.0
        deg.append(dict(k=k, L=L, s=s, sig_all=sig, sig=sg, Ex=Ex, Ey=Ey,
                        Xbar=Qx @ Us * np.sqrt(sg), Ybar=Qy @ Vs * np.sqrt(sg)))
    st = dict(X=X, Y=Y, Nx=Nx, Ny=Ny, d=d, kernel=kernel, l=l, tol=tol, nu=nu, a=a, p=p, K=K,
              tail_at_p=tail_at_p, tau=tau, geo=geo, c=geo["c"], R=geo["R"], Reff=geo["Reff"],
              D=geo["D"], u0=u0, u1=u1, cores=cores, deg=deg)
    st["r"] = sum(harmonics.count(d, dd["k"]) * dd["s"] for dd in deg)
    return st


def features_cross(st, Z, side):
    """U(Z) (side "x", coefficients Ex) or V(Z) (side "y", coefficients Ey)."""
    Z = np.asarray(Z)
    zt = (Z - st["c"][None, :]) / st["Reff"]
    rho2 = np.zeros(Z.shape[0], dtype=zt.dtype)
    for j in range(Z.shape[1]):
        rho2 = rho2 + zt[:, j] * zt[:, j]
    t = cheb_arg(rho2, st["u0"], st["u1"])
    kd = [dd for dd in st["deg"] if dd["s"] > 0]
    if not kd:
        return np.zeros((Z.shape[0], 0))
    Sh = harmonics.solid_harmonics(zt, st["K"], degrees=[dd["k"] for dd in kd])
    cols = []
    for dd in kd:
        q = cheb_basis(t, dd["L"]) @ (dd["Ex"] if side == "x" else dd["Ey"])
        for h in range(Sh[dd["k"]].shape[1]):
            for c in range(dd["s"]):
                cols.append(Sh[dd["k"]][:, h] * q[:, c])
    return np.stack(cols, axis=1)


def factor_cross(st):
    """(U, V) with K(X, Y) ~ U V^T (Algorithm 1 assembly)."""
    return features_cross(st, st["X"], "x"), features_cross(st, st["Y"], "y")


def matvec_cross(st, W, U=None, V=None):
    """K(X, Y) W ~ U (V^T W) (Sec. 3.6); W is (N_y,) or (N_y, m)."""
    if U is None:
        U, V = factor_cross(st)
    W = np.asarray(W, dtype=np.float64)
    W2 = W.reshape(W.shape[0], -1)
    out = U @ (V.T @ W2)
    return out.reshape((U.shape[0],) + W.shape[1:])
