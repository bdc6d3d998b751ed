"""Adjoint of F = sum_c w_c^T K~ v_c through the C ABI (hdf_backward).

Compared with the oracle's frozen-structure derivatives (dF/dl from the
Chebyshev coefficients of dk/dl, dF/dX by complex step; both pinned by
central differences in test_oracle_pins.py), with the dense closed-form
gradient, and through torch.autograd.
"""
import numpy as np
import pytest
import torch

from oracle import dense, hdf as ohdf
from paper_2202_03655_amd import workloads as wl
from tests.gpu_common import gpu_build, oracle_for, rel_fro, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CASES = [
    ("cube4_gauss", lambda: wl.uniform_cube(1_501, 4, 104), "gaussian", 0.7, 1e-5, 1),
    ("ball3_gauss", lambda: wl.unit_ball(1_000, 3, 101), "gaussian", 1.0, 1e-6, 2),
    ("gmm5_cauchy", lambda: wl.max_norm_one(wl.gaussian_mixture(2_003, 5, 103)), "cauchy", 1.0, 1e-4, 5),
    ("shell6_matern52", lambda: wl.shell(801, 6, 105), "matern52", 8.0, 1e-7, 1),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_adjoint_fp64_matches_oracle(case):
    name, gen, kernel, l, tol, m = case
    X = gen()
    st, _ = oracle_for(X, kernel, l, tol)
    f, Xd = gpu_build(X, kernel, l, tol)
    assert f.info()["rank"] == st["r"]
    W = wl.rhs(len(X), m, 21)
    V = wl.rhs(len(X), m, 22)
    dl, dX = f.backward(to_dev(W, torch.float64), to_dev(V, torch.float64))
    gl_o = ohdf.grad_l(st, W, V)
    gx_o = ohdf.grad_x(st, W, V)
    print(f"{name}: dl {dl:.6e} vs oracle {gl_o:.6e}")
    assert abs(dl - gl_o) <= 1e-10 * max(abs(gl_o), 1e-300)
    assert rel_fro(dX.cpu().numpy(), gx_o) <= 1e-10


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_adjoint_mixed_within_tol_of_oracle(case):
    """HDF_MIXED: binary32 points, W, V and dX; the factor is binary32 above
    tol 1e-6 and binary64 at or below it.  dF/dl and dF/dX against the oracle
    on the same binary32 values, within tol (relative; Frobenius for dF/dX)."""
    name, gen, kernel, l, tol, m = case
    X = gen().astype(np.float32)
    st, _ = oracle_for(X, kernel, l, tol, mixed=True)
    f, _ = gpu_build(X, kernel, l, tol, mixed=True)
    assert f.info()["rank"] == st["r"]
    W = wl.rhs(len(X), m, 21).astype(np.float32)
    V = wl.rhs(len(X), m, 22).astype(np.float32)
    dl, dX = f.backward(to_dev(W, torch.float32), to_dev(V, torch.float32))
    W64, V64 = W.astype(np.float64), V.astype(np.float64)
    gl_o = ohdf.grad_l(st, W64, V64)
    gx_o = ohdf.grad_x(st, W64, V64)
    e_l = abs(dl - gl_o) / abs(gl_o)
    e_x = rel_fro(dX.double().cpu().numpy(), gx_o)
    print(f"{name}: mixed (factor {'binary32' if tol > 1e-6 else 'binary64'}) dl rel {e_l:.2e}, "
          f"dX rel {e_x:.2e} (tol {tol:g})")
    assert e_l <= tol and e_x <= tol


def test_adjoint_vs_dense_gradient():
    X = wl.uniform_cube(2000, 4, 104)
    f, _ = gpu_build(X, "gaussian", 0.7, 1e-7)
    w = wl.rhs(2000, 1, 31)[:, 0]
    v = wl.rhs(2000, 1, 32)[:, 0]
    dl, dX = f.backward(to_dev(w[:, None], torch.float64), to_dev(v[:, None], torch.float64))
    gl = dense.dense_grad_l(X, "gaussian", 0.7, w, v)
    gx = dense.dense_grad_x(X, "gaussian", 0.7, w, v)
    print(f"dense: dl rel {abs(dl - gl) / abs(gl):.2e}, dX rel {rel_fro(dX.cpu().numpy(), gx):.2e}")
    assert abs(dl - gl) <= 1e-4 * abs(gl)
    assert rel_fro(dX.cpu().numpy(), gx) <= 1e-3


def test_adjoint_mixed_close_to_fp64():
    X = wl.uniform_cube(20_000, 4, 104)
    f32, _ = gpu_build(X.astype(np.float32), "gaussian", 0.7, 1e-5, mixed=True)
    f64, _ = gpu_build(X.astype(np.float32).astype(np.float64), "gaussian", 0.7, 1e-5)
    W = wl.rhs(20_000, 1, 41)
    V = wl.rhs(20_000, 1, 42)
    dl32, dX32 = f32.backward(to_dev(W, torch.float32), to_dev(V, torch.float32))
    dl64, dX64 = f64.backward(to_dev(W, torch.float64), to_dev(V, torch.float64))
    e_l = abs(dl32 - dl64) / abs(dl64)
    e_x = rel_fro(dX32.double().cpu().numpy(), dX64.cpu().numpy())
    print(f"mixed vs fp64 adjoint: dl {e_l:.2e}, dX {e_x:.2e}")
    assert e_l <= 1e-5 and e_x <= 1e-4


def test_autograd_function():
    from paper_2202_03655_amd import hdf
    X = wl.unit_ball(700, 3, 5)
    Xd = to_dev(X, torch.float64).requires_grad_(True)
    l = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    V = to_dev(wl.rhs(700, 2, 6), torch.float64).requires_grad_(True)
    G = to_dev(wl.rhs(700, 2, 7), torch.float64)
    f = hdf.Factor(Xd.detach(), "gaussian", 1.0, 1e-6, precision=hdf.HDF_FP64)
    Y = hdf.HDFMatvec.apply(Xd, l, V, f)
    (Y * G).sum().backward()
    dl, dX = f.backward(G, V.detach())
    np.testing.assert_allclose(Xd.grad.cpu().numpy(), dX.cpu().numpy(), rtol=1e-12, atol=1e-14)
    assert abs(l.grad.item() - dl) <= 1e-12 * abs(dl)
    np.testing.assert_allclose(V.grad.cpu().numpy(), f.matvec(G).cpu().numpy(), rtol=1e-12, atol=1e-12)
