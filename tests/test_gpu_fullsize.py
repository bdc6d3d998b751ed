"""Parity at the workloads' full sizes (N up to 1e6), through the C ABI.

The oracle builds its own factor on the full cloud (plan, geometry, ranks);
outputs it cannot afford as a whole are compared on sampled rows it computes
one by one (factor rows, rows of K~V, rows of dF/dX), and the rest is checked
through properties that hold at any size:
  - the device K~V equals an independent binary64 contraction (torch GEMMs)
    of the device factor, over all N rows;
  - the mixed-precision K~V stays within tol of the binary64 device K~V;
  - a sampled-pair estimate of ||K - K~||_F / ||K||_F stays below tol.
Launch configuration as the benchmark: one build, then hdf_matvec with the
workload's number of right-hand sides, then hdf_backward.
"""
import numpy as np
import pytest
import torch

from oracle import hdf as ohdf
from paper_2202_03655_amd import workloads as wl
from tests.gpu_common import (ambiguous_ranks, degree_blocks, gpu_build, oracle_for, rel_fro, to_dev,
                               torch_contraction)

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_03655_amd import hdf
    hdf.lib()


def sample_rows(n, count=62, seed=5):
    """First and last point (ragged tail) plus seeded interior rows."""
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([[0, n - 1], rng.choice(n, count, replace=False)]))


def sampled_guarantee(f, X, kernel, l, pairs=16384, seed=9):
    """Unbiased sampled estimate of ||K - K~||_F / ||K||_F from device factor rows."""
    rng = np.random.default_rng(seed)
    n = len(X)
    a = rng.integers(0, n, pairs)
    b = rng.integers(0, n, pairs)
    phi, q = f.factor_parts()
    lam = torch.tensor(f.plan()["lam"], dtype=torch.float64, device="cuda")
    ia = torch.tensor(a, device="cuda")
    ib = torch.tensor(b, device="cuda")
    kt = torch.zeros(pairs, dtype=torch.float64, device="cuda")
    for k, h0, nh, q0, s in degree_blocks(f):
        P = phi[h0:h0 + nh].double()
        hh = (P[:, ia] * P[:, ib]).sum(0)                  # sum_h Phi_h(a) Phi_h(b)
        rr = (q[q0:q0 + s][:, ia].double() * q[q0:q0 + s][:, ib].double() * lam[q0:q0 + s, None]).sum(0)
        kt += hh * rr
    r = np.linalg.norm(X[a] - X[b], axis=1)
    from oracle import kernels
    kv = kernels.kappa(kernel, r, l)
    err = kt.cpu().numpy() - kv
    return float(np.sqrt(np.sum(err ** 2) / np.sum(kv ** 2)))


FULL = [
    # name, workload, compare binary64 path too, right-hand sides
    ("gmm5_cauchy_1e-4", "gmm5_cauchy_1e-4", True),
    ("gmm5_cauchy_1e-3", "gmm5_cauchy_1e-3", False),
    ("normal3_matern32_l10", "normal3_matern32_l10", True),
    ("shell6_matern52_l8", "shell6_matern52_l8", True),
]

# The mixed path meets tol itself: above tol 1e-6 with a binary32 factor, at or
# below it with a binary64 factor of the binary32 points (the rounding of a
# binary32 factor alone exceeds such tolerances).


@pytest.mark.parametrize("case", FULL, ids=[c[0] for c in FULL])
def test_fullsize_plan_rows_and_matvec(case):
    name, wname, with_fp64 = case
    cfg = wl.CONFIGS[wname]
    X32 = wl.points(wname).astype(np.float32)
    n, m = len(X32), cfg["m"]
    kernel, l, tol = cfg["kernel"], cfg["l"], cfg["tol"]
    print(f"{name}: N={n} d={X32.shape[1]} m={m}", flush=True)
    st, Xo = oracle_for(X32, kernel, l, tol, mixed=True)
    f, Xd = gpu_build(X32, kernel, l, tol, mixed=True)
    inf = f.info()
    print(f"{name}: p={inf['degree_p']} r={inf['rank']} s_k={inf['s_k']} oracle s_k="
          f"{[dd['s'] for dd in st['deg']]} factor {'binary32' if inf['factor_precision'] == 1 else 'binary64'}",
          flush=True)
    assert inf["factor_precision"] == (1 if tol > 1e-6 else 0)
    # plan and geometry on the full cloud
    assert inf["center_radius"] == st["R"]
    assert inf["rho2_min"] == st["u0"] and inf["rho2_max"] == st["u1"]
    assert abs(inf["nu"] / st["nu"] - 1) < 1e-12
    assert inf["degree_p"] == st["p"]
    assert abs(inf["tau"] / st["tau"] - 1) < 1e-12
    # sampled factor rows against the oracle (binary32 storage)
    idx = sample_rows(n)
    Sh, qo = ohdf.phi_psi(st, Xo[idx])
    phi, q = f.factor_parts()
    same_ranks = inf["s_k"] == [dd["s"] for dd in st["deg"]]
    for k, h0, nh, q0, s in degree_blocks(f):
        ph = phi[h0:h0 + nh][:, torch.tensor(idx, device="cuda")].double().cpu().numpy().T
        assert np.max(np.abs(ph - Sh[k])) <= 2e-5 * max(1.0, np.max(np.abs(Sh[k]))), (name, k)
        if same_ranks:
            # radial functions: the two compression routes (QR in the oracle,
            # split-precision Gram + eig on the device) agree to about
            # eta (cond(G_k) + |lam|_max / gap), eta ~ 1e-9 for the split
            # Gram, plus binary32 rounding; compared where that is below tol
            qg = q[q0:q0 + s][:, torch.tensor(idx, device="cuda")].double().cpu().numpy().T
            dd = [e for e in st["deg"] if e["k"] == k][0]
            Y = (np.sqrt(st["geo"]["rho2"]) ** k)[:, None] * ohdf.cheb_basis(
                ohdf.cheb_arg(st["geo"]["rho2"], st["u0"], st["u1"]), dd["L"])
            condG = np.linalg.cond(Y.T @ Y)
            lam = dd["lam_all"]
            for j in range(s):
                others = np.delete(lam, j)
                gap = np.min(np.abs(others - lam[j])) if len(others) else np.inf
                bound = 1e-9 * (condG + np.max(np.abs(lam)) / gap) + 1e-5
                if bound < tol:
                    assert rel_fro(qg[:, j], qo[k][:, j]) <= bound, (name, k, j)
    del phi, q
    # K~V: device kernels vs an independent binary64 contraction, all rows
    V = wl.rhs(n, m, 7)
    V32 = to_dev(V.astype(np.float32), torch.float32)
    KV = f.matvec(V32)
    ref = torch_contraction(f, V32)
    e_c = rel_fro(KV.double().cpu().numpy(), ref.cpu().numpy())
    print(f"{name}: mixed K~V vs binary64 contraction of the same factor {e_c:.2e}", flush=True)
    assert e_c <= 2e-5
    # sampled guarantee against the kernel itself
    g = sampled_guarantee(f, Xo, kernel, l)
    print(f"{name}: sampled ||K - K~||_F/||K||_F = {g:.2e} (tol {tol:g})", flush=True)
    assert g <= tol
    if with_fp64:
        f64, _ = gpu_build(Xo, kernel, l, tol)
        inf64 = f64.info()
        if not ambiguous_ranks(st):
            assert inf64["s_k"] == [dd["s"] for dd in st["deg"]]
        KV64 = f64.matvec(to_dev(V, torch.float64))
        ref64 = torch_contraction(f64, to_dev(V, torch.float64))
        e64 = rel_fro(KV64.cpu().numpy(), ref64.cpu().numpy())
        e_mix = rel_fro(f.matvec(to_dev(V.astype(np.float32), torch.float32)).double().cpu().numpy(),
                        KV64.cpu().numpy())
        g64 = sampled_guarantee(f64, Xo, kernel, l)
        print(f"{name}: binary64 K~V vs contraction {e64:.2e}; mixed vs binary64 {e_mix:.2e}; "
              f"binary64 sampled error {g64:.2e}", flush=True)
        assert e64 <= 1e-12
        assert g64 <= tol
        assert e_mix <= tol
        # binary64 factor rows against the oracle
        phi64, q64 = f64.factor_parts()
        ti = torch.tensor(idx, device="cuda")
        for k, h0, nh, q0, s in degree_blocks(f64):
            ph = phi64[h0:h0 + nh][:, ti].cpu().numpy().T
            assert np.max(np.abs(ph - Sh[k])) <= 1e-12 * max(1.0, np.max(np.abs(Sh[k])))


def test_fullsize_backward_cube4():
    """N=2e5, d=4, Gaussian l=0.7, tol 1e-5: sampled rows of K~v and of
    dF/dX against the oracle, dF/dl against the oracle's frozen-structure
    derivative, and the mixed path against binary64."""
    cfg = wl.CONFIGS["cube4_gauss"]
    X = wl.points("cube4_gauss")
    n = len(X)
    kernel, l, tol = cfg["kernel"], cfg["l"], cfg["tol"]
    st, Xo = oracle_for(X, kernel, l, tol)
    f, Xd = gpu_build(Xo, kernel, l, tol)
    inf = f.info()
    print(f"cube4: N={n} p={inf['degree_p']} r={inf['rank']}", flush=True)
    if not ambiguous_ranks(st):
        assert inf["s_k"] == [dd["s"] for dd in st["deg"]]
    if inf["s_k"] != [dd["s"] for dd in st["deg"]]:
        pytest.skip("knife-edge rank decision (reported, not compared)")
    w = wl.rhs(n, 1, 21)
    v = wl.rhs(n, 1, 22)
    pv = ohdf.passes(st, v)                       # U^T v, U^T w (oracle, chunked)
    pw = ohdf.passes(st, w)
    Dv = ohdf.features(st, Xo[:1])[1]
    gv, gw = Dv[:, None] * pv, Dv[:, None] * pw
    idx = sample_rows(n, 30)
    # rows of K~v
    Ui, _ = ohdf.features(st, Xo[idx])
    kv_o = Ui @ gv
    kv_g = f.matvec(to_dev(v, torch.float64)).cpu().numpy()[idx]
    assert rel_fro(kv_g, kv_o) <= 1e-12
    # rows of dF/dX by complex step on the oracle's features
    dl, dX = f.backward(to_dev(w, torch.float64), to_dev(v, torch.float64))
    dXg = dX.cpu().numpy()[idx]
    h = 1e-30
    dXo = np.zeros((len(idx), X.shape[1]))
    for j in range(X.shape[1]):
        Xc = Xo[idx].astype(complex)
        Xc[:, j] += 1j * h
        Uc, _ = ohdf.features(st, Xc)
        dU = Uc.imag / h
        dXo[:, j] = w[idx, 0] * (dU @ gv)[:, 0] + v[idx, 0] * (dU @ gw)[:, 0]
    e_x = rel_fro(dXg, dXo)
    print(f"cube4: sampled dF/dX rows vs oracle {e_x:.2e}", flush=True)
    assert e_x <= 1e-10
    # dF/dl from the oracle's own passes U^T w, U^T v
    gl = ohdf.grad_l_from_passes(st, pw, pv)
    print(f"cube4: dl {dl:.9e} vs oracle {gl:.9e}", flush=True)
    assert abs(dl - gl) <= 1e-10 * abs(gl)
    # mixed vs binary64
    f32, _ = gpu_build(X.astype(np.float32), kernel, l, tol, mixed=True)
    dl32, dX32 = f32.backward(to_dev(w, torch.float32), to_dev(v, torch.float32))
    f64b, _ = gpu_build(X.astype(np.float32).astype(np.float64), kernel, l, tol)
    dl64, dX64 = f64b.backward(to_dev(w, torch.float64), to_dev(v, torch.float64))
    e_l = abs(dl32 - dl64) / abs(dl64)
    e_xm = rel_fro(dX32.double().cpu().numpy(), dX64.cpu().numpy())
    print(f"cube4: mixed vs binary64 dl {e_l:.2e} dX {e_xm:.2e}", flush=True)
    assert e_l <= 1e-4 and e_xm <= 1e-3


@pytest.mark.parametrize("wname", ["normal3_matern32", "gmm5_cauchy_zscore", "shell6_matern52"])
def test_fullsize_literal_configs_are_infeasible(wname):
    """The literal configurations need a Chebyshev degree far above the limit
    (the kernel is not low rank on those clouds): the build reports it."""
    from paper_2202_03655_amd import hdf
    cfg = wl.CONFIGS[wname]
    X = wl.points(wname).astype(np.float32)
    with pytest.raises(hdf.HDFError) as e:
        hdf.Factor(to_dev(X, torch.float32), cfg["kernel"], cfg["l"], cfg["tol"], precision=hdf.HDF_MIXED)
    assert e.value.status == -4                   # HDF_E_INFEASIBLE
    print(f"{wname}: {e.value}")
