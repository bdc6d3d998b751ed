"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

FP64 path: degree, ranks and the harmonic enumeration bit-exact (apart from
knife-edge decisions), geometry exact, factor values and K~V within 1e-12
relative.  Mixed path: K~V within the requested tolerance of the FP64 result
and of the dense kernel.
"""
import numpy as np
import pytest
import torch

from oracle import dense, hdf as ohdf
from paper_2202_03655_amd import workloads as wl
from tests.gpu_common import ambiguous_ranks, gpu_build, oracle_for, oracle_phi, rel_fro, to_dev, torch_contraction

pytestmark = pytest.mark.gpu

CASES = [
    # name, points, kernel, l, tol, m
    ("ball3_gauss_2000", lambda: wl.unit_ball(2000, 3, 101), "gaussian", 1.0, 1e-6, 1),
    ("gmm5_cauchy_ragged", lambda: wl.max_norm_one(wl.gaussian_mixture(12_037, 5, 103)), "cauchy", 1.0, 1e-4, 16),
    ("cube4_gauss_ragged", lambda: wl.uniform_cube(5_013, 4, 104), "gaussian", 0.7, 1e-5, 3),
    ("shell6_matern52_l8", lambda: wl.shell(3_001, 6, 105), "matern52", 8.0, 1e-7, 17),
    ("normal3_matern32_l10", lambda: wl.normal_cloud(4_099, 3, 102), "matern32", 10.0, 1e-4, 33),
    ("ball7_gauss", lambda: wl.unit_ball(1_500, 7, 7), "gaussian", 2.0, 1e-4, 5),
    ("ball8_cauchy", lambda: wl.unit_ball(1_200, 8, 8), "cauchy", 3.0, 1e-3, 2),
]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_03655_amd import hdf
    hdf.lib()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fp64_parity(case):
    name, gen, kernel, l, tol, m = case
    X = gen()
    st, Xo = oracle_for(X, kernel, l, tol)
    f, Xd = gpu_build(X, kernel, l, tol)
    inf = f.info()
    plan = f.plan()
    print(f"{name}: p={inf['degree_p']} rank={inf['rank']} refined degrees={inf['n_refined']}")
    # geometry: exact (same IEEE operations in the same order)
    assert inf["center_radius"] == st["R"]
    assert inf["rho2_min"] == st["u0"] and inf["rho2_max"] == st["u1"]
    assert abs(inf["nu"] / st["nu"] - 1) < 1e-12
    amb = ambiguous_ranks(st)
    if not amb:
        assert inf["degree_p"] == st["p"]
        assert inf["s_k"] == [dd["s"] for dd in st["deg"]]
    if inf["degree_p"] != st["p"] or inf["s_k"] != [dd["s"] for dd in st["deg"]]:
        pytest.skip(f"{name}: knife-edge rank decision (reported, not compared)")
    assert abs(inf["tau"] / st["tau"] - 1) < 1e-12
    assert inf["rank"] == st["r"] and inf["n_harmonics"] == st["H"]
    # enumeration: bit-exact
    enum = ohdf.enumeration(st)
    tab = plan["index_table"]
    assert [(int(r[0]),) + tuple(int(v) for v in r[1:]) for r in tab] == [(k,) + mu for k, mu in enum]
    # eigenvalues
    lam_o = np.concatenate([dd["lam"] for dd in st["deg"]])
    np.testing.assert_allclose(plan["lam"], lam_o, rtol=0, atol=1e-12 * np.max(np.abs(lam_o)))
    # factor values
    phi, q = f.factor_parts()
    kept = [dd["k"] for dd in st["deg"] if dd["s"] > 0]
    phi_o = oracle_phi(st, kept)
    phi_g = phi.cpu().numpy()
    assert np.max(np.abs(phi_g - phi_o)) <= 1e-12 * np.max(np.abs(phi_o))
    # radial functions, column by column: the two compression routes (QR here,
    # Gram + eig on the device) agree to ~eps * (cond(G_k) + |lam|_max / gap)
    t = ohdf.cheb_arg(st["geo"]["rho2"], st["u0"], st["u1"])
    rho = np.sqrt(st["geo"]["rho2"])
    q_g = q.cpu().numpy()
    row = 0
    for dd in st["deg"]:
        if dd["s"] == 0:
            continue
        Y = (rho ** dd["k"])[:, None] * ohdf.cheb_basis(t, dd["L"])
        condG = np.linalg.cond(Y.T @ Y)
        qo = ohdf.cheb_basis(t, dd["L"]) @ dd["E"]
        lam = dd["lam_all"]
        for l in range(dd["s"]):
            others = np.delete(lam, l)
            gap = np.min(np.abs(others - lam[l])) if len(others) else np.inf
            bound = 1e-11 * (condG + np.max(np.abs(lam)) / gap)
            err = rel_fro(q_g[row], qo[:, l])
            if bound < 1e-6:           # compare only well-determined functions
                assert err <= bound, (dd["k"], l, err, bound)
            row += 1
    # K~V
    V = wl.rhs(len(X), m, 7)
    KV_o = ohdf.matvec(st, V)
    KV_g = f.matvec(to_dev(V, torch.float64)).cpu().numpy()
    assert rel_fro(KV_g, KV_o) <= 1e-12, rel_fro(KV_g, KV_o)


def test_fp64_guarantee_against_dense():
    X = wl.unit_ball(2000, 3, 101)
    f, _ = gpu_build(X, "gaussian", 1.0, 1e-6)
    K = dense.dense_K(X, "gaussian", 1.0)
    Kt = f.matvec(torch.eye(2000, dtype=torch.float64, device="cuda")[:, :256]).cpu().numpy()
    err = np.linalg.norm(K[:, :256] - Kt) / np.linalg.norm(K[:, :256])
    assert err <= 1e-6
    # symmetry of the applied operator: u^T (K~ v) = v^T (K~ u)
    u = torch.randn(2000, dtype=torch.float64, device="cuda")
    v = torch.randn(2000, dtype=torch.float64, device="cuda")
    a = torch.dot(u, f.matvec(v)).item()
    b = torch.dot(v, f.matvec(u)).item()
    assert abs(a - b) <= 1e-12 * abs(a)


@pytest.mark.parametrize("case", [
    ("ball3_gauss_hilo", lambda: wl.unit_ball(2000, 3, 101), "gaussian", 1.0, 1e-6, 4),
    ("gmm5_cauchy_1e-3", lambda: wl.max_norm_one(wl.gaussian_mixture(30_011, 5, 103)), "cauchy", 1.0, 1e-3, 16),
    ("gmm5_cauchy_1e-4", lambda: wl.max_norm_one(wl.gaussian_mixture(30_011, 5, 103)), "cauchy", 1.0, 1e-4, 16),
    ("cube4_gauss_1e-5", lambda: wl.uniform_cube(20_000, 4, 104), "gaussian", 0.7, 1e-5, 2),
], ids=lambda c: c[0])
def test_mixed_within_tol(case):
    name, gen, kernel, l, tol, m = case
    X = gen().astype(np.float32)
    f32, _ = gpu_build(X, kernel, l, tol, mixed=True)
    f64, _ = gpu_build(X.astype(np.float64), kernel, l, tol)
    V = wl.rhs(len(X), m, 11)
    KV32 = f32.matvec(to_dev(V, torch.float32)).double().cpu().numpy()
    KV64 = f64.matvec(to_dev(V, torch.float64)).cpu().numpy()
    err = rel_fro(KV32, KV64)
    print(f"{name}: mixed vs fp64 {err:.2e} (tol {tol:g}); ranks {f32.info()['rank']} / {f64.info()['rank']}")
    assert err <= tol


@pytest.mark.parametrize("m", [1, 16, 17, 64])
def test_mixed_product_against_contraction(m):
    """The binary32 passes against an independent binary64 torch contraction of the same factor, on a ragged
    size (several pass-1 splits and a partial last chunk): m = 16 takes the pass-1 form with V in registers,
    the others the form that reads V from LDS."""
    X = wl.max_norm_one(wl.gaussian_mixture(12_037, 5, 103)).astype(np.float32)
    f, _ = gpu_build(X, "cauchy", 1.0, 1e-4, mixed=True)
    V = to_dev(wl.rhs(len(X), m, 21 + m).astype(np.float32), torch.float32)
    e = rel_fro(f.matvec(V).double().cpu().numpy(), torch_contraction(f, V).cpu().numpy())
    print(f"m={m}: binary32 K~V vs binary64 contraction of the same factor {e:.2e}")
    # same stored factor on both sides: only binary32 products and partial sums differ (6e-7 to 8e-7 measured)
    assert e <= 4e-6, e


def test_edge_cases_small_and_degenerate():
    from paper_2202_03655_amd import hdf
    # a single point and coincident points: rank-1 factor k(0) 1 1^T
    for n in (1, 2, 5):
        X = np.ones((n, 3)) * 0.25
        f, _ = gpu_build(X, "gaussian", 1.0, 1e-6)
        inf = f.info()
        assert inf["degree_p"] == 0 and inf["rank"] == 1
        V = wl.rhs(n, 2, 3)
        KV = f.matvec(to_dev(V, torch.float64)).cpu().numpy()
        np.testing.assert_allclose(KV, np.ones((n, n)) @ V, rtol=1e-13, atol=1e-13)
    # two distinct points
    X = np.array([[0.0, 0.0, 0.0], [0.3, -0.2, 0.1]])
    f, _ = gpu_build(X, "cauchy", 1.0, 1e-8)
    K = dense.dense_K(X, "cauchy", 1.0)
    KV = f.matvec(torch.eye(2, dtype=torch.float64, device="cuda")).cpu().numpy()
    assert np.linalg.norm(KV - K) <= 1e-8 * np.linalg.norm(K)
    # points on a sphere (zero-width radial interval)
    g = np.random.default_rng(5).normal(size=(500, 4))
    X = g / np.linalg.norm(g, axis=1)[:, None]
    st, _ = oracle_for(X, "gaussian", 1.0, 1e-5)
    f, _ = gpu_build(X, "gaussian", 1.0, 1e-5)
    V = wl.rhs(500, 3, 4)
    KV = f.matvec(to_dev(V, torch.float64)).cpu().numpy()
    assert rel_fro(KV, ohdf.matvec(st, V)) <= 1e-11
    K = dense.dense_K(X, "gaussian", 1.0)
    assert rel_fro(KV, K @ V) <= 1e-5


def test_error_paths():
    from paper_2202_03655_amd import hdf
    Xg = torch.zeros((10, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(hdf.HDFError) as e:
        hdf.Factor(Xg, "gaussian", 1.0, 1e-3)
    assert e.value.status == -2
    X = np.random.default_rng(0).normal(size=(100, 3))
    X[17, 1] = np.nan
    with pytest.raises(hdf.HDFError) as e:
        hdf.Factor(to_dev(X, torch.float64), "gaussian", 1.0, 1e-3)
    assert e.value.status == -3
    # dtype / precision mismatch, rejected by the C ABI itself
    import ctypes
    X32 = to_dev(np.ones((10, 3)), torch.float32)
    h = ctypes.c_void_p()
    st = hdf.lib().hdf_build(X32.data_ptr(), 0, 10, 3, 3, 0, 1.0, 1e-3, hdf.HDF_FP64, None, ctypes.byref(h))
    assert st == -1 and not h.value
    # diameter / lengthscale too large for the degree limit (normal cloud,
    # Matern-3/2, l = 0.5)
    X = wl.normal_cloud(20_000, 3, 102)
    with pytest.raises(hdf.HDFError) as e:
        hdf.Factor(to_dev(X, torch.float64), "matern32", 0.5, 1e-4)
    assert e.value.status == -4
    f = hdf.Factor(to_dev(np.random.default_rng(1).normal(size=(64, 3)), torch.float64), "gaussian", 1.0, 1e-3)
    with pytest.raises(ValueError):
        f.matvec(torch.zeros((63, 1), dtype=torch.float64, device="cuda"))
    with pytest.raises(hdf.HDFError):
        f.matvec(torch.zeros((64, 300), dtype=torch.float64, device="cuda"))
    # dF/dX of a matrix-free factor (it contracts the stored harmonics) is refused before any device work
    Z = torch.zeros((64, 1), dtype=torch.float64, device="cuda")
    fm = hdf.Factor(to_dev(np.random.default_rng(1).normal(size=(64, 3)), torch.float64), "gaussian", 1.0, 1e-3,
                    storage="none")
    with pytest.raises(hdf.HDFError) as e:
        fm.backward(Z, Z, need_l=False, need_x=True)
    assert e.value.status == -1
