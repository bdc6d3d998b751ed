"""Host-side checks of the C ABI library (no GPU needed).

* the library loads and exports every function declared in include/hdf.h;
* the host planner (extended-precision Rodrigues route) agrees with the
  oracle's exact-rational expansion of App. A, its Chebyshev transform and
  degree rule, and its index-set enumeration (bit-exact);
* argument errors of the host entry points.
"""
import os
import re

import numpy as np
import pytest

from oracle import chebyshev, expansion, harmonics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2202_03655_amd import hdf
    return hdf


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hdf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hdf_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    hdf = _lib()
    L = hdf.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert sorted(hdf.EXPORTS) == names


def test_status_strings():
    L = _lib().lib()
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert len(L.hdf_status_string(s)) > 0


@pytest.mark.parametrize("name,D,l", [("gaussian", 2.0, 1.0), ("cauchy", 1.9, 1.0),
                                      ("matern32", 2.0, 2.0), ("matern52", 2.2, 0.9)])
def test_planner_chebyshev_and_degree(name, D, l):
    hdf = _lib()
    a_o = chebyshev.cheb_coeffs(name, D, l)
    a_p = hdf.plan_chebyshev(name, D, l)
    np.testing.assert_allclose(a_p, a_o, atol=2e-15)
    assert np.all(a_p[1::2] == 0.0)
    for eps in (1e-3, 1e-5, 1e-7):
        p_o, tail_o, thr = chebyshev.choose_degree(a_o, eps, 0.4)
        if p_o is None or p_o > 60:
            with pytest.raises(hdf.HDFError):
                hdf.plan_degree(a_p, eps, 0.4)
            continue
        p_p, tail_p = hdf.plan_degree(a_p, eps, 0.4)
        ambiguous = abs(tail_o - thr) <= 1e-9 * thr
        assert p_p == p_o or ambiguous
        # each of the N_F coefficients carries ~1e-16 absolute rounding noise
        assert abs(tail_p - tail_o) <= 1e-12 * tail_o + 1e-13


@pytest.mark.parametrize("d", [3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("p", [0, 2, 10, 20, 30])
def test_planner_cores_match_exact_expansion(d, p):
    hdf = _lib()
    a = chebyshev.cheb_coeffs("cauchy", 1.9, 1.0)
    u0, u1 = 0.013, 0.997
    c_o = expansion.radial_cores(a, p, d, u0, u1)
    c_p = hdf.plan_cores(a, p, d, u0, u1)
    for k, (Mo, Mp) in enumerate(zip(c_o, c_p)):
        Mo = np.array(Mo)
        assert Mp.shape == Mo.shape == (p // 2 - k + 1,) * 2
        np.testing.assert_allclose(Mp, Mo, rtol=0, atol=1e-15 * np.max(np.abs(Mo)))


def test_planner_cores_other_kernels_and_intervals():
    hdf = _lib()
    for name, D, l, p, d, u0, u1 in [("gaussian", 4.0, 0.7, 28, 4, 0.0, 1.0),
                                      ("matern52", 2.2, 8.0, 14, 6, 0.67, 1.0),
                                      ("matern32", 10.0, 10.0, 36, 3, 1e-6, 0.9)]:
        a = chebyshev.cheb_coeffs(name, D, l)
        c_o = expansion.radial_cores(a, p, d, u0, u1)
        c_p = hdf.plan_cores(a, p, d, u0, u1)
        for Mo, Mp in zip(c_o, c_p):
            Mo = np.array(Mo)
            np.testing.assert_allclose(Mp, Mo, rtol=0, atol=2e-15 * np.max(np.abs(Mo)))


@pytest.mark.parametrize("d", [3, 4, 5, 6, 7, 8])
def test_planner_index_sets_bit_exact(d):
    hdf = _lib()
    for k in range(0, 9):
        t = hdf.plan_index_set(d, k)
        assert [tuple(int(v) for v in r) for r in t] == harmonics.index_set(d, k)
        assert len(t) == harmonics.count(d, k)


def test_host_entry_point_errors():
    hdf = _lib()
    with pytest.raises(hdf.HDFError) as e:
        hdf.plan_index_set(2, 3)
    assert e.value.status == -2
    with pytest.raises(hdf.HDFError) as e:
        hdf.plan_cores(np.zeros(20), 5, 3, 0.0, 1.0)       # odd p
    assert e.value.status == -1
    with pytest.raises(hdf.HDFError):
        hdf.plan_cores(np.zeros(20), 4, 3, 0.5, 0.5)       # empty interval
    with pytest.raises(hdf.HDFError):
        hdf.plan_chebyshev("gaussian", 1.0, -1.0)
    with pytest.raises(hdf.HDFError):
        hdf.plan_chebyshev("gaussian", 1.0, 1.0, n_nodes=1000)


def test_planner_cross_compression_matches_oracle():
    """Gram + SVD route of the library vs the oracle's QR + SVD (Algorithm 1,
    general case) on well-conditioned degrees: singular values and radial
    functions Y_x E_x, Y_y E_y agree."""
    import numpy as np
    from oracle import cross, hdf as ohdf
    hdf = _lib()
    rng = np.random.default_rng(12)
    X = rng.uniform(-1, 1, size=(600, 4))
    Y = rng.normal(size=(500, 4)) * 0.5
    sc = cross.build_cross(X, Y, "cauchy", 1.0, 1e-5)
    rx2, ry2 = sc["geo"]["rho2"][:600], sc["geo"]["rho2"][600:]
    for dd in sc["deg"]:
        k, L = dd["k"], dd["L"]
        if L > 6 or dd["s"] == 0:
            continue
        Yx = (np.sqrt(rx2) ** k)[:, None] * ohdf.cheb_basis(ohdf.cheb_arg(rx2, sc["u0"], sc["u1"]), L)
        Yy = (np.sqrt(ry2) ** k)[:, None] * ohdf.cheb_basis(ohdf.cheb_arg(ry2, sc["u0"], sc["u1"]), L)
        cond = max(np.linalg.cond(Yx.T @ Yx), np.linalg.cond(Yy.T @ Yy))
        sig, Ex, Ey = hdf.plan_compress_cross(Yx.T @ Yx, Yy.T @ Yy, np.array(sc["cores"][k]), sc["tau"])
        assert len(sig) == dd["s"]
        np.testing.assert_allclose(sig, dd["sig"], rtol=0, atol=1e-13 * cond * dd["sig_all"][0])
        gaps = np.abs(np.diff(dd["sig_all"]))
        for c in range(dd["s"]):
            gap = min(gaps[c - 1] if c > 0 else np.inf, gaps[c] if c < len(gaps) else np.inf)
            bound = 1e-13 * cond * (1 + dd["sig_all"][0] / gap)
            if bound < 1e-6:
                qx, qxo = Yx @ Ex[:, c], Yx @ dd["Ex"][:, c]
                qy, qyo = Yy @ Ey[:, c], Yy @ dd["Ey"][:, c]
                assert np.linalg.norm(qx - qxo) <= bound * np.linalg.norm(qxo), (k, c)
                assert np.linalg.norm(qy - qyo) <= bound * np.linalg.norm(qyo), (k, c)
