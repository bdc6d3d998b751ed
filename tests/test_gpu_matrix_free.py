"""Matrix-free factor (HDF_STORE_NONE) through the C ABI, both forms: the
fused kernels (16 points at a time evaluated and contracted in LDS) and the
chunk scratch.

The factor is the same as the stored one (the build differs only in not
evaluating it), so K~V is checked against the oracle to the stored path's
tolerance and against the stored path on the same device: binary64 within
1e-12 of the oracle and 1e-13 of the stored product (the partial sums are
added in another order), binary32 within 1e-6 of the stored product.
Chunkings: many small chunks, a ragged last chunk, one chunk covering all
points; m = 1, 17, 70 and 256 (16 column tiles); dF/dl; the sampled rank
rule; N = 1 and N below one 16-point chunk; a binary64 factor of binary32
points; a factor whose harmonics do not fit in LDS (chunk scratch chosen);
the headline workload at full size against the stored factor.
"""
import numpy as np
import pytest
import torch

from oracle import hdf as ohdf
from paper_2202_03655_amd import workloads as wl
from tests.gpu_common import rel_fro, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def hdf():
    from paper_2202_03655_amd import hdf as h
    return h


@pytest.mark.parametrize("chunk,fused", [(64, False), (1000, False), (4096, False), (0, True)])
def test_fp64_against_oracle_and_stored(chunk, fused):
    X = wl.unit_ball(2345, 3, 71)
    st = ohdf.build(X, "gaussian", 1.0, 1e-6)
    Xd = to_dev(X, torch.float64)
    fs = hdf().Factor(Xd, "gaussian", 1.0, 1e-6, precision=hdf().HDF_FP64)
    fm = hdf().Factor(Xd, "gaussian", 1.0, 1e-6, precision=hdf().HDF_FP64, storage="none", chunk=chunk, fused=fused)
    inf = fm.info()
    assert inf["storage"] == 1 and inf["rank"] == st["r"] and bool(inf["mf_fused"]) == fused
    if fused:
        assert inf["factor_bytes"] == 0
    else:
        assert inf["chunk_points"] == min(chunk, 2345)
        assert inf["factor_bytes"] < fs.info()["factor_bytes"] or chunk >= 2345
    for m in (1, 17, 70) + ((256,) if fused else ()):
        V = wl.rhs(2345, m, 72 + m)
        Vd = to_dev(V, torch.float64)
        km = fm.matvec(Vd).cpu().numpy()
        assert rel_fro(km, ohdf.matvec(st, V)) <= 1e-12
        assert rel_fro(km, fs.matvec(Vd).cpu().numpy()) <= 1e-13


def test_mixed_and_dl_and_sampled():
    h = hdf()
    Xf = wl.uniform_cube(5013, 4, 104).astype(np.float32)
    Xd = to_dev(Xf, torch.float32)
    fs = h.Factor(Xd, "gaussian", 0.7, 1e-5, precision=h.HDF_MIXED)
    fm = h.Factor(Xd, "gaussian", 0.7, 1e-5, precision=h.HDF_MIXED, storage="none", chunk=2048)
    V = to_dev(wl.rhs(5013, 16, 82).astype(np.float32), torch.float32)
    W = to_dev(wl.rhs(5013, 16, 83).astype(np.float32), torch.float32)
    assert rel_fro(fm.matvec(V).cpu().numpy(), fs.matvec(V).cpu().numpy()) <= 1e-6
    dlm, _ = fm.backward(W, V, need_x=False)
    dls, _ = fs.backward(W, V, need_x=False)
    assert abs(dlm - dls) <= 1e-6 * abs(dls)
    # the sampled rank rule with a matrix-free factor: same degree, ranks and product as stored
    ss = h.Factor(Xd, "gaussian", 0.7, 1e-5, precision=h.HDF_MIXED, rank_rule="sampled")
    sm = h.Factor(Xd, "gaussian", 0.7, 1e-5, precision=h.HDF_MIXED, rank_rule="sampled", storage="none", chunk=999)
    assert sm.info()["s_k"] == ss.info()["s_k"]
    assert rel_fro(sm.matvec(V).cpu().numpy(), ss.matvec(V).cpu().numpy()) <= 1e-6


@pytest.mark.parametrize("fused", [True, False])
def test_mixed_against_stored_and_dl(fused):
    h = hdf()
    Xf = wl.uniform_cube(5013, 4, 104).astype(np.float32)
    Xd = to_dev(Xf, torch.float32)
    fs = h.Factor(Xd, "gaussian", 0.7, 1e-5, precision=h.HDF_MIXED)
    fm = h.Factor(Xd, "gaussian", 0.7, 1e-5, precision=h.HDF_MIXED, storage="none", chunk=2048, fused=fused)
    assert bool(fm.info()["mf_fused"]) == fused
    for m in (3, 16, 40):
        V = to_dev(wl.rhs(5013, m, 90 + m).astype(np.float32), torch.float32)
        e = rel_fro(fm.matvec(V).cpu().numpy(), fs.matvec(V).cpu().numpy())
        print(f"fused={fused} m={m}: matrix-free vs stored {e:.2e}")
        assert e <= 1e-6
    W = to_dev(wl.rhs(5013, 4, 83).astype(np.float32), torch.float32)
    V = to_dev(wl.rhs(5013, 4, 84).astype(np.float32), torch.float32)
    dlm, _ = fm.backward(W, V, need_x=False)
    dls, _ = fs.backward(W, V, need_x=False)
    assert abs(dlm - dls) <= 1e-6 * abs(dls)


def test_fused_binary64_factor_of_binary32_points():
    """tol 1e-7 under HDF_MIXED: binary64 factor, binary32 data, fused kernels; against the oracle on
    the same binary32 values within tol, and the stored factor within 1e-12."""
    h = hdf()
    Xf = wl.unit_ball(3001, 3, 101).astype(np.float32)
    st = ohdf.build(Xf.astype(np.float64), "gaussian", 1.0, 1e-7)
    Xd = to_dev(Xf, torch.float32)
    fm = h.Factor(Xd, "gaussian", 1.0, 1e-7, precision=h.HDF_MIXED, storage="none")
    fs = h.Factor(Xd, "gaussian", 1.0, 1e-7, precision=h.HDF_MIXED)
    inf = fm.info()
    assert inf["mf_fused"] == 1 and inf["factor_precision"] == h.HDF_FP64 and inf["rank"] == st["r"]
    V = wl.rhs(3001, 5, 85).astype(np.float32)
    km = fm.matvec(to_dev(V, torch.float32)).cpu().numpy().astype(np.float64)
    e1 = rel_fro(km, ohdf.matvec(st, V.astype(np.float64)))
    e2 = rel_fro(km, fs.matvec(to_dev(V, torch.float32)).cpu().numpy().astype(np.float64))
    print(f"binary64 factor, fused: vs oracle {e1:.2e}, vs stored {e2:.2e}")
    assert e1 <= 1e-7 and e2 <= 1e-7


def test_fused_d5_and_too_large_for_lds():
    """d = 5 binary32 through the fused kernels against the oracle (within tol) and the stored product;
    d = 6 binary64 with 2,000+ harmonics, whose 16-point tile does not fit in LDS: the chunk scratch is
    chosen and still matches."""
    h = hdf()
    X5 = wl.max_norm_one(wl.gaussian_mixture(2003, 5, 103)).astype(np.float32)
    st5 = ohdf.build(X5.astype(np.float64), "cauchy", 1.0, 1e-4)
    X5d = to_dev(X5, torch.float32)
    f5 = h.Factor(X5d, "cauchy", 1.0, 1e-4, precision=h.HDF_MIXED, storage="none")
    s5 = h.Factor(X5d, "cauchy", 1.0, 1e-4, precision=h.HDF_MIXED)
    assert f5.info()["mf_fused"] >= 1
    V = wl.rhs(2003, 16, 86).astype(np.float32)
    km = f5.matvec(to_dev(V, torch.float32)).cpu().numpy().astype(np.float64)
    e1 = rel_fro(km, ohdf.matvec(st5, V.astype(np.float64)))
    e2 = rel_fro(km, s5.matvec(to_dev(V, torch.float32)).cpu().numpy().astype(np.float64))
    print(f"d=5 fused: vs oracle {e1:.2e}, vs stored {e2:.2e}")
    assert e1 <= 1e-4 and e2 <= 1e-6
    X6 = wl.shell(801, 6, 105)
    st6 = ohdf.build(X6, "matern52", 8.0, 1e-7)
    f6 = h.Factor(to_dev(X6, torch.float64), "matern52", 8.0, 1e-7, precision=h.HDF_FP64, storage="none")
    assert f6.info()["mf_fused"] == 0 and f6.info()["factor_bytes"] > 0
    V = wl.rhs(801, 2, 87)
    assert rel_fro(f6.matvec(to_dev(V, torch.float64)).cpu().numpy(), ohdf.matvec(st6, V)) <= 1e-12


@pytest.mark.parametrize("dd,n,l,tol", [(3, 2345, 1.0, 1e-5), (5, 1501, 3.0, 1e-4), (4, 5013, 0.7, 1e-5)])
def test_fused_double_buffered(dd, n, l, tol):
    """binary32 factors whose 16-point tiles fit twice in LDS: half of the wavefronts evaluate the
    next chunk while the others contract the current one (mf_fused == 2); against the oracle within
    tol and the stored product within 1e-6, m = 2, 17 and 64, and dF/dl."""
    h = hdf()
    X = wl.unit_ball(n, dd, 400 + dd).astype(np.float32)
    st = ohdf.build(X.astype(np.float64), "gaussian", l, tol)
    Xd = to_dev(X, torch.float32)
    fm = h.Factor(Xd, "gaussian", l, tol, precision=h.HDF_MIXED, storage="none")
    fs = h.Factor(Xd, "gaussian", l, tol, precision=h.HDF_MIXED)
    assert fm.info()["mf_fused"] == 2 and fm.info()["rank"] == st["r"]
    for m in (2, 17, 64):
        V = wl.rhs(n, m, 95 + dd + m).astype(np.float32)
        km = fm.matvec(to_dev(V, torch.float32)).cpu().numpy().astype(np.float64)
        e1 = rel_fro(km, ohdf.matvec(st, V.astype(np.float64)))
        e2 = rel_fro(km, fs.matvec(to_dev(V, torch.float32)).cpu().numpy().astype(np.float64))
        print(f"d={dd} m={m}: double-buffered vs oracle {e1:.2e} (tol {tol:g}), vs stored {e2:.2e}")
        assert e1 <= tol and e2 <= 1e-6
    W = to_dev(wl.rhs(n, 2, 97).astype(np.float32), torch.float32)
    V = to_dev(wl.rhs(n, 2, 98).astype(np.float32), torch.float32)
    dlm, _ = fm.backward(W, V, need_x=False)
    dls, _ = fs.backward(W, V, need_x=False)
    assert abs(dlm - dls) <= 1e-5 * abs(dls)


@pytest.mark.parametrize("n", [1, 7, 16, 17, 33])
def test_fused_tiny_point_counts(n):
    """Fewer points than one 16-point chunk, exactly one, and ragged tails of one point."""
    h = hdf()
    X = wl.unit_ball(n, 3, 200 + n)
    st = ohdf.build(X, "gaussian", 1.0, 1e-6)
    f = h.Factor(to_dev(X, torch.float64), "gaussian", 1.0, 1e-6, precision=h.HDF_FP64, storage="none")
    assert f.info()["mf_fused"] == int(st["r"] > 0)
    V = wl.rhs(n, 3, 300 + n)
    assert rel_fro(f.matvec(to_dev(V, torch.float64)).cpu().numpy(), ohdf.matvec(st, V)) <= 1e-12


def test_edges_and_errors():
    h = hdf()
    X = wl.unit_ball(1, 3, 3)
    st = ohdf.build(X, "gaussian", 1.0, 1e-6)
    f = h.Factor(to_dev(X, torch.float64), "gaussian", 1.0, 1e-6, precision=h.HDF_FP64, storage="none", chunk=64)
    V = wl.rhs(1, 2, 4)
    assert rel_fro(f.matvec(to_dev(V, torch.float64)).cpu().numpy(), ohdf.matvec(st, V)) <= 1e-12
    X = wl.unit_ball(300, 5, 5)
    f = h.Factor(to_dev(X, torch.float64), "cauchy", 1.0, 1e-5, precision=h.HDF_FP64, storage="none", chunk=128)
    with pytest.raises(h.HDFError):
        f.factor_parts()
    with pytest.raises(h.HDFError):
        h.Factor(to_dev(X, torch.float64), "cauchy", 1.0, 1e-5, precision=h.HDF_FP64, storage="none", chunk=10)


def test_full_size_headline_against_stored():
    h = hdf()
    X = wl.points("gmm5_cauchy_1e-4").astype(np.float32)
    Xd = to_dev(X, torch.float32)
    fs = h.Factor(Xd, "cauchy", 1.0, 1e-4, precision=h.HDF_MIXED)
    V = to_dev(wl.rhs(len(X), 16, 7).astype(np.float32), torch.float32)
    b = fs.matvec(V).cpu().numpy().astype(np.float64)
    ifs = fs.info()
    for fused in (True, False):
        fm = h.Factor(Xd, "cauchy", 1.0, 1e-4, precision=h.HDF_MIXED, storage="none", fused=fused)
        a = fm.matvec(V).cpu().numpy().astype(np.float64)
        e = rel_fro(a, b)
        ifm = fm.info()
        print(f"matrix-free ({'fused' if fused else 'chunked'}) vs stored: {e:.2e}; scratch "
              f"{ifm['factor_bytes'] / 1e6:.0f} MB vs stored {ifs['factor_bytes'] / 1e6:.0f} MB; pass 1 "
              f"{ifm['t_mv_t_ms']:.3f} ms, pass 2 {ifm['t_mv_n_ms']:.3f} ms", flush=True)
        assert ifm["rank"] == ifs["rank"] and ifm["mf_fused"] == (2 if fused else 0)
        assert e <= 2e-6
