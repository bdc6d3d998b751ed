"""Matrix-free factor (HDF_STORE_NONE) through the C ABI.

The factor is the same as the stored one (the build differs only in not
evaluating it), so K~V is checked against the oracle to the stored path's
tolerance and against the stored path on the same device: binary64 within
1e-12 of the oracle and 1e-13 of the stored product (the chunk-wise pass-1
partial sums are added in another order), binary32 within 1e-6 of the
stored product.  Chunkings: many small chunks, a ragged last chunk, one chunk
covering all points; m = 1, 17 and 70 (past the LDS-staged pass 1); dF/dl;
the sampled rank rule; N = 1; the headline workload at full size against
the stored factor.
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


@pytest.mark.parametrize("chunk", [64, 1000, 4096])
def test_fp64_against_oracle_and_stored(chunk):
    X = wl.unit_ball(2345, 3, 71)
    st = ohdf.build(X, "gaussian", 1.0, 1e-6)
    Xd = to_dev(X, torch.float64)
    fs = hdf().Factor(Xd, "gaussian", 1.0, 1e-6, precision=hdf().HDF_FP64)
    fm = hdf().Factor(Xd, "gaussian", 1.0, 1e-6, precision=hdf().HDF_FP64, storage="none", chunk=chunk)
    inf = fm.info()
    assert inf["storage"] == 1 and inf["chunk_points"] == min(chunk, 2345) and inf["rank"] == st["r"]
    assert inf["factor_bytes"] < fs.info()["factor_bytes"] or chunk >= 2345
    for m in (1, 17, 70):
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
    fm = h.Factor(Xd, "cauchy", 1.0, 1e-4, precision=h.HDF_MIXED, storage="none")
    V = to_dev(wl.rhs(len(X), 16, 7).astype(np.float32), torch.float32)
    a = fm.matvec(V).cpu().numpy().astype(np.float64)
    b = fs.matvec(V).cpu().numpy().astype(np.float64)
    e = rel_fro(a, b)
    ifm, ifs = fm.info(), fs.info()
    print(f"matrix-free vs stored: {e:.2e}; scratch {ifm['factor_bytes'] / 1e6:.0f} MB vs stored "
          f"{ifs['factor_bytes'] / 1e6:.0f} MB; pass 1 {ifm['t_mv_t_ms']:.3f} ms, pass 2 {ifm['t_mv_n_ms']:.3f} ms")
    assert ifm["rank"] == ifs["rank"]
    assert e <= 2e-6
