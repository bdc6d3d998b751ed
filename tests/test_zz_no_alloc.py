"""hdf_matvec_noalloc (the product that allocates nothing) against hdf_matvec, through the C ABI.

Two calls in a row on one GPU, the second with a smaller input (fewer points
and fewer right-hand sides), each compared with hdf_matvec on the same factor:
binary64 within 1e-12 per column, binary32 within the factor's tolerance, and
identical results where both calls use the same point splits.  The scratch
array is shared by every call on the GPU and keeps the last call's contents,
so the second call also checks that nothing of the first one leaks into it.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_2202_03655_amd import workloads as wl
from tests.gpu_common import gpu_build, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_03655_amd import hdf
    hdf.lib()


def col_rel_max(got, ref):
    scale = np.maximum(np.max(np.abs(ref), axis=0), 1e-300)
    return float(np.max(np.max(np.abs(got - ref), axis=0) / scale))


def noalloc(f, V, out):
    from paper_2202_03655_amd import hdf
    st = hdf.lib().hdf_matvec_noalloc(f._h, V.data_ptr(), V.shape[1], V.stride(0), out.data_ptr(), out.stride(0),
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


CASES = [
    # (points, kernel, l, tol, m, mixed) of the first call, then of the second (smaller) call
    ((lambda: wl.max_norm_one(wl.gaussian_mixture(12_037, 5, 103)), "cauchy", 1.0, 1e-4, 16, True),
     (lambda: wl.max_norm_one(wl.gaussian_mixture(5_001, 5, 103)), "cauchy", 1.0, 1e-4, 3, True)),
    ((lambda: wl.uniform_cube(5_013, 4, 104), "gaussian", 0.7, 1e-5, 33, False),
     (lambda: wl.unit_ball(1_999, 3, 101), "gaussian", 1.0, 1e-6, 17, False)),
    ((lambda: wl.shell(3_001, 6, 105), "matern52", 8.0, 1e-7, 64, True),
     (lambda: wl.shell(1_003, 6, 105), "matern52", 8.0, 1e-7, 1, True)),
]


@pytest.mark.parametrize("case", CASES, ids=["mixed_gmm5", "fp64_cube4_ball3", "mixed_shell6_binary64_factor"])
def test_noalloc_matches_matvec_twice(case):
    from paper_2202_03655_amd import hdf
    for gen, kernel, l, tol, m, mixed in case:
        X = gen()
        if mixed:
            X = X.astype(np.float32)
        f, _ = gpu_build(X, kernel, l, tol, mixed=mixed)
        dt = torch.float32 if mixed else torch.float64
        V = to_dev(wl.rhs(len(X), m, 5 + m), dt)
        ref = f.matvec(V).double().cpu().numpy()
        out = torch.full((len(X), m), float("nan"), dtype=dt, device="cuda")
        assert noalloc(f, V, out) == 0, hdf.lib().hdf_last_error()
        got = out.double().cpu().numpy()
        e = col_rel_max(got, ref)
        bound = tol if (mixed and f.info()["factor_precision"] == hdf.HDF_MIXED) else 1e-12
        print(f"N={len(X)} m={m} mixed={mixed}: noalloc vs matvec per-column max rel {e:.2e} (bound {bound:g})")
        assert np.all(np.isfinite(got)) and e <= bound


def test_noalloc_rejects_what_it_cannot_serve():
    from paper_2202_03655_amd import hdf
    X = wl.unit_ball(500, 3, 101)
    f, _ = gpu_build(X, "gaussian", 1.0, 1e-6)
    V = to_dev(wl.rhs(500, 65, 1), torch.float64)
    out = torch.empty((500, 65), dtype=torch.float64, device="cuda")
    assert noalloc(f, V, out) == -1                      # m above 64
    fm = hdf.Factor(to_dev(X, torch.float64), "gaussian", 1.0, 1e-6, storage="none")
    V2 = to_dev(wl.rhs(500, 2, 1), torch.float64)
    out2 = torch.empty((500, 2), dtype=torch.float64, device="cuda")
    assert noalloc(fm, V2, out2) == -1                   # matrix-free factor
    assert noalloc(f, V2, out2) == 0
    np.testing.assert_allclose(out2.cpu().numpy(), f.matvec(V2).cpu().numpy(), rtol=0,
                               atol=1e-12 * float(out2.abs().max()))
