"""The oracle's full-size passes U^T M, split over host processes (test infrastructure).

U^T M is a sum over points, so disjoint point ranges can be contracted in
separate processes and their partial products added in range order; each
range runs the oracle's own `passes` unchanged.  Workers are spawned (not
forked: the parent holds a HIP context) and import numpy and the oracle only.
"""
import os
from concurrent.futures import ProcessPoolExecutor
import multiprocessing as mp

import numpy as np

from oracle import hdf as ohdf

# entries of the oracle's state that `features` reads (the per-point arrays of the
# build, such as Q W_s of every degree, stay in the parent)
_KEYS = ("d", "K", "c", "Reff", "u0", "u1", "p", "kernel", "l", "D")
_DEG_KEYS = ("k", "L", "s", "E", "Ep", "lam")


def slim_state(st):
    out = {k: st[k] for k in _KEYS}
    out["deg"] = [{k: dd[k] for k in _DEG_KEYS} for dd in st["deg"]]
    return out


def _range_pass(args):
    slim, X, M, chunk = args
    st = dict(slim)
    st["X"] = X
    return ohdf.passes(st, M, chunk=chunk)


def workers():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def passes(st, M, chunk=8192, nproc=None):
    """U^T M over all points of st["X"] (the oracle's `passes`, by point ranges)."""
    X = st["X"]
    M = np.asarray(M, dtype=np.float64).reshape(X.shape[0], -1)
    nproc = nproc or workers()
    n = X.shape[0]
    step = max(chunk, -(-n // nproc) // chunk * chunk) if n > chunk else n
    ranges = [(a, min(n, a + step)) for a in range(0, n, step)]
    slim = slim_state(st)
    jobs = [(slim, X[a:b], M[a:b], chunk) for a, b in ranges]
    if len(jobs) == 1:
        return _range_pass(jobs[0])
    with ProcessPoolExecutor(max_workers=len(jobs), mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(_range_pass, jobs))
    out = parts[0]
    for p in parts[1:]:
        out = out + p
    return out
