"""Helpers shared by the GPU tests: run the HIP path and the oracle on the
same inputs and compare what is unique (knife-edge rank and degree decisions
are reported as ambiguous instead of compared)."""
import numpy as np
import torch

from oracle import harmonics, hdf as ohdf

AMBIG = 1e-9



def to_dev(X, dtype):
    return torch.tensor(np.ascontiguousarray(X), dtype=dtype, device="cuda")


def gpu_build(X, kernel, l, tol, mixed=False):
    from paper_2202_03655_amd import hdf
    dt = torch.float32 if mixed else torch.float64
    Xd = to_dev(X, dt)
    f = hdf.Factor(Xd, kernel, l, tol, precision=hdf.HDF_MIXED if mixed else hdf.HDF_FP64)
    return f, Xd


def oracle_for(X, kernel, l, tol, mixed=False):
    """Oracle on exactly the values the device consumed."""
    Xo = np.asarray(X, dtype=np.float32 if mixed else np.float64).astype(np.float64)
    return ohdf.build(Xo, kernel, l, tol), Xo


def ambiguous_ranks(st):
    """True if a rank or degree decision lies within AMBIG of its threshold."""
    for dd in st["deg"]:
        lam = np.abs(dd["lam_all"])
        if np.any(np.abs(lam - st["tau"]) <= AMBIG * st["tau"]):
            return True
    if st["tail_at_p"] is not None:
        thr = st["tol"] * st["nu"] / 2
        if abs(st["tail_at_p"] - thr) <= AMBIG * thr:
            return True
    return False


def oracle_phi(st, kept):
    """H x N harmonics of the kept degrees, canonical order (oracle)."""
    Sh = harmonics.solid_harmonics(st["geo"]["xt"], st["K"], degrees=kept)
    return np.concatenate([Sh[k].T for k in kept], axis=0)


def rel_fro(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def degree_blocks(f):
    """(k, harmonic offset, |H_k|, radial offset, s_k) of the kept degrees."""
    inf = f.info()
    out, h0, q0 = [], 0, 0
    for k, s in enumerate(inf["s_k"]):
        if s == 0:
            continue
        nh = harmonics.count(f.d, k)
        out.append((k, h0, nh, q0, s))
        h0 += nh
        q0 += s
    return out


def torch_contraction(f, V):
    """K~V = sum_k sum_l q_kl o (Phi_k^T (lam_kl (Phi_k^T (q_kl o V)))) in
    binary64 with torch GEMMs on the device factor (no library kernels)."""
    phi, q = f.factor_parts()
    lam = torch.tensor(f.plan()["lam"], dtype=torch.float64, device="cuda")
    Vd = V.double()
    out = torch.zeros_like(Vd)
    for k, h0, nh, q0, s in degree_blocks(f):
        P = phi[h0:h0 + nh].double()                       # nh x N
        for l in range(s):
            ql = q[q0 + l].double()                        # N
            W = P @ (ql[:, None] * Vd)                     # nh x m
            out += ql[:, None] * (P.t().contiguous() @ (lam[q0 + l] * W))
    return out
