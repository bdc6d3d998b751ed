"""SplitMix64 and the ||K||_F estimate nu (oracle, test infrastructure).

SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): state += 0x9E3779B97F4A7C15, then the output is the
state passed through two xor-shift-multiply rounds and a final xor-shift.
All arithmetic is modulo 2^64.

nu^2 is the mean of k(||x_a - x_b||)^2 over M pairs of indices drawn from the
generator, an unbiased estimate of ||K||_F^2 / N^2.  It scales the absolute
error budget eps * ||K||_F (relative Frobenius error, the reading of the
paper's undefined "relative error", Sec. 4.1).
"""
import numpy as np

from .kernels import kappa

MASK = (1 << 64) - 1
NU_SEED = 0x48444600
NU_PAIRS = 65536


class SplitMix64:
    def __init__(self, seed):
        self.state = seed & MASK

    def next(self):
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        return z ^ (z >> 31)


def sample_pairs(N, M=NU_PAIRS, seed=NU_SEED, Nb=None):
    """M index pairs (a_t, b_t), a_t < N, b_t < Nb (default N), two outputs per pair."""
    Nb = N if Nb is None else Nb
    g = SplitMix64(seed)
    a = np.empty(M, dtype=np.int64)
    b = np.empty(M, dtype=np.int64)
    for t in range(M):
        a[t] = (g.next() >> 11) % N
        b[t] = (g.next() >> 11) % Nb
    return a, b


def norm_scale(X, name, l, M=NU_PAIRS, seed=NU_SEED):
    """nu = sqrt(mean_t k(||x_a - x_b||)^2), summed in t order."""
    X = np.asarray(X, dtype=np.float64)
    N, d = X.shape
    a, b = sample_pairs(N, M, seed)
    s = np.zeros(M)
    for j in range(d):
        t = X[a, j] - X[b, j]
        s = s + t * t
    kv = kappa(name, np.sqrt(s), l)
    acc = 0.0
    for t in range(M):
        acc += kv[t] * kv[t]
    return float(np.sqrt(acc / M))


def norm_scale_cross(X, Y, name, l, M=NU_PAIRS, seed=NU_SEED):
    """nu = sqrt(mean_t k(||x_a - y_b||)^2), a < N_x, b < N_y: estimates
    ||K(X, Y)||_F / sqrt(N_x N_y)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    a, b = sample_pairs(X.shape[0], M, seed, Nb=Y.shape[0])
    s = np.zeros(M)
    for j in range(X.shape[1]):
        t = X[a, j] - Y[b, j]
        s = s + t * t
    kv = kappa(name, np.sqrt(s), l)
    acc = 0.0
    for t in range(M):
        acc += kv[t] * kv[t]
    return float(np.sqrt(acc / M))
