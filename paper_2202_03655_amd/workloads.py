"""Seeded synthetic point clouds shaped like the paper's workloads.

Input generators only (no arithmetic of the method): the tests, the
benchmark and the oracle timing all draw their points and right-hand sides
from here.  numpy Generator(PCG64(seed)), generated in binary64; the
mixed-precision path casts to binary32 and every comparison feeds the oracle
the same cast values.
"""
import numpy as np


def unit_ball(n, d, seed):
    """Uniform in the unit ball: g/||g|| * U^(1/d) (Gaussian kernel workload)."""
    rng = np.random.default_rng(seed)
    g = rng.normal(size=(n, d))
    return g / np.linalg.norm(g, axis=1)[:, None] * rng.random(n)[:, None] ** (1.0 / d)


def normal_cloud(n, d, seed):
    """i.i.d. N(0, I) points."""
    return np.random.default_rng(seed).normal(size=(n, d))


def max_norm_one(X):
    """Centre by the mean and scale so the largest norm is 1 (the paper's
    preparation of its synthetic data, Sec. 4.1)."""
    Y = X - X.mean(axis=0)
    return Y / np.max(np.linalg.norm(Y, axis=1))


def gaussian_mixture(n, d, seed, n_comp=10, mean_std=2.0, comp_std=0.5):
    """Equal-weight mixture: means ~ N(0, mean_std^2 I), cov comp_std^2 I."""
    rng = np.random.default_rng(seed)
    mu = rng.normal(scale=mean_std, size=(n_comp, d))
    z = rng.integers(0, n_comp, size=n)
    return mu[z] + comp_std * rng.normal(size=(n, d))


def uniform_cube(n, d, seed):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n, d))


def shell(n, d, seed, r0=0.9, r1=1.1):
    """Uniform direction, radius uniform in [r0, r1]."""
    rng = np.random.default_rng(seed)
    g = rng.normal(size=(n, d))
    return g / np.linalg.norm(g, axis=1)[:, None] * rng.uniform(r0, r1, size=n)[:, None]


def housing_like(n, seed):
    """Tabular cloud in d = 8 shaped like the California Housing features of Sec. 4.2 (not available
    here): a skewed income, a uniform age, three log-normal counts and a ratio, and two clustered
    location coordinates (six centres); every feature min-max scaled to [0, 1] as the paper does."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-1.0, 1.0, size=(6, 2))
    loc = centres[rng.integers(0, 6, n)] + 0.15 * rng.normal(size=(n, 2))
    inc = rng.lognormal(1.2, 0.45, n)
    age = rng.uniform(1.0, 52.0, n)
    rooms = rng.lognormal(1.6, 0.25, n)
    beds = rooms * rng.uniform(0.15, 0.25, n)
    pop = rng.lognormal(7.0, 0.7, n)
    occ = rng.lognormal(1.0, 0.3, n)
    F = np.column_stack([inc, age, rooms, beds, pop, occ, loc])
    return (F - F.min(axis=0)) / (F.max(axis=0) - F.min(axis=0))


def housing_labels(F, seed):
    """Smooth response of the features plus N(0, 0.05^2) noise."""
    noise = np.random.default_rng(seed).normal(scale=0.05, size=len(F))
    return (np.sin(3.0 * F[:, 0] + 2.0 * F[:, 6]) + F[:, 1] * F[:, 7] - 2.0 * (F[:, 2] - 0.2) ** 2 + noise)


def housing_split(n, seed=11, n_points=20640):
    """Seeded shuffle and the 2/3 - 1/3 train/test split of Sec. 4.2: (X_train, y_train, X_test,
    y_test) from the first n of n_points (n = n_points: the full set)."""
    F_all = housing_like(n_points, seed)
    F, y = F_all[:n], housing_labels(F_all, seed + 1)[:n]
    order = np.random.default_rng(seed + 2).permutation(n)
    ntr = 2 * n // 3
    return F[order[:ntr]], y[order[:ntr]], F[order[ntr:]], y[order[ntr:]]


# KRR consumer (Sec. 4.2): clusters, kernel, lengthscale, block tol, lambda, CG rtol and limit
KRR = dict(n=20640, d=8, clusters=30, kernel="gaussian", l=0.5, tol=1e-4, lam=0.1, rtol=1e-6, max_iter=1024,
           kmeans_iter=100)


def rhs(n, m, seed):
    return np.random.default_rng(seed).normal(size=(n, m))


# name -> (points(n), kernel, lengthscale, tol, m); n defaults to the full size
CONFIGS = {
    # N=2000 in the unit ball, d=3, Gaussian l=1, tol 1e-6 (plain FP64 check)
    "ball3_gauss": dict(n=2000, d=3, gen=lambda n: unit_ball(n, 3, 101), kernel="gaussian",
                        l=1.0, tol=1e-6, m=1),
    # N=1e5 i.i.d. normal, d=3, Matern-3/2 l=0.5, tol 1e-4 (degree far above
    # the limit: the method is not low rank here)
    "normal3_matern32": dict(n=100_000, d=3, gen=lambda n: normal_cloud(n, 3, 102),
                             kernel="matern32", l=0.5, tol=1e-4, m=16),
    # ... the same cloud with lengthscale 10 (feasible variant)
    "normal3_matern32_l10": dict(n=100_000, d=3, gen=lambda n: normal_cloud(n, 3, 102),
                                 kernel="matern32", l=10.0, tol=1e-4, m=16),
    # N=1e6, d=5, 10-component Gaussian mixture scaled to max-norm 1, Cauchy l=1
    "gmm5_cauchy_1e-3": dict(n=1_000_000, d=5, gen=lambda n: max_norm_one(gaussian_mixture(n, 5, 103)),
                             kernel="cauchy", l=1.0, tol=1e-3, m=16),
    "gmm5_cauchy_1e-4": dict(n=1_000_000, d=5, gen=lambda n: max_norm_one(gaussian_mixture(n, 5, 103)),
                             kernel="cauchy", l=1.0, tol=1e-4, m=16),
    # the same mixture z-scored per coordinate (degree above the limit)
    "gmm5_cauchy_zscore": dict(n=1_000_000, d=5,
                               gen=lambda n: (lambda X: (X - X.mean(0)) / X.std(0))(gaussian_mixture(n, 5, 103)),
                               kernel="cauchy", l=1.0, tol=1e-3, m=16),
    # N=2e5 uniform in [-1,1]^4, Gaussian l=0.7, tol 1e-5 (derivatives)
    "cube4_gauss": dict(n=200_000, d=4, gen=lambda n: uniform_cube(n, 4, 104), kernel="gaussian",
                        l=0.7, tol=1e-5, m=1),
    # N=5e5 shell in d=6, Matern-5/2 l=0.3, tol 1e-7 (degree far above the limit)
    "shell6_matern52": dict(n=500_000, d=6, gen=lambda n: shell(n, 6, 105), kernel="matern52",
                            l=0.3, tol=1e-7, m=64),
    # feasible variants of the shell workload
    "shell6_matern52_l8": dict(n=500_000, d=6, gen=lambda n: shell(n, 6, 105), kernel="matern52",
                               l=8.0, tol=1e-7, m=64),
    "shell6_matern52_l4": dict(n=100_000, d=6, gen=lambda n: shell(n, 6, 105), kernel="matern52",
                               l=4.0, tol=1e-7, m=64),
}


def points(name, n=None, dtype=np.float64):
    cfg = CONFIGS[name]
    X = cfg["gen"](cfg["n"] if n is None else n)
    return X.astype(dtype)
