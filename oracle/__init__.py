"""Plain, slow FP64 CPU oracle for the Harmonic Decomposition Factorization (HDF).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding) may import, call or link anything in this package.  It may be
used by ``tests/``, by ``__graft_entry__.smoke()`` and by the ``cpu_baseline``
leg of ``bench.py``, nothing else.

It follows the paper "Linear Time Kernel Matrix Approximation via
Hyperspherical Harmonics" (Ryan & Damle, ICML 2022) step by step:

* kernels.py    -- the isotropic kernels of Sec. 4.1 (Fig. 3 text) and their
                   derivatives (closed forms),
* geometry.py   -- the diameter normalisation of Sec. 3.3 (footnote 1),
* chebyshev.py  -- the even extension and truncated Chebyshev series of
                   Sec. 3.3 (Eq. chebtrunc), the monomial coefficients t_{i,j}
                   (Eq. chebdef) and the degree selection of Sec. 3.5 (Remark 3),
* splitmix.py   -- the SplitMix64 counter-based generator used to sample the
                   pairs that estimate ||K||_F (published by Steele, Lea and
                   Flood, OOPSLA 2014),
* expansion.py  -- the multinomial / Gegenbauer re-expansion of App. A that
                   gives the coefficients T'_{j,m,n} and the per-degree radial
                   core (Eq. preharm, Eq. preeigen, Eq. rdef),
* harmonics.py  -- the real hyperspherical harmonics, index sets H_k and the
                   addition-theorem normalisation Z_k (Eq. additiontheorem,
                   App. B),
* hdf.py        -- Algorithm 1 with the symmetric simplification of Remark 1:
                   Vandermonde-like radial matrices (Eq. vandermonde), QR,
                   truncated eigendecomposition (Eq. svd, Eq. rapprox), factor
                   assembly and the O(Nr) matvec (Sec. 3.6), plus the
                   frozen-structure derivatives,
* cross.py      -- Algorithm 1 in the general case X != Y (QR of both radial
                   matrices, SVD of R_x M_k R_y^T, K(X, Y) ~ U V^T),
* adaptive.py   -- the tighter degree and rank selection of the remark after
                   Eq. bound (sampled Frobenius error, tau raised while the
                   estimate stays within the tolerance),
* dense.py      -- the dense kernel matrix and its truncated eigendecomposition
                   (the optimal-rank reference of Sec. 4.1, Fig. 3).

All floating point is IEEE binary64; the data-free expansion coefficients are
computed in exact rational arithmetic (``fractions.Fraction``) and rounded to
binary64 once.
"""
