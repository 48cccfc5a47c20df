"""Plain FP64 CPU oracle for the pass-efficient randomized SVD.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code, tables or constants with the
GPU library; the two meet only in the seeded input generators (``synth``),
which hold none of the method's arithmetic.

Everything here is written for a reader holding the paper (Bjarkason 2018,
"Pass-Efficient Randomized Algorithms for Low-Rank Matrix Approximation Using
Any Number of Views"):

* ``philox``   -- the counter-based Gaussian test matrices (the paper's randn,
                  Sect. 2), defined from the Philox4x32-10 generator of
                  Salmon et al. (SC'11) and the Box-Muller transform.
* ``linalg``   -- the primitives of Sect. 2: qr, orth, tsvd (LAPACK via numpy).
* ``rsvd``     -- Alg. 1, Alg. 2 (and its range/co-range helper Alg. 3),
                  Alg. 7 and Alg. 8 (one view, with the l_c rules of
                  Sect. 6.6), the extended one-view sketch of Sect. 6.7,
                  Alg. 9 (generalized block Krylov) and the row-wise
                  accuracy-enhanced block Krylov of Sect. 7.3.
* ``normal``   -- Alg. 4 (Nystrom), Alg. 5 (pinched) and the J / J^T rule for
                  truncated eigendecompositions of J^T J (Sect. 4.2).
* ``stream``   -- one-view sketches of a matrix given as a stream of linear
                  updates (Sect. 6.1) and their post-processing.
* ``srft``     -- the subsampled randomized DCT test matrices of Sect. 6.7.
* ``errors``   -- the relative Frobenius / spectral errors of Sect. 8.2.
* ``formats``  -- exact decoders for BF16 and OCP FP8-e4m3 storage.

Letters.  The paper's target rank is p and its oversampling l, with sketch
width p+l.  This package uses the library's letters: target rank k,
oversampling p, sketch width s = k+p.

Parity status of each function is stated in its docstring ("pinned by" lists
the tests that fix it from outside the oracle).
"""

from . import philox, linalg, srft, rsvd, normal, stream, errors, formats  # noqa: F401
