"""Plain FP64 CPU oracle for Haar-tSVD (arXiv 2508.10307).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import it: only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the HIP path (no kernels, headers,
helpers, tables or constants): it is written directly from the paper, step by
step in the order of Algorithm 1 (grouping, collaborative filtering,
aggregation), in float64 / exact integers, with NumPy library primitives
(FFT, matmul, eigh, sort) as single steps.

Where the paper is silent or ambiguous the oracle follows a fixed reading;
each reading is stated in the docstring of the function that applies it.

Modules
  haar      Haar matrix, Eq. 8-9.
  grid      reference grid and truncated search windows (Alg. 1 Step 1).
  matching  quantised guide, GCP mode (Eq. 10), exact distances, top-K.
  basis     global circulant basis from all reference patches (Eq. 11-12).
  filtering t-SVD projection + Haar (Eq. 18), hard threshold (Eq. 19),
            inverse (Eq. 20), averaged write-back (Eq. 2).
  pipeline  Algorithm 1 end to end, with overrides for parity tests.
  adjoint   the frozen-index/frozen-mask linear map and its transpose.
  basis_adjoint  the derivative through the learned basis (eigenvector
            perturbation, phase gauge, covariance chain rule).
  video     spatio-temporal grouping across frames and the video pipeline
            on the stacked frames.
  adaptive  A-Haar-tSVD noise-level adjustment (Sec. III.D, Eq. 21-22): the
            circulant eigenvalue rank test, the vote, sub-image denoising.

Parity status (each function is pinned by a test in tests/test_oracle_*.py
against printed values, closed forms, invariants or brute force):
  haar, grid, matching, basis, filtering, pipeline, adjoint, basis_adjoint,
  video, adaptive: pinned.
  End-to-end denoising quality: parity unpinned by the paper (its PSNR tables
  need datasets that are not available); only a sanity band is checked.
"""
