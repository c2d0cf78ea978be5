"""FP64 CPU oracle for the kernel-independent FMM (kiFMM) and its M2L forms.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares
no code with the HIP library (``paper_2408_07436_amd``) and never imports it;
the product path never calls it.

What it computes (each function cites the passage it follows):

* ``kernel``   - the 3D Laplace kernel and the direct O(MN) sum (Section 1,
  the N-body sum and the Laplace kernel).
* ``tree``     - uniform octree with locational (Morton) keys, empty-branch
  pruning, near fields and interaction lists (Section 2).
* ``surfaces`` - equivalent / check surfaces with 6(P-1)^2+2 points
  (Section 2.1.1, Appendix A.3).
* ``linalg``   - the backward-stable two-factor pseudo-inverse
  (Section 2.1.1).
* ``fmm``      - the dense, uncompressed kiFMM: P2M, M2M, M2L, L2L, L2P, P2P
  (Sections 2 and 2.2), with the M2L applied densely, through the paper's
  FFT convolution (Appendix A.1) or through the SVD-compressed operators
  (Section 3.1).
* ``fft_m2l``  - reference FFT-M2L of one source/target pair on the 2P-point
  convolution grid (Appendix A.1); self-test only.
* ``blas_m2l`` - K_fat / K_thin SVD compression and directional
  recompression (Section 3.1); it forms the operator the compressed method
  applies as a dense matrix.

Floating point is float64 throughout.  Parity status of each part is listed
in ``tests/test_oracle_*.py``; conventions that the paper leaves open (surface
radii, Morton bit order, accumulation order) are stated in the code and are
"parity unpinned" beyond being shared with the library's header.
"""

from . import kernel, tree, surfaces, linalg, fmm, fft_m2l, blas_m2l  # noqa: F401
