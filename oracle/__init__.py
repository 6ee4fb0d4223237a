"""Plain FP64 CPU oracle for Householder QR of Block Low-Rank (BLR) matrices.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference that the GPU library is checked against.  Only the test suite,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the library (``paper_2208_06194_amd``) never does, and the oracle
never imports the library.  The two share no code: the only common module is
``synth`` (seeded input generators, no arithmetic of the method).

Source: Apriansyah & Yokota, "Parallel QR Factorization of Block Low-Rank
Matrices" (arXiv 2208.06194).  Each function cites the section, equation or
algorithm it follows.  Where the paper is silent or garbled the reading taken
is stated in the function.

Everything is float64 numpy.  Library primitives used as single steps: matrix
products, ``numpy.linalg.qr`` (QR of the stacked bases in Alg. 6) and
``numpy.linalg.svd`` (the truncated SVD in compression and in Alg. 6).
Householder reflector generation and the tile operations are written out.
"""
