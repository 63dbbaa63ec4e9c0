"""CPU reference ("oracle") for randomized strong recursive skeletonization.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 NumPy/SciPy
implementation of the method of Yesypenko & Martinsson, "Randomized Strong
Recursive Skeletonization" (Sec. 3-4, Algorithm 1).  Only the test suite,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the HIP library under
``paper_2311_01451_amd/csrc``; the two meet only through the seeded input
generators in ``paper_2311_01451_amd/inputs.py``.

Modules
  tree       quad/oct-tree, 2:1 balance, neighbours, box order (Sec. 3)
  operators  the synthetic black-box operators as dense / sparse matrices
  rsrs       Algorithm 1 (factor), the inverse and forward factorizations
             (eq. Afact, Ainvfact), refinement and error metrics (eq. error)
  flops      algorithmic flop / byte model of one factorization

Every function names the passage of the paper it follows.  Readings of
passages that are silent or ambiguous are listed in the repository's design
notes and repeated in the docstring of the function that takes them.
"""
