"""Oracle: a plain, slow FP64 CPU reference of randomized symmetric NMF.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
HIP library never calls it and shares no code, constants or helpers with it.

Source: Hayashi, Aksoy, Ballard, Park, "Randomized Algorithms for Symmetric
Nonnegative Matrix Factorization" (arXiv 2402.08134).  Each function names the
section / equation / algorithm it follows.  Everything is NumPy/SciPy in FP64;
the library primitives used as single steps are matrix products, Householder
QR (``numpy.linalg.qr``), the symmetric eigensolver (``numpy.linalg.eigh``),
``scipy.optimize.nnls`` and a sort.

Pinning status (what fixes each function other than itself) is listed in
``tests/test_oracle_pins.py``; every public function here is pinned.
"""
from . import philox  # noqa: F401
from . import symnmf  # noqa: F401
